"""Empty inputs through the C ABI on the GPU: zero entries, zero voxels and zero
signals are valid calls that launch nothing and leave empty outputs, and the
inputs around them are untouched; an empty dictionary has no entry to match
and is rejected with an error, not searched."""
import pytest

from paper_1506_05393_amd import inputs as I
from tests.gpu_common import need_gpu, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    need_gpu()
    from paper_1506_05393_amd import api
    ctx = api.Context(0)
    seq = I.make_sequence(40, 3)
    grid = I.make_grid([400.0, 900.0, 1600.0], [40.0, 90.0], I.grid_arange(-8, 8, 4))
    return api, ctx, api.Sequence(ctx, seq), grid


def _empty(res):
    return all(t.numel() == 0 for t in res.values() if isinstance(t, torch.Tensor))


@pytest.mark.parametrize("dtype", ["f32", "bf16", "f32rows"])
def test_zero_entries(env, dtype):
    api, ctx, sq, grid = env
    d = api.simulate_dictionary(ctx, sq, grid, dtype=dtype, entry_begin=5, entry_count=0)
    torch.cuda.synchronize()
    assert d.norm.numel() == 0
    # an empty dictionary cannot be matched against
    if dtype != "f32rows":
        v = torch.ones((3, 40), dtype=torch.complex64, device="cuda")
        kw = dict(top_k=8, seq=sq, grid=grid) if dtype == "bf16" else {}
        from paper_1506_05393_amd import _lib
        with pytest.raises(_lib.MRFError, match="n_entries"):
            api.match_bruteforce(ctx, d, v, **kw)


def test_zero_voxels(env):
    api, ctx, sq, grid = env
    V = torch.randn((5, 40), dtype=torch.complex64, device="cuda")
    keep = V.clone()
    d32 = api.simulate_dictionary(ctx, sq, grid)
    d16 = api.simulate_dictionary(ctx, sq, grid, dtype="bf16")
    rows = api.simulate_dictionary(ctx, sq, grid, dtype="f32rows")
    res = [api.match_bruteforce(ctx, d32, V[:0]),
           api.match_bruteforce(ctx, d16, V[:0], top_k=8, seq=sq, grid=grid),
           api.zoom_search(ctx, sq, grid, V[:0]),
           api.zoom_search_dict(ctx, rows, grid, V[:0], api.schedule_paper(ctx, sq, grid))]
    sm = api.smooth_signals(ctx, V[:0], 5, seq=sq)
    torch.cuda.synchronize()
    assert all(_empty(r) for r in res)
    assert sm.shape == (0, 40)
    assert torch.equal(V, keep)


def test_zero_readouts_smoothing(env):
    api, ctx, sq, grid = env
    x = torch.randn((4, 40), dtype=torch.complex64, device="cuda")
    y = api.smooth_signals(ctx, x[:, :0], 3)
    torch.cuda.synchronize()
    assert y.shape == (4, 0)
