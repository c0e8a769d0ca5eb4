"""Device peak probes (measurement aids of the benchmark): the MFMA-only loops
really run `iters` rounds of four MFMAs per wave, and the write stream writes
exactly the documented pattern. Values are exact (operands 0.5 and 0.25, all
partial sums representable), so the checks are equalities."""
import pytest

from tests.gpu_common import need_gpu, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    need_gpu()
    from paper_1506_05393_amd import api
    return api.Context(0)


@pytest.mark.parametrize("dtype,per_lane,per_mfma", [("f32", 16, 4096), ("bf16", 128, 32768)])
@pytest.mark.parametrize("iters", [1, 7, 1000])
def test_mfma_probe_counts_every_round(ctx, dtype, per_lane, per_mfma, iters):
    from paper_1506_05393_amd import api
    out = torch.full((3 * 256,), -1.0, dtype=torch.float32, device="cuda")
    fl = api.probe_mfma(ctx, dtype, iters, out)
    torch.cuda.synchronize()
    assert torch.equal(out, torch.full_like(out, float(per_lane * iters)))
    # 3 workgroups x 4 waves x 4 MFMAs per round
    assert fl == 3 * 4 * 4 * iters * per_mfma


@pytest.mark.parametrize("nbytes", [16, 4096 * 16 + 48, (1 << 26) + 16])
def test_write_probe_pattern(ctx, nbytes):
    from paper_1506_05393_amd import api
    buf = torch.zeros(nbytes + 64, dtype=torch.uint8, device="cuda")
    api.probe_write(ctx, buf[:nbytes], pattern=0x0BADF00D)
    torch.cuda.synchronize()
    w = buf[:nbytes].view(torch.int32).view(-1, 4).cpu()
    n = w.shape[0]
    i = torch.arange(n, dtype=torch.int64)
    assert torch.all(w[:, 0] == 0x0BADF00D) and torch.all(w[:, 2] == 0x0BADF00D)
    assert torch.all(w[:, 1].to(torch.int64) == i) and torch.all(w[:, 3].to(torch.int64) == i)
    assert torch.all(buf[nbytes:].cpu() == 0)  # nothing past the end


def test_probe_argument_errors(ctx):
    from paper_1506_05393_amd import api
    with pytest.raises(Exception):
        api.probe_mfma(ctx, "f32", 10, torch.empty(100, dtype=torch.float32, device="cuda"))
    with pytest.raises(Exception):
        api.probe_mfma(ctx, "bf16", 0, torch.empty(256, dtype=torch.float32, device="cuda"))
    with pytest.raises(Exception):
        api.probe_write(ctx, torch.empty(24, dtype=torch.uint8, device="cuda"))
