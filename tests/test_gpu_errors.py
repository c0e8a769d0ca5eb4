"""The boundary's error contract, one case per error the C ABI lists: each
call returns MRF_ERR_INVALID with a message naming the problem and launches
nothing. (An unknown serving ticket is checked on the host-simulated device
in test_serve_cpu.py.)"""
import ctypes as C

import numpy as np
import pytest

from paper_1506_05393_amd import inputs as I
from tests.gpu_common import need_gpu, torch

pytestmark = pytest.mark.gpu
INVALID = 1


@pytest.fixture(scope="module")
def env():
    need_gpu()
    from paper_1506_05393_amd import api
    ctx = api.Context(0)
    seq = I.make_sequence(40, 1)
    grid = I.make_grid([500.0, 900.0, 1300.0], [50.0, 80.0], [0.0, 4.0])
    sq = api.Sequence(ctx, seq)
    d = api.simulate_dictionary(ctx, sq, grid, dtype="f32")
    b = api.simulate_dictionary(ctx, sq, grid, dtype="bf16")
    v = torch.zeros((3, 40), dtype=torch.complex64, device="cuda")
    torch.cuda.synchronize()
    return dict(api=api, ctx=ctx, seq=seq, grid=grid, sq=sq, d=d, b=b, v=v)


def _err(lib):
    return lib.mrf_last_error().decode()


def test_n_tr_beyond_the_sequence(env):
    api, ctx, sq, grid = env["api"], env["ctx"], env["sq"], env["grid"]
    lib = ctx._lib
    g = api.GridArg(grid)
    re = torch.empty((41, 256), dtype=torch.float32, device="cuda")
    im = torch.empty_like(re)
    st = lib.mrf_simulate_dictionary(ctx.handle, sq.handle, g.ptr, 41, 0, grid.size, 0,
                                     re.data_ptr(), im.data_ptr(), 256, None, 0, None)
    assert st == INVALID and "n_tr" in _err(lib)
    with pytest.raises(api.L.MRFError, match="n_tr"):
        api.zoom_search(ctx, sq, grid, torch.zeros((2, 41), dtype=torch.complex64,
                                                   device="cuda"), n_tr=41)


def test_te_not_below_tr(env):
    api, ctx = env["api"], env["ctx"]
    s = env["seq"]
    bad = I.Sequence(s.fa_deg, s.phase_deg, s.tr_ms, s.tr_ms.copy(), 1, 0.0)
    with pytest.raises(api.L.MRFError, match="te"):
        api.Sequence(ctx, bad)


def test_non_increasing_axis(env):
    api, ctx, sq = env["api"], env["ctx"], env["sq"]
    bad = I.Grid(np.array([900.0, 500.0]), np.array([50.0]), np.array([0.0]))
    with pytest.raises(api.L.MRFError, match="strictly increasing"):
        api.simulate_dictionary(ctx, sq, bad)


def test_ld_below_the_entry_count(env):
    api, ctx, sq, grid, d = env["api"], env["ctx"], env["sq"], env["grid"], env["d"]
    lib = ctx._lib
    g = api.GridArg(grid)
    re = torch.empty((40, 256), dtype=torch.float32, device="cuda")
    im = torch.empty_like(re)
    st = lib.mrf_simulate_dictionary(ctx.handle, sq.handle, g.ptr, 40, 0, grid.size, 0,
                                     re.data_ptr(), im.data_ptr(), grid.size - 1, None, 0, None)
    assert st == INVALID and "ld" in _err(lib)
    view = d.view()
    view.ld = d.n_entries - 1
    nb = C.c_size_t()
    assert lib.mrf_match_workspace(ctx.handle, C.byref(view), 3, 1, C.byref(nb)) == INVALID
    assert "ld" in _err(lib)


def test_bf16_without_sequence_and_grid(env):
    api, ctx, b, v = env["api"], env["ctx"], env["b"], env["v"]
    with pytest.raises(api.L.MRFError, match="seq and grid"):
        api.match_bruteforce(ctx, b, v, top_k=8)


def test_top_k_out_of_range(env):
    api, ctx, d, b, v = env["api"], env["ctx"], env["d"], env["b"], env["v"]
    for k in (0, 65):
        with pytest.raises(api.L.MRFError, match="top_k"):
            api.match_bruteforce(ctx, d, v, top_k=k)
    for k in (1, 9):
        with pytest.raises(api.L.MRFError, match="top_k"):
            api.match_bruteforce(ctx, b, v, top_k=k, seq=env["sq"], grid=env["grid"])


def test_workspace_too_small(env):
    api, ctx, d, v, sq, grid = env["api"], env["ctx"], env["d"], env["v"], env["sq"], env["grid"]
    lib = ctx._lib
    buf = torch.empty(16, dtype=torch.uint8, device="cuda")
    r = api._result_tensors(3, "cuda", with_nsim=True)
    st = lib.mrf_match_bruteforce(ctx.handle, C.byref(d.view()), v.data_ptr(), 3, 40, 1, None,
                                  None, api._result_view(r), None, None, buf.data_ptr(), 16,
                                  None)
    assert st == INVALID and "workspace too small" in _err(lib)
    sched = api.schedule_from_dict(api.schedule_paper(ctx, sq, grid))
    g = api.GridArg(grid)
    st = lib.mrf_zoom_search(ctx.handle, sq.handle, g.ptr, C.byref(sched), v.data_ptr(), 3, 40,
                             40, None, api._result_view(r), buf.data_ptr(), 16, None)
    assert st == INVALID and "workspace too small" in _err(lib)


def test_null_required_pointers(env):
    api, ctx, d, v, sq, grid = env["api"], env["ctx"], env["d"], env["v"], env["sq"], env["grid"]
    lib = ctx._lib
    ws = torch.empty(api.match_workspace_bytes(ctx, d, 3, 1), dtype=torch.uint8, device="cuda")
    r = api._result_tensors(3, "cuda")
    view = d.view()
    rv = api._result_view(r)
    # no voxels
    st = lib.mrf_match_bruteforce(ctx.handle, C.byref(view), None, 3, 40, 1, None, None, rv,
                                  None, None, ws.data_ptr(), ws.numel(), None)
    assert st == INVALID and "vox" in _err(lib)
    # no idx output
    rv0 = api._result_view(r)
    rv0.idx = None
    st = lib.mrf_match_bruteforce(ctx.handle, C.byref(view), v.data_ptr(), 3, 40, 1, None, None,
                                  rv0, None, None, ws.data_ptr(), ws.numel(), None)
    assert st == INVALID and "idx" in _err(lib)
    # no context, no sequence, no dictionary view
    st = lib.mrf_match_bruteforce(None, C.byref(view), v.data_ptr(), 3, 40, 1, None, None, rv,
                                  None, None, ws.data_ptr(), ws.numel(), None)
    assert st == INVALID
    g = api.GridArg(grid)
    re = torch.empty((40, 256), dtype=torch.float32, device="cuda")
    st = lib.mrf_simulate_dictionary(ctx.handle, None, g.ptr, 40, 0, grid.size, 0,
                                     re.data_ptr(), re.data_ptr(), 256, None, 0, None)
    assert st == INVALID
    st = lib.mrf_match_bruteforce(ctx.handle, None, v.data_ptr(), 3, 40, 1, None, None, rv,
                                  None, None, ws.data_ptr(), ws.numel(), None)
    assert st == INVALID and "view" in _err(lib)
    # a dictionary view without its planes
    view.im = None
    st = lib.mrf_match_bruteforce(ctx.handle, C.byref(view), v.data_ptr(), 3, 40, 1, None, None,
                                  rv, None, None, ws.data_ptr(), ws.numel(), None)
    assert st == INVALID and "im" in _err(lib)
