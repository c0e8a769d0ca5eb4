"""The allocation-free FP32 brute force (mrf_match_bruteforce_noalloc, whose
workspace is the library's static device array) against the allocating
entry point (mrf_match_bruteforce, caller workspace), through the C ABI.

Both run the same kernels, so the outputs must be equal bit for bit; the
first call is also held to the oracle bar on its pinned voxels. Two calls in
a row, the second with fewer voxels and readouts (the array keeps the first
call's contents), then the error cases.
"""
import numpy as np
import pytest

from tests.gpu_common import need_gpu, oracle_fingerprints, to_dev, torch

pytestmark = pytest.mark.gpu
KEYS = ("idx", "cc", "margin", "pd_re", "pd_im", "topk_idx", "topk_cc")


@pytest.fixture(scope="module")
def ctx():
    need_gpu()
    from paper_1506_05393_amd import api
    return api.Context(0)


def _outputs(n_vox, top_k):
    from paper_1506_05393_amd import api
    r = api._result_tensors(n_vox, "cuda")
    r["topk_idx"] = torch.empty((n_vox, top_k), dtype=torch.int64, device="cuda")
    r["topk_cc"] = torch.empty((n_vox, top_k), dtype=torch.float32, device="cuda")
    return r


def test_noalloc_equals_allocating_entry_point(ctx, orc):
    from paper_1506_05393_amd import api, workloads
    w = workloads.small_dgs(False)
    V = oracle_fingerprints(orc, w.seq, w.phantom)
    sq = api.Sequence(ctx, w.seq)
    d = api.simulate_dictionary(ctx, sq, w.grid, dtype="f32")
    pre = api.simulate_dictionary(ctx, sq, w.grid, n_tr=150, dtype="f32")
    torch.cuda.synchronize()
    assert ctx._lib.mrf_static_scratch_bytes() == 64 << 20
    calls = [(V, None, 4), (V[:37, :150], pre, 3)]  # second call: fewer voxels, a prefix view
    for i, (Vc, norms, top_k) in enumerate(calls):
        n_tr = Vc.shape[1]
        dv = api.Dictionary(d.dtype, d.n_tr, d.n_entries, d.ld, d.re, d.im,
                            norms.norm if norms is not None else d.norm)
        Vd = to_dev(Vc)
        ref = api.match_bruteforce(ctx, dv, Vd, top_k=top_k, n_tr=n_tr, with_topk=True)
        out = _outputs(len(Vc), top_k)
        torch.cuda.synchronize()
        # torch's cumulative count of allocation requests: the call makes none
        before = torch.cuda.memory_stats()["allocation.all.allocated"]
        got = api.match_bruteforce_noalloc(ctx, dv, Vd, top_k=top_k, n_tr=n_tr, with_topk=True,
                                           out=out)
        torch.cuda.synchronize()
        assert torch.cuda.memory_stats()["allocation.all.allocated"] == before
        for k in KEYS:
            assert torch.equal(got[k], ref[k]), (i, k)
        print(f"call {i}: {len(Vc)} voxels x {n_tr} readouts, top_k {top_k}: bitwise equal")
        if i == 0:
            o = orc.bruteforce(w.seq, w.grid, Vc, top_k=top_k, threads=8)
            pinned = o["margin"] > 1e-5
            idx = got["idx"].cpu().numpy()
            assert pinned.sum() > 0 and np.all(idx[pinned] == o["idx"][pinned])
            assert np.abs(got["cc"].cpu().numpy() - o["cc"]).max() < 1e-5


def test_noalloc_rejects_what_does_not_fit(ctx):
    from paper_1506_05393_amd import _lib, api
    from paper_1506_05393_amd import inputs as I
    seq = I.make_sequence(1000, 3)
    grid = I.make_grid([500.0, 900.0], [50.0, 80.0], [0.0, 4.0])
    sq = api.Sequence(ctx, seq)
    d = api.simulate_dictionary(ctx, sq, grid, dtype="f32")
    need = api.match_workspace_bytes(ctx, d, 8192, 1, None)
    assert need > ctx._lib.mrf_static_scratch_bytes()
    v = torch.zeros((8192, 1000), dtype=torch.complex64, device="cuda")
    with pytest.raises(_lib.MRFError, match="need .* bytes of scratch"):
        api.match_bruteforce_noalloc(ctx, d, v)
    # the slice shape (4096 voxels x 1000 readouts) fits
    assert api.match_workspace_bytes(ctx, d, 4096, 1, None) <= ctx._lib.mrf_static_scratch_bytes()
    b = api.simulate_dictionary(ctx, sq, grid, dtype="bf16")
    with pytest.raises(_lib.MRFError, match="FP32 dictionaries only"):
        api.match_bruteforce_noalloc(ctx, b, v[:4])
    with pytest.raises(_lib.MRFError, match="top_k"):
        api.match_bruteforce_noalloc(ctx, d, v[:4], top_k=0)
    # the array still serves a valid call afterwards
    r = api.match_bruteforce_noalloc(ctx, d, v[:4].contiguous())
    torch.cuda.synchronize()
    assert r["idx"].shape == (4,)
