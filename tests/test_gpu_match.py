"""GPU parity of brute-force matching (K2 + K3 MFMA GEMM + K4) against the oracle.

Bar: on voxels whose oracle top-2 CC margin exceeds 1e-5 the GPU returns the
oracle's argmax index, and |CC| agrees within 1e-5 on every voxel.
"""
import json
import os

import numpy as np
import pytest

from paper_1506_05393_amd import inputs as I
from tests.gpu_common import (check_cc_at_index, need_gpu, oracle_fingerprints, to_dev, torch,
                              unit_stencil)

pytestmark = pytest.mark.gpu
CC_TOL = 1e-5
MARGIN = 1e-5


@pytest.fixture(scope="module")
def ctx():
    need_gpu()
    from paper_1506_05393_amd import api
    return api.Context(0)


def _check(res, ref, label):
    idx = res["idx"].cpu().numpy()
    cc = res["cc"].cpu().numpy().astype(np.float64)
    pinned = ref["margin"] > MARGIN
    agree = idx == ref["idx"]
    ap = f"{agree[pinned].mean():.4f}" if pinned.any() else "n/a"
    print(f"{label}: pinned {pinned.sum()}/{len(idx)}, agreement pinned "
          f"{ap} all {agree.mean():.4f}, max |dCC| "
          f"{np.abs(cc - ref['cc']).max():.2e}")
    assert bool(np.all(agree[pinned])), np.flatnonzero(pinned & ~agree)[:10]
    dcc = float(np.abs(cc - ref["cc"]).max())
    assert dcc < CC_TOL, dcc
    # where the indices differ the two entries are within the margin rule
    gap = ref["cc"][~agree] - cc[~agree]
    assert bool(np.all(gap <= MARGIN + CC_TOL)), float(gap.max())
    return agree


@pytest.mark.parametrize("on_grid", [True, False])
def test_bruteforce_f32_small_workload(ctx, orc, on_grid):
    from paper_1506_05393_amd import api, workloads
    w = workloads.small_dgs(on_grid)
    V = oracle_fingerprints(orc, w.seq, w.phantom)
    ref = orc.bruteforce(w.seq, w.grid, V, top_k=4, threads=8)
    sq = api.Sequence(ctx, w.seq)
    d = api.simulate_dictionary(ctx, sq, w.grid, dtype="f32")
    res = api.match_bruteforce(ctx, d, to_dev(V), top_k=4, with_topk=True)
    torch.cuda.synchronize()
    _check(res, ref, f"small on_grid={on_grid}")
    mg = res["margin"].cpu().numpy()
    mg_err = float(np.abs(mg - ref["margin"]).max())
    assert mg_err < 2 * CC_TOL, mg_err
    pd = (res["pd_re"] + 1j * res["pd_im"]).cpu().numpy()
    same = res["idx"].cpu().numpy() == ref["idx"]
    pd_err = float(np.abs(pd - ref["pd"])[same].max())
    assert pd_err < 1e-4 * float(np.abs(ref["pd"]).max()), pd_err
    tk = res["topk_idx"].cpu().numpy()
    assert np.all(tk[:, 0] == res["idx"].cpu().numpy())
    tkc = res["topk_cc"].cpu().numpy()
    assert bool(np.all(np.diff(tkc, axis=1) <= 0))
    tk_err = float(np.abs(tkc - ref["topk_cc"]).max())
    assert tk_err < CC_TOL, tk_err


def test_bruteforce_f32_long_candidate_lists(ctx, orc):
    """top_k up to 64 (a GEMM instance with 64-entry lists, merged one wave
    per voxel): the list's CCs rank by rank and the oracle's CC of every
    listed entry within 1e-5, the argmax bar, and its first 16 entries equal
    bit for bit to the 16-entry instance's list."""
    from paper_1506_05393_amd import api, workloads
    w = workloads.small_dgs(False)
    V = oracle_fingerprints(orc, w.seq, w.phantom)[:96]
    sq = api.Sequence(ctx, w.seq)
    d = api.simulate_dictionary(ctx, sq, w.grid, dtype="f32")
    r64 = api.match_bruteforce(ctx, d, to_dev(V), top_k=64, with_topk=True)
    r16 = api.match_bruteforce(ctx, d, to_dev(V), top_k=16, with_topk=True)
    torch.cuda.synchronize()
    ref = orc.bruteforce(w.seq, w.grid, V, top_k=64, threads=8)
    _check(r64, ref, "fp32 top_k 64")
    tki, tkc = r64["topk_idx"].cpu().numpy(), r64["topk_cc"].cpu().numpy().astype(np.float64)
    assert float(np.abs(tkc - ref["topk_cc"]).max()) < CC_TOL
    at = orc.cc_at(w.seq, w.grid, V, tki)
    assert float(np.abs(at - tkc).max()) < CC_TOL
    assert bool(np.all(np.diff(tkc, axis=1) <= 0))
    assert torch.equal(r64["topk_idx"][:, :16], r16["topk_idx"])
    assert torch.equal(r64["topk_cc"][:, :16], r16["topk_cc"])
    for k in ("idx", "cc", "margin", "pd_re", "pd_im"):
        assert torch.equal(r64[k], r16[k]), k


def test_bruteforce_ragged_shapes(ctx, orc):
    """Voxel count, entry count and n_tr all off the tile sizes; zero voxel."""
    from paper_1506_05393_amd import api
    seq = I.make_sequence(57, 21)
    grid = I.make_grid(I.grid_linspace(200, 2500, 7), I.grid_geomspace(15, 600, 5),
                       I.grid_arange(-36, 36, 6))
    ph = I.phantom_quadrants(grid, 6, 7, snr=15.0, on_grid=False)
    V = oracle_fingerprints(orc, seq, ph)
    V = np.concatenate([V[:36], np.zeros((1, 57), np.complex64)])
    ref = orc.bruteforce(seq, grid, V, top_k=5)
    sq = api.Sequence(ctx, seq)
    d = api.simulate_dictionary(ctx, sq, grid, dtype="f32")
    res = api.match_bruteforce(ctx, d, to_dev(V), top_k=5, with_topk=True)
    torch.cuda.synchronize()
    agree = _check(res, ref, "ragged")
    # the zero voxel scores 0 everywhere: lowest index, CC 0
    assert res["idx"][-1].item() == 0 and res["cc"][-1].item() == 0.0


def test_bruteforce_prefix_view(ctx, orc):
    """A view of the first n_tr readouts of a longer dictionary, with the
    norms of that prefix."""
    from paper_1506_05393_amd import api, workloads
    w = workloads.small_dgs(False)
    n_tr = 120
    V = oracle_fingerprints(orc, w.seq, w.phantom, n_tr=n_tr)
    ref = orc.bruteforce(w.seq, w.grid, V, n_tr=n_tr, threads=8)
    sq = api.Sequence(ctx, w.seq)
    d = api.simulate_dictionary(ctx, sq, w.grid, dtype="f32")
    pre = api.simulate_dictionary(ctx, sq, w.grid, n_tr=n_tr, dtype="f32")
    d.norm = pre.norm  # prefix norms
    res = api.match_bruteforce(ctx, d, to_dev(V), n_tr=n_tr)
    torch.cuda.synchronize()
    _check(res, ref, "prefix")


def test_bruteforce_noise_free_on_grid_exact(ctx, orc):
    from paper_1506_05393_amd import api, workloads
    w = workloads.small_dgs(True)
    V = oracle_fingerprints(orc, w.seq, w.phantom, noise=False)
    sq = api.Sequence(ctx, w.seq)
    d = api.simulate_dictionary(ctx, sq, w.grid, dtype="f32")
    res = api.match_bruteforce(ctx, d, to_dev(V))
    ref = orc.bruteforce(w.seq, w.grid, V, threads=8)
    pinned = ref["margin"] > MARGIN
    assert np.all(res["idx"].cpu().numpy()[pinned] == w.phantom.truth_idx[pinned])
    assert np.abs(res["cc"].cpu().numpy() - 1.0).max() < CC_TOL


def test_invalid_match_arguments(ctx):
    from paper_1506_05393_amd import api, _lib
    seq = I.make_sequence(40, 1)
    grid = I.make_grid([500.0, 900.0], [50.0], [0.0, 4.0])
    sq = api.Sequence(ctx, seq)
    d = api.simulate_dictionary(ctx, sq, grid)
    v = torch.zeros((3, 40), dtype=torch.complex64, device="cuda")
    with pytest.raises(_lib.MRFError, match="top_k"):
        api.match_bruteforce(ctx, d, v, top_k=0)
    with pytest.raises(_lib.MRFError, match="top_k"):
        api.match_bruteforce(ctx, d, v, top_k=65)
    with pytest.raises(_lib.MRFError, match="ld_vox"):
        api.match_bruteforce(ctx, d, torch.zeros((3, 30), dtype=torch.complex64, device="cuda"))
    ws = api.Workspace(ctx.device)
    ws.buf = torch.empty(16, dtype=torch.uint8, device="cuda")
    import ctypes as C
    view = d.view()
    r = api._result_tensors(3, ctx.device)
    st = ctx._lib.mrf_match_bruteforce(ctx.handle, C.byref(view), v.data_ptr(), 3, 40, 1, None,
                                       None, api._result_view(r), None, None, ws.buf.data_ptr(),
                                       16, None)
    assert st == 1 and b"workspace too small" in ctx._lib.mrf_last_error()


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "slice64_bruteforce_oracle.json")


def _slice64_inputs(orc):
    """The slice workload, all 4096 fingerprints, the 96 subset fingerprints
    of the stored oracle results and those results."""
    from paper_1506_05393_amd import workloads
    from tests import slice64_subsets as S
    w = workloads.slice64()
    with open(GOLDEN) as f:
        G = json.load(f)
    Vsub, truth = S.fingerprints(orc, w)
    assert S.digest(Vsub) == G["inputs_sha256"], "stored oracle results are for other inputs"
    assert [int(x) for x in S.noisy_voxels(w.phantom.n_vox)] == G["noisy_voxels"]
    V = oracle_fingerprints(orc, w.seq, w.phantom)
    nz = np.array(G["noisy_voxels"])
    assert np.array_equal(V[nz], Vsub[:len(nz)])
    ref = {k: np.array(G[k]) for k in ("idx", "cc", "margin", "topk_idx", "topk_cc")}
    return w, V, Vsub, np.array(truth), nz, ref


def _full_size_checks(orc, w, V, Vsub, truth, nz, ref, full, sub, label):
    """full: GPU results on all 4096 voxels; sub: on the 32 on-grid
    fingerprints. Index bar on pinned subset voxels, CC bar on all of them,
    validity of every voxel's result under the oracle."""
    n_noisy = len(nz)
    res = {k: np.concatenate([full[k].cpu().numpy()[nz], sub[k].cpu().numpy()])
           for k in ("idx", "cc")}
    _check({k: torch.from_numpy(v) for k, v in res.items()}, ref, f"{label} 96-voxel subsets")
    pinned = ref["margin"] > MARGIN
    print(f"{label}: pinned noisy {pinned[:n_noisy].sum()}/{n_noisy}, on-grid "
          f"{pinned[n_noisy:n_noisy + 16].sum()}/16, short-relaxation {pinned[n_noisy + 16:].sum()}/16")
    assert pinned.sum() > 0
    # noise-free on-grid fingerprints: the truth wherever the margin rule pins it, CC 1
    ong = slice(n_noisy, len(ref["idx"]))
    assert np.all(res["idx"][ong][pinned[ong]] == truth[pinned[ong]])
    assert np.abs(res["cc"][ong] - 1.0).max() < CC_TOL
    # every voxel of the slice: the CC reported is the oracle's CC of the entry
    # returned, and no entry near the truth beats it by more than the tolerance
    idx = full["idx"].cpu().numpy()
    cc = full["cc"].cpu().numpy().astype(np.float64)
    check_cc_at_index(orc, w.seq, w.grid, V, idx, cc, CC_TOL, f"{label} all 4096 voxels")
    ph, g = w.phantom, w.grid
    near = g.ravel(*[np.array([int(np.argmin(np.abs(ax - val))) for val in vals])
                     for ax, vals in ((g.t1_ms, ph.t1), (g.t2_ms, ph.t2), (g.df_hz, ph.df))])
    moves = [[(0, a), (1, b), (2, c)] for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)]
    around = orc.cc_at(w.seq, g, V, unit_stencil(g, near, moves))
    short = around.max(axis=1) - cc
    print(f"{label}: best oracle CC among the 27 entries around the truth minus the GPU CC: "
          f"max {short.max():.2e}")
    assert float(short.max()) <= CC_TOL


def test_full_size_bruteforce_subsets(ctx, orc):
    """64x64 slice, N = 1000, 12,636,729 entries (FP32, resident), all 4096
    voxels in the benchmark's launch shape; the stored oracle brute force of
    a seeded 64-voxel subset and of 32 noise-free on-grid fingerprints."""
    from paper_1506_05393_amd import api
    w, V, Vsub, truth, nz, ref = _slice64_inputs(orc)
    sq = api.Sequence(ctx, w.seq)
    d = api.simulate_dictionary(ctx, sq, w.grid, dtype="f32")
    full = api.match_bruteforce(ctx, d, to_dev(V), top_k=2)
    sub = api.match_bruteforce(ctx, d, to_dev(Vsub[len(nz):]), top_k=2)
    torch.cuda.synchronize()
    del d
    torch.cuda.empty_cache()
    _full_size_checks(orc, w, V, Vsub, truth, nz, ref, full, sub, "fp32 slice")


# ------------------------------------------------------------ BF16 + re-score

def _bf16_dict(api, ctx, sq, grid, n_tr=None):
    return api.simulate_dictionary(ctx, sq, grid, n_tr=n_tr, dtype="bf16")


@pytest.mark.parametrize("on_grid", [True, False])
def test_bruteforce_bf16_rescored_small_workload(ctx, orc, on_grid):
    """BF16 GEMM with FP32 accumulation, top-8 re-simulated and re-scored in
    FP32: same bar as FP32 wherever the oracle argmax is among the 8."""
    from paper_1506_05393_amd import api, workloads
    w = workloads.small_dgs(on_grid)
    V = oracle_fingerprints(orc, w.seq, w.phantom)
    ref = orc.bruteforce(w.seq, w.grid, V, top_k=8, threads=8)
    sq = api.Sequence(ctx, w.seq)
    d = _bf16_dict(api, ctx, sq, w.grid)
    res = api.match_bruteforce(ctx, d, to_dev(V), top_k=8, seq=sq, grid=w.grid, with_topk=True)
    torch.cuda.synchronize()
    tk = res["topk_idx"].cpu().numpy()
    recall = np.array([ref["idx"][v] in tk[v] for v in range(len(V))])
    print(f"bf16 top-8 recall of the oracle argmax: {recall.mean():.4f} (reported)")
    # every voxel is held to the margin rule, whether or not its argmax was kept
    _check(res, ref, f"bf16+rescore on_grid={on_grid}")
    pd = (res["pd_re"] + 1j * res["pd_im"]).cpu().numpy()
    same = res["idx"].cpu().numpy() == ref["idx"]
    pd_err = float(np.abs(pd - ref["pd"])[same].max())
    assert pd_err < 1e-4 * float(np.abs(ref["pd"]).max()), pd_err


def test_bruteforce_bf16_ragged(ctx, orc):
    from paper_1506_05393_amd import api
    seq = I.make_sequence(60, 23)
    grid = I.make_grid(I.grid_linspace(200, 2500, 9), I.grid_geomspace(15, 600, 7),
                       I.grid_arange(-36, 36, 6))
    ph = I.phantom_quadrants(grid, 7, 9, snr=25.0, on_grid=False)
    V = oracle_fingerprints(orc, seq, ph)
    ref = orc.bruteforce(seq, grid, V, top_k=4)
    sq = api.Sequence(ctx, seq)
    d = _bf16_dict(api, ctx, sq, grid)
    res = api.match_bruteforce(ctx, d, to_dev(V), top_k=4, seq=sq, grid=grid, with_topk=True)
    torch.cuda.synchronize()
    tk = res["topk_idx"].cpu().numpy()
    recall = np.array([ref["idx"][v] in tk[v] for v in range(len(V))])
    print(f"bf16 ragged: top-4 recall {recall.mean():.4f} (reported)")
    _check(res, ref, "bf16 ragged")


@pytest.mark.parametrize("dtype", ["bf16", "f32"])
def test_bruteforce_tiling_invariance(ctx, orc, dtype):
    """1100 voxels (9 row tiles of the BF16 GEMM, a ragged second group of row
    tiles on each XCD; 18 of the FP32 one) give, voxel by voxel, the same
    top-k lists bit for bit as the same voxels matched 128 at a time (one or
    two row tiles, other entry chunks); sampled voxels meet the oracle bar."""
    from paper_1506_05393_amd import api, workloads
    w = workloads.small_dgs(False)
    V0 = oracle_fingerprints(orc, w.seq, w.phantom)
    rng = np.random.default_rng(11)
    reps = -(-1100 // len(V0))
    V = np.concatenate([V0 * np.exp(1j * rng.uniform(0, 2 * np.pi, (len(V0), 1)))
                        for _ in range(reps)])[:1100].astype(np.complex64)
    sq = api.Sequence(ctx, w.seq)
    d = (_bf16_dict(api, ctx, sq, w.grid) if dtype == "bf16"
         else api.simulate_dictionary(ctx, sq, w.grid))
    kw = dict(top_k=8, seq=sq, grid=w.grid, with_topk=True)
    Vd = to_dev(V)
    full = api.match_bruteforce(ctx, d, Vd, **kw)
    parts = [api.match_bruteforce(ctx, d, Vd[i:i + 128].contiguous(), **kw)
             for i in range(0, len(V), 128)]
    torch.cuda.synchronize()
    for key in ("idx", "cc", "topk_idx", "topk_cc"):
        assert torch.equal(full[key], torch.cat([p[key] for p in parts])), key
    sample = np.sort(rng.choice(len(V), 24, replace=False))
    ref = orc.bruteforce(w.seq, w.grid, V[sample], top_k=8, threads=8)
    tk = full["topk_idx"].cpu().numpy()[sample]
    recall = np.array([ref["idx"][i] in tk[i] for i in range(len(sample))])
    print(f"{dtype} 1100 voxels: top-8 recall of the sample {recall.mean():.3f} (reported)")
    sub = {k: v[sample] for k, v in full.items() if isinstance(v, torch.Tensor) and v.dim() == 1}
    _check(sub, ref, f"{dtype} 1100 voxels")


def test_bf16_requires_sequence_and_grid(ctx):
    from paper_1506_05393_amd import api, _lib
    seq = I.make_sequence(40, 1)
    grid = I.make_grid([500.0, 900.0], [50.0], [0.0, 4.0])
    sq = api.Sequence(ctx, seq)
    d = _bf16_dict(api, ctx, sq, grid)
    v = torch.zeros((3, 40), dtype=torch.complex64, device="cuda")
    with pytest.raises(_lib.MRFError, match="seq and grid"):
        api.match_bruteforce(ctx, d, v, top_k=8)
    with pytest.raises(_lib.MRFError, match="top_k"):
        api.match_bruteforce(ctx, d, v, top_k=1, seq=sq, grid=grid)


def test_full_size_bruteforce_bf16_subsets(ctx, orc):
    """64x64 slice, N = 1000, BF16 dictionary (50.5 GB resident) + top-8 FP32
    re-scoring, all 4096 voxels; the same oracle subsets and checks as FP32."""
    from paper_1506_05393_amd import api
    w, V, Vsub, truth, nz, ref = _slice64_inputs(orc)
    sq = api.Sequence(ctx, w.seq)
    d = _bf16_dict(api, ctx, sq, w.grid)
    kw = dict(top_k=8, seq=sq, grid=w.grid, with_topk=True)
    full = api.match_bruteforce(ctx, d, to_dev(V), **kw)
    sub = api.match_bruteforce(ctx, d, to_dev(Vsub[len(nz):]), **kw)
    torch.cuda.synchronize()
    del d
    torch.cuda.empty_cache()
    tk = np.concatenate([full["topk_idx"].cpu().numpy()[nz], sub["topk_idx"].cpu().numpy()])
    recall = np.array([ref["idx"][i] in tk[i] for i in range(len(tk))])
    print(f"bf16 slice: top-8 recall of the oracle argmax {recall.mean():.3f} (reported)")
    _full_size_checks(orc, w, V, Vsub, truth, nz, ref, full, sub, "bf16 slice")
