"""GPU parity of MRF-ZOOM over a resident dictionary (the paper's MZfulldict
variant: visited entries are read, not simulated) and of the entry-major
dictionary layout it reads.

Layout: K1's entry-major rows hold the same FP32 values as its planar output
(the same recursion; only the stores differ), so they are compared bit for
bit, with odd readout counts (a last unpaired readout), ragged entry ranges,
padded rows, smoothing and unit norms.
Search: the ZOOM bar against the oracle (on voxels whose path margin exceeds
1e-5: same index and number of distinct entries visited, |CC| within 1e-5).
"""
import dataclasses

import numpy as np
import pytest

from paper_1506_05393_amd import inputs as I
from tests.gpu_common import need_gpu, oracle_fingerprints, to_dev, torch
from tests.test_gpu_zoom import _check

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    need_gpu()
    from paper_1506_05393_amd import api
    return api.Context(0)


def _planar(d, count):
    re = d.re[:, :count].double().cpu().numpy()
    im = d.im[:, :count].double().cpu().numpy()
    return (re + 1j * im).T


def _rows(d, count, n_tr):
    r = d.re[:count, :n_tr].double().cpu().numpy()
    return r[..., 0] + 1j * r[..., 1]


@pytest.mark.parametrize("n_tr,smooth", [(77, 0), (200, 0), (77, 5), (1, 0), (2, 3)])
def test_rows_equal_planar_entries(ctx, n_tr, smooth):
    from paper_1506_05393_amd import api
    seq = dataclasses.replace(I.make_sequence(200, 5), smooth=smooth)
    grid = I.make_grid([300.0, 800.0, 1500.0], [25.0, 60.0, 200.0], I.grid_arange(-30, 30, 3),
                       [0.85, 1.0, 1.15])
    sq = api.Sequence(ctx, seq)
    k0, cnt = 37, grid.size - 37 - 11
    p = api.simulate_dictionary(ctx, sq, grid, n_tr=n_tr, entry_begin=k0, entry_count=cnt)
    ld = n_tr + (n_tr % 2) + 4  # even, padded
    r = api.alloc_dictionary(n_tr, cnt, "f32rows", ld=ld)
    sentinel = torch.full_like(r.re, 7.0)
    r.re.copy_(sentinel)
    api.simulate_dictionary(ctx, sq, grid, n_tr=n_tr, entry_begin=k0, entry_count=cnt, out=r)
    torch.cuda.synchronize()
    assert np.array_equal(_rows(r, cnt, n_tr), _planar(p, cnt))
    assert torch.equal(r.norm, p.norm)
    # the padding is never written
    assert bool(torch.all(r.re[:cnt, n_tr:] == 7.0))
    u = api.alloc_dictionary(n_tr, cnt, "f32rows", ld=ld)
    api.simulate_dictionary(ctx, sq, grid, n_tr=n_tr, entry_begin=k0, entry_count=cnt, out=u,
                            unit_norm=True)
    pu = api.simulate_dictionary(ctx, sq, grid, n_tr=n_tr, entry_begin=k0, entry_count=cnt,
                                 unit_norm=True)
    torch.cuda.synchronize()
    assert np.array_equal(_rows(u, cnt, n_tr), _planar(pu, cnt))


def _small(on_grid=True):
    from paper_1506_05393_amd import workloads
    return workloads.small_dgs(on_grid)


@pytest.mark.parametrize("variant", ["paper", "pruned"])
def test_zoom_dict_small_workload(ctx, orc, variant):
    from paper_1506_05393_amd import api
    w = _small()
    V = oracle_fingerprints(orc, w.seq, w.phantom)
    sched = orc.schedule_paper(w.seq, w.grid)
    if variant == "pruned":
        sched["pruned"] = 1
    ref = orc.zoom(w.seq, w.grid, sched, V, threads=8)
    sq = api.Sequence(ctx, w.seq)
    d = api.simulate_dictionary(ctx, sq, w.grid, dtype="f32rows")
    res = api.zoom_search_dict(ctx, d, w.grid, to_dev(V), sched)
    torch.cuda.synchronize()
    _check(res, ref, f"zoom dict {variant}", min_pinned_frac=0.25, orc=orc, seq=w.seq,
           grid=w.grid, V=V)
    # the simulating engine on the same voxels: the same search up to rounding
    sim = api.zoom_search(ctx, sq, w.grid, to_dev(V), sched=sched)
    torch.cuda.synchronize()
    a, b = res["idx"].cpu().numpy(), sim["idx"].cpu().numpy()
    print(f"dict vs simulate index agreement {np.mean(a == b):.4f}")
    assert np.mean(a == b) >= 0.95
    same = a == b
    assert np.abs(res["cc"].cpu().numpy()[same] - sim["cc"].cpu().numpy()[same]).max() < 2e-6


def test_zoom_dict_prior_odd_readouts_and_prefix(ctx, orc):
    """An odd readout count (the last readout pairs with row padding), a
    prefix of a longer resident dictionary, a prior (Experiment 3)."""
    from paper_1506_05393_amd import api
    w = _small()
    n_tr = 151
    seq = w.seq.prefix(n_tr)
    V = oracle_fingerprints(orc, seq, w.phantom)
    sched = orc.schedule_paper(seq, w.grid)
    sched["prior_half"] = [10, 8, 5, -1]
    tr = np.stack(w.grid.unravel(w.phantom.truth_idx), axis=1).astype(np.int32)
    rng = np.random.default_rng(1)
    init = np.clip(tr + rng.integers(-3, 4, tr.shape), 0, [59, 39, 20, 0]).astype(np.int32)
    init[:, 3] = 0
    ref = orc.zoom(seq, w.grid, sched, V, init=init, threads=8)
    sq = api.Sequence(ctx, w.seq)
    d = api.simulate_dictionary(ctx, sq, w.grid, n_tr=n_tr, dtype="f32rows")
    res = api.zoom_search_dict(ctx, d, w.grid, to_dev(V), sched, init=to_dev(init))
    torch.cuda.synchronize()
    _check(res, ref, "zoom dict odd N + prior", min_pinned_frac=0.25, orc=orc, seq=seq,
           grid=w.grid, V=V)
    # a longer resident dictionary searched over its first n_tr readouts
    d2 = api.simulate_dictionary(ctx, sq, w.grid, dtype="f32rows")
    res2 = api.zoom_search_dict(ctx, d2, w.grid, to_dev(V), sched, n_tr=n_tr,
                                init=to_dev(init))
    torch.cuda.synchronize()
    assert torch.equal(res2["idx"], res["idx"])
    # proton density <v, d> / ||d||^2 of the returned entry, against the oracle's entry
    pd = (res["pd_re"] + 1j * res["pd_im"]).cpu().numpy()
    idx = res["idx"].cpu().numpy()
    for v in range(0, len(V), 37):
        t1, t2, df, b1 = w.grid.values(int(idx[v]))
        dv = orc.simulate(seq, float(t1), float(t2), float(df), float(b1))
        want = np.vdot(dv, V[v]) / np.vdot(dv, dv).real
        assert abs(pd[v] - want) < 1e-4 * abs(want) + 1e-6


def test_zoom_dict_rejects_other_layouts(ctx, orc):
    from paper_1506_05393_amd import api
    w = _small()
    sq = api.Sequence(ctx, w.seq)
    V = to_dev(oracle_fingerprints(orc, w.seq, w.phantom, voxels=[0, 1]))
    sched = orc.schedule_paper(w.seq, w.grid)
    planar = api.simulate_dictionary(ctx, sq, w.grid, dtype="f32")
    with pytest.raises(Exception):  # the planar layout
        api.zoom_search_dict(ctx, planar, w.grid, V, sched)
    part = api.simulate_dictionary(ctx, sq, w.grid, dtype="f32rows", entry_begin=8)
    with pytest.raises(Exception):  # not the whole grid
        api.zoom_search_dict(ctx, part, w.grid, V, sched)
    short = api.simulate_dictionary(ctx, sq, w.grid, n_tr=100, dtype="f32rows")
    with pytest.raises(Exception):  # fewer readouts than searched
        api.zoom_search_dict(ctx, short, w.grid, V, sched, n_tr=200)
    with pytest.raises(Exception):  # rows layout is not a GEMM operand
        api.match_bruteforce(ctx, short, V[:, :100].contiguous())
