"""GPU parity of temporal smoothing (Methods, Experiment 4; Results, Fig. 7B)
against the oracle.

Fingerprints: mrf_smooth_signals against the oracle's smoothing, FP32 vs FP64
(a 3- or 5-term weighted sum between two complex rotations: a few FP32
ulps), with and without a sequence's RF phases (the demodulated frame).
Dictionary side: every path that simulates entries of a smoothing sequence
(K1 FP32 and BF16, CC map, BF16 re-scoring, ZOOM) against the oracle with the
dictionary-parity bars:
unit-entry L2 error below 5e-6, |CC| within 1e-5, the oracle's index where
its margin exceeds 1e-5. The oracle smooths its own copy of the fingerprints.
"""
import dataclasses

import numpy as np
import pytest

from paper_1506_05393_amd import inputs as I
from tests.gpu_common import need_gpu, oracle_fingerprints, to_dev, torch

pytestmark = pytest.mark.gpu
UNIT_L2_TOL = 5e-6
CC_TOL = 1e-5
MARGIN = 1e-5


@pytest.fixture(scope="module")
def ctx():
    need_gpu()
    from paper_1506_05393_amd import api
    return api.Context(0)


def _entries(d, count):
    if d.dtype == "f32":
        re = d.re[:, :count].double().cpu().numpy()
        im = d.im[:, :count].double().cpu().numpy()
        return (re + 1j * im).T
    raw = d.re[:, :count].contiguous().view(torch.bfloat16).float().double().cpu().numpy()
    z = raw[..., 0] + 1j * raw[..., 1]
    return z.transpose(1, 0, 2).reshape(count, -1)


def _unit(x):
    n = np.linalg.norm(x, axis=-1, keepdims=True)
    return x / np.where(n > 0, n, 1)


def _small(taps):
    from paper_1506_05393_amd import workloads
    w = workloads.small_dgs(False)
    return dataclasses.replace(w, seq=dataclasses.replace(w.seq, smooth=taps))


def _phase_seq(n, seed):
    """A sequence whose RF phases are multiples of 90 degrees on even readouts
    and arbitrary on odd ones (both demodulation paths)."""
    rng = np.random.default_rng(seed)
    s = I.make_sequence(n, seed)
    ph = rng.choice([0.0, 90.0, 180.0, 270.0, -90.0], n)
    ph[1::2] = rng.uniform(-180.0, 180.0, ph[1::2].shape)
    return dataclasses.replace(s, phase_deg=ph)


@pytest.mark.parametrize("taps", [3, 5])
@pytest.mark.parametrize("n_tr", [1, 2, 3, 4, 5, 63, 64, 65, 130, 1000])
@pytest.mark.parametrize("framed", [False, True])
def test_smooth_signals_matches_oracle(ctx, orc, taps, n_tr, framed):
    from paper_1506_05393_amd import api
    rng = np.random.default_rng(n_tr * 10 + taps)
    x = (rng.standard_normal((7, n_tr)) + 1j * rng.standard_normal((7, n_tr))).astype(np.complex64)
    seq = _phase_seq(1000, 3) if framed else None
    sq = api.Sequence(ctx, seq) if framed else None
    ref = orc.smooth(x, taps, seq)
    tol = 1e-6 * np.abs(x).max()
    out = api.smooth_signals(ctx, to_dev(x), taps, seq=sq).cpu().numpy()
    assert np.abs(out - ref).max() < tol
    # in place, on rows of a wider buffer (row stride n_tr + 3)
    wide = to_dev(np.concatenate([x, np.full((7, 3), 9 + 9j, np.complex64)], axis=1))
    view = wide[:, :n_tr]
    api.smooth_signals(ctx, view, taps, out=view, seq=sq)
    w = wide.cpu().numpy()
    assert np.array_equal(w[:, :n_tr], out)
    assert np.all(w[:, n_tr:] == 9 + 9j)


def test_smooth_signals_copy_and_errors(ctx):
    from paper_1506_05393_amd import api
    x = to_dev((np.arange(40) * (1 + 2j)).astype(np.complex64).reshape(4, 10))
    for taps in (0, 1):
        assert torch.equal(api.smooth_signals(ctx, x, taps), x)
    with pytest.raises(Exception):
        api.smooth_signals(ctx, x, 4)
    with pytest.raises(Exception):  # rows that overlap without being the same rows
        api.smooth_signals(ctx, x[:, :9], 3, out=x.view(-1)[1:37].view(4, 9))
    with pytest.raises(Exception):  # longer than the sequence
        api.smooth_signals(ctx, x, 3, seq=api.Sequence(ctx, I.make_sequence(8, 1)))


def test_sequence_rejects_other_lengths(ctx):
    from paper_1506_05393_amd import api
    seq = dataclasses.replace(I.make_sequence(20, 1), smooth=2)
    with pytest.raises(Exception):
        api.Sequence(ctx, seq)


@pytest.mark.parametrize("taps", [3, 5])
def test_smoothed_dictionary_f32_bf16(ctx, orc, taps):
    from paper_1506_05393_amd import api
    w = _small(taps)
    sq = api.Sequence(ctx, w.seq)
    ref, nref = orc.simulate_grid(w.seq, w.grid, threads=8)
    d = api.simulate_dictionary(ctx, sq, w.grid, dtype="f32")
    torch.cuda.synchronize()
    gpu = _entries(d, w.grid.size)
    err = np.linalg.norm(_unit(gpu) - _unit(ref), axis=1)
    print(f"taps {taps}: max unit-entry L2 error {err.max():.3e}")
    assert err.max() < UNIT_L2_TOL
    assert np.max(np.abs(d.norm.cpu().numpy() / nref - 1)) < 1e-6
    b = api.simulate_dictionary(ctx, sq, w.grid, dtype="bf16")
    torch.cuda.synchronize()
    gb = _entries(b, w.grid.size)
    assert np.all(np.abs(gb.real - ref.real) <= np.abs(ref.real) * 2.0 ** -8 + 1e-6)
    assert np.all(np.abs(gb.imag - ref.imag) <= np.abs(ref.imag) * 2.0 ** -8 + 1e-6)
    u = api.simulate_dictionary(ctx, sq, w.grid, dtype="f32", unit_norm=True)
    torch.cuda.synchronize()
    assert np.linalg.norm(_entries(u, w.grid.size) - _unit(ref), axis=1).max() < UNIT_L2_TOL


@pytest.mark.parametrize("n_tr", [1, 2, 3, 5, 53])
@pytest.mark.parametrize("phases", ["alternating", "general"])
def test_smoothed_dictionary_ragged(ctx, orc, n_tr, phases):
    """Short sequences (both ends of the window cut), an entry range off the
    block size, row padding and a B1 axis (per-lane pulses); RF phases 0/180
    or arbitrary (general pulses, rounded demodulation)."""
    from paper_1506_05393_amd import api
    base = I.make_sequence(77, 5) if phases == "alternating" else _phase_seq(77, 5)
    seq = dataclasses.replace(base, smooth=5)
    grid = I.make_grid([300.0, 800.0, 1500.0], [25.0, 60.0, 200.0], I.grid_arange(-30, 30, 3),
                       [0.85, 1.0, 1.15])
    sq = api.Sequence(ctx, seq)
    k0, cnt = 37, grid.size - 37 - 11
    d = api.alloc_dictionary(n_tr, cnt, "f32", ld=cnt + 29)
    api.simulate_dictionary(ctx, sq, grid, n_tr=n_tr, entry_begin=k0, entry_count=cnt, out=d)
    torch.cuda.synchronize()
    gpu = _entries(d, cnt)
    ref, nref = orc.simulate_grid(seq, grid, k0=k0, count=cnt, n_tr=n_tr)
    assert np.linalg.norm(_unit(gpu) - _unit(ref), axis=1).max() < UNIT_L2_TOL


def test_smoothed_signals_equal_smoothed_entries(ctx):
    """On-grid raw signals equal the raw entries bit for bit; smoothing both
    with the same weights and order of operations keeps them equal."""
    from paper_1506_05393_amd import api
    w = _small(3)
    sq = api.Sequence(ctx, w.seq)
    d = api.simulate_dictionary(ctx, sq, w.grid, dtype="f32")
    ks = np.array([0, 5, 777, 4321, w.grid.size - 1])
    params = np.stack([np.array(w.grid.values(int(k)), np.float64) for k in ks])
    raw = api.simulate_signals(ctx, sq, to_dev(params))
    sm = api.smooth_signals(ctx, raw, 3, seq=sq).cpu().numpy()
    torch.cuda.synchronize()
    ent = _entries(d, w.grid.size)[ks]
    assert np.array_equal(sm.astype(np.complex128), ent)


def test_smoothed_cc_map(ctx, orc):
    from paper_1506_05393_amd import api
    w = _small(3)
    V = orc.smooth(oracle_fingerprints(orc, w.seq, w.phantom, voxels=[0, 77, 200]), 3, w.seq)
    sq = api.Sequence(ctx, w.seq)
    Vg = api.smooth_signals(ctx, to_dev(oracle_fingerprints(orc, w.seq, w.phantom,
                                                            voxels=[0, 77, 200])), 3, seq=sq)
    k0, cnt = 1000, 20000
    ref = orc.cc_map(w.seq, w.grid, V, k0=k0, count=cnt, threads=8)
    got = api.cc_map(ctx, sq, w.grid, Vg, entry_begin=k0, entry_count=cnt).cpu().numpy()
    err = float(np.abs(got - ref).max())
    print(f"smoothed CC map max |dCC| {err:.2e}")
    assert err < CC_TOL


def _match_check(res, ref, label):
    idx = res["idx"].cpu().numpy()
    cc = res["cc"].cpu().numpy().astype(np.float64)
    pinned = ref["margin"] > MARGIN
    agree = idx == ref["idx"]
    print(f"{label}: pinned {pinned.sum()}/{len(idx)}, agreement all {agree.mean():.4f}, "
          f"max |dCC| {np.abs(cc - ref['cc']).max():.2e}")
    assert bool(np.all(agree[pinned])), np.flatnonzero(pinned & ~agree)[:10]
    assert float(np.abs(cc - ref["cc"]).max()) < CC_TOL


@pytest.mark.parametrize("taps", [3, 5])
def test_smoothed_bruteforce_f32_and_bf16(ctx, orc, taps):
    """Both operands smoothed (Fig. 7B): K1 smooths the entries, the
    fingerprints go through mrf_smooth_signals; BF16 candidates are
    re-simulated with the same smoothing before re-scoring."""
    from paper_1506_05393_amd import api
    w = _small(taps)
    V = oracle_fingerprints(orc, w.seq, w.phantom)
    Vs = orc.smooth(V, taps, w.seq)
    ref = orc.bruteforce(w.seq, w.grid, Vs, top_k=8, threads=8)
    sq = api.Sequence(ctx, w.seq)
    Vg = api.smooth_signals(ctx, to_dev(V), taps, seq=sq)
    d = api.simulate_dictionary(ctx, sq, w.grid, dtype="f32")
    res = api.match_bruteforce(ctx, d, Vg, top_k=4)
    torch.cuda.synchronize()
    _match_check(res, ref, f"smoothed f32 taps {taps}")
    b = api.simulate_dictionary(ctx, sq, w.grid, dtype="bf16")
    rb = api.match_bruteforce(ctx, b, Vg, top_k=8, seq=sq, grid=w.grid, with_topk=True)
    torch.cuda.synchronize()
    tk = rb["topk_idx"].cpu().numpy()
    recall = np.array([ref["idx"][v] in tk[v] for v in range(len(V))])
    assert recall.mean() >= 0.99
    sub = {k: v[recall] for k, v in rb.items() if isinstance(v, torch.Tensor) and v.dim() == 1}
    _match_check(sub, {k: v[recall] for k, v in ref.items()}, f"smoothed bf16 taps {taps}")


@pytest.mark.parametrize("taps", [3, 5])
def test_smoothed_zoom(ctx, orc, taps):
    from paper_1506_05393_amd import api
    w = _small(taps)
    V = oracle_fingerprints(orc, w.seq, w.phantom)
    Vs = orc.smooth(V, taps, w.seq)
    sched = orc.schedule_paper(w.seq, w.grid)
    ref = orc.zoom(w.seq, w.grid, sched, Vs, threads=8)
    sq = api.Sequence(ctx, w.seq)
    Vg = api.smooth_signals(ctx, to_dev(V), taps, seq=sq)
    res = api.zoom_search(ctx, sq, w.grid, Vg, sched=sched)
    torch.cuda.synchronize()
    idx = res["idx"].cpu().numpy()
    cc = res["cc"].cpu().numpy().astype(np.float64)
    ns = res["n_sim"].cpu().numpy()
    pinned = ref["min_margin"] > MARGIN
    agree = idx == ref["idx"]
    print(f"smoothed zoom taps {taps}: pinned {pinned.sum()}/{len(idx)}, agreement all "
          f"{agree.mean():.4f}")
    assert pinned.mean() >= 0.25
    assert bool(np.all(agree[pinned])), np.flatnonzero(pinned & ~agree)[:10]
    assert bool(np.all(ns[pinned] == ref["n_sim"][pinned]))
    assert float(np.abs(cc - ref["cc"])[agree].max()) < CC_TOL
    # wherever the paths differ, the GPU's CC is the CC of the smoothed entry it returns
    for v in np.flatnonzero(~agree)[:16]:
        t1, t2, df, b1 = w.grid.values(int(idx[v]))
        dv = orc.smooth(orc.simulate(w.seq, float(t1), float(t2), float(df), float(b1)), taps,
                        w.seq)
        assert abs(orc.cc(Vs[v], dv) - cc[v]) < CC_TOL


def test_serving_rejects_smoothing(ctx):
    from paper_1506_05393_amd import api
    w = _small(3)
    sq = api.Sequence(ctx, w.seq)
    srv = api.Server(ctx, 1 << 30, n_streams=1)
    try:
        with pytest.raises(Exception):
            srv.register(sq, w.grid, "f32", lengths=(200,))
    finally:
        srv.close()
