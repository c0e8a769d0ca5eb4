"""Pins of the oracle's second ZOOM objective: the distance of the
non-normalised fingerprint from the raw entry (M0 = 1) with only a global
phase fitted (Discussion: the paper removed its long-T1 errors at the finest
resolution with the Euclidean distance on non-normalised fingerprints and
entries), score = -min_phi ||v - exp(i phi) d||^2 / ||v||^2.

What fixes it, independently of the closed form the oracle uses:
* a numerical minimisation over the phase (dense scan, then a bounded 1-D
  minimiser) gives the same minimum;
* a fingerprint that is an entry times a unit phase scores exactly 0, and
  twice that fingerprint exactly -1/4 although its CC is still 1;
* letting the magnitude float too turns the distance into 1 - CC^2
  (Cauchy-Schwarz), tying the two objectives together;
* a full-range unit-step scan with the distance objective is the NumPy
  argmin of the phase-fitted distance over a dictionary from the
  independent matrix-exponential integrator;
* the engine simulates each entry once whatever objectives its stages use,
  and each stage decides by its own objective.
"""
import numpy as np
from scipy.optimize import minimize_scalar

from paper_1506_05393_amd import inputs as I
from tests import bloch_ref


def _tiny():
    seq = I.make_sequence(30, 4)
    grid = I.make_grid([300.0, 700.0, 1200.0, 1900.0], [30.0, 60.0, 120.0],
                       np.arange(-12.0, 13.0, 6.0))
    return seq, grid


def _phase_min(v, d):
    """min over phi of ||v - exp(i phi) d||^2, numerically."""
    f = lambda p: float(np.sum(np.abs(v - np.exp(1j * p) * d) ** 2))
    ps = np.linspace(0.0, 2 * np.pi, 721)
    p0 = ps[int(np.argmin([f(p) for p in ps]))]
    r = minimize_scalar(f, bounds=(p0 - 0.01, p0 + 0.01), method="bounded",
                        options={"xatol": 1e-12})
    return min(r.fun, f(p0))


def test_distance_score_is_the_phase_fitted_residual(orc):
    seq, grid = _tiny()
    rng = np.random.default_rng(3)
    ks = rng.integers(0, grid.size, 6)
    V = np.stack([orc.simulate(seq, *map(float, grid.values(int(k)))) for k in ks])
    V = V * rng.uniform(0.5, 1.5, (6, 1)) * np.exp(1j * rng.uniform(0, 6.28, (6, 1)))
    V = V + 0.05 * (rng.normal(size=V.shape) + 1j * rng.normal(size=V.shape))
    idx = rng.integers(0, grid.size, (6, 5))
    cc, sc = orc.objectives_at(seq, grid, V, idx)
    for v in range(6):
        for i in range(5):
            d = orc.simulate(seq, *map(float, grid.values(int(idx[v, i]))))
            ref = -_phase_min(V[v], d) / float(np.sum(np.abs(V[v]) ** 2))
            assert abs(sc[v, i] - ref) < 1e-9 * max(1.0, abs(ref)), (v, i, sc[v, i], ref)
            assert abs(cc[v, i] - orc.cc(V[v], d)) < 1e-14


def test_exact_fingerprint_scores_zero_and_scale_is_seen(orc):
    seq, grid = _tiny()
    k = np.arange(0, grid.size, 7)
    D = np.stack([orc.simulate(seq, *map(float, grid.values(int(x)))) for x in k])
    ph = np.exp(1j * np.linspace(0.1, 6.0, len(k)))[:, None]
    cc1, sc1 = orc.objectives_at(seq, grid, D * ph, k[:, None])
    assert np.abs(sc1).max() < 1e-13 and np.abs(cc1 - 1.0).max() < 1e-13
    cc2, sc2 = orc.objectives_at(seq, grid, 2.0 * D * ph, k[:, None])
    assert np.abs(cc2 - 1.0).max() < 1e-13
    assert np.abs(sc2 + 0.25).max() < 1e-13  # ||2d - d||^2 / ||2d||^2
    # a zero fingerprint: the entry's squared norm, negated
    cc0, sc0 = orc.objectives_at(seq, grid, np.zeros((1, 30)), k[:1, None])
    assert cc0[0, 0] == 0.0
    assert abs(sc0[0, 0] + float(np.sum(np.abs(D[0]) ** 2))) < 1e-12


def test_floating_magnitude_gives_one_minus_cc_squared(orc):
    """max over a scale s of score(s v) = -(1 - CC^2): the distance with the
    magnitude fitted as well ranks entries as CC does."""
    seq, grid = _tiny()
    rng = np.random.default_rng(8)
    k = int(rng.integers(0, grid.size))
    v = orc.simulate(seq, *map(float, grid.values(k))) * 0.8
    v = v + 0.1 * (rng.normal(size=30) + 1j * rng.normal(size=30))
    for e in rng.integers(0, grid.size, 4):
        c = orc.cc(v, orc.simulate(seq, *map(float, grid.values(int(e)))))
        f = lambda s: -orc.objectives_at(seq, grid, s * v, [[int(e)]])[1][0, 0]
        r = minimize_scalar(f, bounds=(0.05, 20.0), method="bounded", options={"xatol": 1e-10})
        assert abs(r.fun - (1.0 - c * c)) < 1e-9, (r.fun, 1 - c * c)


def test_distance_scan_equals_numpy_argmin(orc):
    """Over every entry of a tiny grid, the oracle's score peaks where the
    NumPy argmin of the phase-fitted distance does, over a dictionary from
    the independent matrix-exponential integrator, with the same values
    (times -||v||^2); a search of unit-step scans with the distance
    objective reports the score and CC of the entry it returns."""
    seq, grid = _tiny()
    D = np.stack([bloch_ref.simulate(seq, *map(float, grid.values(k))) for k in range(grid.size)])
    rng = np.random.default_rng(12)
    truth = rng.integers(0, grid.size, 5)
    V = D[truth] * np.exp(1j * rng.uniform(0, 6.28, (5, 1)))
    V = V + 0.03 * (rng.normal(size=V.shape) + 1j * rng.normal(size=V.shape))
    dots = V.conj() @ D.T  # conj(v) . d, |.| = |<v, d>|
    dist = (np.sum(np.abs(V) ** 2, axis=1)[:, None] + np.sum(np.abs(D) ** 2, axis=1)[None, :]
            - 2.0 * np.abs(dots))
    best = np.argmin(dist, axis=1)
    all_idx = np.tile(np.arange(grid.size), (5, 1))
    _, sc = orc.objectives_at(seq, grid, V, all_idx)
    assert np.array_equal(np.argmax(sc, axis=1), best)
    np.testing.assert_allclose(-sc * np.sum(np.abs(V) ** 2, axis=1)[:, None], dist,
                               rtol=0, atol=1e-10)
    # the same through the engine: scanning T1, T2 and df in turn at unit
    # steps, twice, from the corner
    sched = dict(stages=[dict(kind=0, axis0=a, step0=1, objective=1) for a in (0, 1, 2)] * 2,
                 starts=[[0, 0, 0, 0]])
    r = orc.zoom(seq, grid, sched, V)
    for v in range(5):
        assert sc[v, r["idx"][v]] == r["score"][v]
        assert r["cc"][v] == orc.objectives_at(seq, grid, V[v:v + 1], [[r["idx"][v]]])[0][0, 0]


def test_stages_use_their_own_objective_and_entries_are_evaluated_once(orc):
    """Analytic two-valued objective: CC-like values peak at index 2, the
    distance values at index 7. A CC scan goes to 2, a distance hill climb
    from there to 7; every entry is evaluated once although both values of
    the entries scanned first are read again."""
    f = lambda i, *_: (-abs(i - 2.0), -abs(i - 7.0))
    sched = dict(stages=[dict(kind=0, axis0=0, step0=1, objective=0),
                         dict(kind=3, axis0=0, step0=1, objective=1)],
                 starts=[[5, 0, 0, 0]])
    r = orc.zoom_generic(sched, (10, 1, 1, 1), f)
    assert r["idx"][0] == 7
    assert r["vals"] == (-5.0, 0.0)
    assert r["n_eval"] == 10 and len(r["calls"]) == 10
    # the objective switch re-reads the centre's second value from the memo
    sched["stages"][1]["objective"] = 0
    r0 = orc.zoom_generic(sched, (10, 1, 1, 1), f)
    assert r0["idx"][0] == 2 and r0["n_eval"] == 10


def test_distance_separates_long_t1_neighbours_more_than_cc(orc):
    """At T1 = 3000 ms on a 1 ms grid (Experiment 3's finest resolution) a
    noise-free unit-PD fingerprint scores 0 at its truth, and its 1 ms T1
    neighbours fall further below it in the distance score than in CC."""
    seq = I.make_sequence(500, 1)
    grid = I.make_grid(np.arange(2995.0, 3006.0), [100.0, 101.0, 102.0], [0.0, 1.0])
    k = grid.ravel(5, 1, 0)
    v = orc.simulate(seq, *map(float, grid.values(int(k))))[None]
    nb = [grid.ravel(4, 1, 0), grid.ravel(6, 1, 0)]
    cc, sc = orc.objectives_at(seq, grid, v, [[k] + nb])
    assert abs(sc[0, 0]) < 1e-14 and abs(cc[0, 0] - 1.0) < 1e-14
    gap_cc = cc[0, 0] - cc[0, 1:]
    gap_sc = sc[0, 0] - sc[0, 1:]
    assert np.all(gap_cc > 0) and np.all(gap_sc > gap_cc)
