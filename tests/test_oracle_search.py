"""Pins of the oracle's brute-force search and ZOOM engine.

Brute force (Introduction; Experiment 2): argmax of Eq. 1 over every entry.
ZOOM (Theory: MRF ZOOM; Methods: Experiment 2 steps 1-5): checked on analytic
objectives whose argmax is known, on the evaluation counts the Theory section
states for the evaluation-saving move rules, and on the special case the
Methods state (df hops at the finest resolution = brute force).
"""
import math

import numpy as np
import pytest

from paper_1506_05393_amd import inputs as I
from tests import bloch_ref


def _tiny():
    seq = I.make_sequence(24, 11)
    grid = I.make_grid([300.0, 700.0, 1200.0, 1900.0, 2600.0], [30.0, 60.0, 120.0, 250.0],
                       np.arange(-12.0, 13.0, 4.0))
    return seq, grid


def test_bruteforce_equals_numpy_reduction(orc):
    """Dictionary from the independent expm integration, CC matrix by NumPy."""
    seq, grid = _tiny()
    D = np.stack([bloch_ref.simulate(seq, *map(float, grid.values(k))) for k in range(grid.size)])
    rng = np.random.default_rng(5)
    truth = rng.integers(0, grid.size, 6)
    V = D[truth] * np.exp(1j * rng.uniform(0, 6.28, 6))[:, None] * 1.7
    V = V + 0.02 * (rng.normal(size=V.shape) + 1j * rng.normal(size=V.shape))
    V = np.concatenate([V, rng.normal(size=(3, 24)) + 1j * rng.normal(size=(3, 24))])
    res = orc.bruteforce(seq, grid, V, top_k=5, threads=3)
    Dn = D / np.linalg.norm(D, axis=1, keepdims=True)
    Vn = V / np.linalg.norm(V, axis=1, keepdims=True)
    S = np.abs(Vn @ Dn.conj().T)
    order = np.argsort(-S, axis=1, kind="stable")
    assert np.array_equal(res["idx"], order[:, 0])
    assert np.max(np.abs(res["cc"] - S[np.arange(len(V)), order[:, 0]])) < 1e-13
    assert np.array_equal(res["topk_idx"], order[:, :5])
    s2 = S[np.arange(len(V)), order[:, 1]]
    assert np.max(np.abs(res["margin"] - (res["cc"] - s2))) < 1e-13
    best = D[order[:, 0]]
    pd = np.sum(V * best.conj(), axis=1) / np.sum(np.abs(best) ** 2, axis=1)
    assert np.max(np.abs(res["pd"] - pd)) < 1e-12


def test_cc_at_listed_entries_equals_numpy(orc):
    """CC at listed entries (Eq. 1) = NumPy |Vn Dn^H| on the expm dictionary,
    read at the listed columns; a negative index gives 0."""
    seq, grid = _tiny()
    D = np.stack([bloch_ref.simulate(seq, *map(float, grid.values(k))) for k in range(grid.size)])
    rng = np.random.default_rng(15)
    V = rng.normal(size=(5, 24)) + 1j * rng.normal(size=(5, 24))
    V[:3] += 3.0 * D[rng.integers(0, grid.size, 3)]
    idx = rng.integers(0, grid.size, (5, 7))
    idx[1, 2] = -1
    got = orc.cc_at(seq, grid, V, idx, threads=2)
    S = np.abs((V / np.linalg.norm(V, axis=1, keepdims=True))
               @ (D / np.linalg.norm(D, axis=1, keepdims=True)).conj().T)
    want = np.take_along_axis(S, np.maximum(idx, 0), axis=1)
    want[1, 2] = 0.0
    assert np.max(np.abs(got - want)) < 1e-13
    with pytest.raises(ValueError):
        orc.cc_at(seq, grid, V, np.full((5, 1), grid.size))


def test_bruteforce_noise_free_on_grid_is_exact(orc):
    """On-grid noise-free fingerprints return the truth with CC = 1 (Experiment 2)."""
    seq, grid = _tiny()
    ks = np.array([0, 17, 33, grid.size - 1])
    D, _ = orc.simulate_grid(seq, grid)
    V = D[ks] * (0.8 * np.exp(0.3j))
    res = orc.bruteforce(seq, grid, V)
    assert np.array_equal(res["idx"], ks)
    assert np.max(np.abs(res["cc"] - 1.0)) < 1e-14
    assert np.max(np.abs(res["pd"] - 0.8 * np.exp(0.3j))) < 1e-13


def test_bruteforce_independent_of_thread_count(orc):
    seq, grid = _tiny()
    rng = np.random.default_rng(2)
    V = rng.normal(size=(4, 24)) + 1j * rng.normal(size=(4, 24))
    a = orc.bruteforce(seq, grid, V, top_k=8, threads=1)
    b = orc.bruteforce(seq, grid, V, top_k=8, threads=4)
    for key in a:
        assert np.array_equal(a[key], b[key])


def test_bruteforce_ties_go_to_lower_index(orc):
    """A zero voxel has CC = 0 against every entry: the lowest index wins."""
    seq, grid = _tiny()
    res = orc.bruteforce(seq, grid, np.zeros((1, 24), complex), top_k=3)
    assert res["idx"][0] == 0
    assert list(res["topk_idx"][0]) == [0, 1, 2]
    assert res["margin"][0] == 0.0


# ---------------------------------------------------------------- ZOOM -----

def _cfg1():
    seq = I.make_sequence(200, 0)
    grid = I.make_grid(I.grid_linspace(100, 2000, 60), I.grid_geomspace(20, 400, 40),
                       I.grid_arange(-40, 40, 4))
    return seq, grid


def test_paper_schedule_index_steps(orc):
    """Physical steps of Experiment 2 converted with max(1, round(r / step))."""
    seq, grid = _cfg1()
    s = orc.schedule_paper(seq, grid)
    d1 = 1900.0 / 59.0
    d2 = 380.0 / 39.0
    r = lambda x, d: max(1, int(math.floor(x / d + 0.5)))
    omega = 1000.0 / seq.tr_ms.min()
    st = s["stages"]
    assert [x["kind"] for x in st] == [0, 1, 2, 4, 4, 1, 3, 3, 3, 3, 3, 3, 3, 3, 4]
    assert st[0]["step0"] == r(60, 4) == 15
    assert (st[1]["step0"], st[1]["window"]) == (r(3, 4), r(75, 4))
    assert abs(st[2]["hop"] - omega / 4.0) < 1e-12
    assert (st[3]["step0"], st[3]["step1"]) == (r(200, d1), r(200, d2))
    assert (st[4]["step0"], st[4]["step1"]) == (r(100, d1), r(100, d2))
    assert st[5]["window"] == r(0.5 * omega, 4)
    assert [x["step0"] for x in st[6:14]] == [r(100, d1), r(100, d2), r(50, d1), r(20, d1),
                                              r(10, d1), r(50, d2), r(20, d2), r(10, d2)]
    assert [x["axis0"] for x in st[6:14]] == [0, 1, 0, 0, 0, 1, 1, 1]
    assert s["starts"] == [[int(np.argmin(np.abs(grid.t1_ms - 1000))), 39, 0, 0]]


def _bowl(t, w=(1.0, 0.7, 1.3, 1.0)):
    return lambda a, b, c, d: -(w[0] * (a - t[0]) ** 2 + w[1] * (b - t[1]) ** 2
                                + w[2] * (c - t[2]) ** 2 + w[3] * (d - t[3]) ** 2)


@pytest.mark.parametrize("pruned", [0, 1])
def test_zoom_finds_bowl_maximum(orc, pruned):
    seq, grid = _cfg1()
    s = orc.schedule_paper(seq, grid)
    s["pruned"] = pruned
    rng = np.random.default_rng(3)
    for _ in range(25):
        t = (int(rng.integers(0, 60)), int(rng.integers(0, 40)), int(rng.integers(0, 21)), 0)
        r = orc.zoom_generic(s, (60, 40, 21, 1), _bowl(t))
        assert r["idx"] == t
        assert r["n_eval"] == len(set(r["calls"]))  # memoised: each entry once
        assert r["n_eval"] < 60 * 40 * 21 // 10


def test_zoom_result_is_local_max_of_final_stencil(orc):
    """Two-mode objective: whatever mode ZOOM lands in, no unit-step neighbour
    in (T1, T2) beats it, and the path value only ever increases."""
    seq, grid = _cfg1()
    s = orc.schedule_paper(seq, grid)
    rng = np.random.default_rng(4)
    for _ in range(10):
        m1 = rng.integers(0, [60, 40, 21])
        m2 = rng.integers(0, [60, 40, 21])

        def f(a, b, c, d, m1=m1, m2=m2):
            g1 = math.exp(-((a - m1[0]) ** 2 + (b - m1[1]) ** 2 + (c - m1[2]) ** 2) / 200.0)
            g2 = 1.2 * math.exp(-((a - m2[0]) ** 2 + (b - m2[1]) ** 2 + (c - m2[2]) ** 2) / 30.0)
            return g1 + g2
        r = orc.zoom_generic(s, (60, 40, 21, 1), f)
        a, b, c, _ = r["idx"]
        for da in (-1, 0, 1):
            for db in (-1, 0, 1):
                if 0 <= a + da < 60 and 0 <= b + db < 40:
                    assert f(a + da, b + db, c, 0) <= r["val"]


def test_zoom_plateau_keeps_centre(orc):
    """Ties keep the current centre (moves need a strictly larger CC)."""
    sched = dict(stages=[dict(kind=orc.ZOOM2, axis0=0, axis1=1, step0=2, step1=2),
                         dict(kind=orc.ZOOM1, axis0=0, step0=1)], starts=[[5, 6, 0, 0]])
    r = orc.zoom_generic(sched, (12, 12, 1, 1), lambda *i: 1.0)
    assert r["idx"] == (5, 6, 0, 0)
    assert r["min_margin"] == 0.0


def test_zoom2_ties_follow_fixed_neighbour_order(orc):
    """Equal best neighbours: the first in the order L, R, D, U, LD, LU, RD, RU."""
    sched = dict(stages=[dict(kind=orc.ZOOM2, axis0=0, axis1=1, step0=1, step1=1)],
                 starts=[[5, 5, 0, 0]])
    # R and U tie above the centre, everything else lower; after one move stop
    def f(a, b, c, d):
        if (a, b) in ((6, 5), (5, 6)):
            return 2.0
        return 1.0 if (a, b) == (5, 5) else 0.0
    r = orc.zoom_generic(sched, (12, 12, 1, 1), f)
    assert r["idx"] == (6, 5, 0, 0)


def _count_first_move(orc, values, pruned=1):
    """Calls made by one pruned 2-D move from centre (5,5) with neighbour values."""
    sched = dict(stages=[dict(kind=orc.ZOOM2, axis0=0, axis1=1, step0=1, step1=1)],
                 starts=[[5, 5, 0, 0]], pruned=pruned)
    names = {(-1, 0): "L", (1, 0): "R", (0, -1): "D", (0, 1): "U", (-1, -1): "LD",
             (-1, 1): "LU", (1, -1): "RD", (1, 1): "RU"}

    def f(a, b, c, d):
        da, db = a - 5, b - 5
        if (da, db) == (0, 0):
            return 1.0
        if abs(da) <= 1 and abs(db) <= 1:
            return values.get(names[(da, db)], 0.0)
        return -1.0  # everything beyond the first stencil is worse: stop after one move
    r = orc.zoom_generic(sched, (12, 12, 1, 1), f)
    # evaluations of the first move: calls[0] is the centre, the move log
    # records how many evaluations had been made when the centre first moved
    end = r["moves"][0][1] if r["moves"] else len(r["calls"])
    first = [names[(c[0] - 5, c[1] - 5)] for c in r["calls"][1:end]]
    dest = r["moves"][0][0] if r["moves"] else (5, 5, 0, 0)
    return first, dest


def test_pruned_2d_evaluation_counts(orc):
    """Theory section: 3 evaluations when L and D both beat C (move to LD); 4
    when none of L, D, R, U does (stop); 5 when R and U both do (move to RU);
    L > C > D: 4 with U > C (move to LU), else 3 (move to L); symmetric for D."""
    ev, idx = _count_first_move(orc, dict(L=2, D=2, LD=3))
    assert ev == ["L", "D", "LD"] and idx[:2] == (4, 4)
    ev, idx = _count_first_move(orc, dict(L=0, D=0, R=0, U=0))
    assert ev == ["L", "D", "R", "U"] and idx[:2] == (5, 5)
    ev, idx = _count_first_move(orc, dict(L=0, D=0, R=2, U=2, RU=3))
    assert ev == ["L", "D", "R", "U", "RU"] and idx[:2] == (6, 6)
    ev, idx = _count_first_move(orc, dict(L=2, D=0, U=2, LU=3))
    assert ev == ["L", "D", "U", "LU"] and idx[:2] == (4, 6)
    ev, idx = _count_first_move(orc, dict(L=2, D=0, U=0))
    assert ev == ["L", "D", "U"] and idx[:2] == (4, 5)
    ev, idx = _count_first_move(orc, dict(L=0, D=2, R=2, RD=3))
    assert ev == ["L", "D", "R", "RD"] and idx[:2] == (6, 4)
    ev, idx = _count_first_move(orc, dict(L=0, D=2, R=0))
    assert ev == ["L", "D", "R"] and idx[:2] == (5, 4)


def test_pruned_corner_not_better_falls_back(orc):
    ev, idx = _count_first_move(orc, dict(L=2, D=3, LD=0.5))
    assert ev == ["L", "D", "LD"] and idx[:2] == (5, 4)


def test_pruned_1d_skips_left_when_right_is_better(orc):
    """Theory section: if R beats C, move without evaluating L."""
    sched = dict(stages=[dict(kind=orc.ZOOM1, axis0=0, step0=3)], starts=[[10, 0, 0, 0]], pruned=1)
    r = orc.zoom_generic(sched, (40, 1, 1, 1), lambda a, b, c, d: -abs(a - 22))
    assert r["idx"][0] == 22 or abs(r["idx"][0] - 22) <= 1
    # the left neighbour of the start is never requested
    assert (7, 0, 0, 0) not in r["calls"]


def test_half_range_fov_first_decision_two_requests(orc):
    """Theory section: with a FOV of half the range started at the centre, the
    first decision requests 2 entries and compares 3 CCs."""
    n = 41
    sched = dict(stages=[dict(kind=orc.ZOOM1, axis0=0, step0=(n - 1) // 4)],
                 starts=[[(n - 1) // 2, 0, 0, 0]])
    r = orc.zoom_generic(sched, (n, 1, 1, 1), lambda a, b, c, d: -abs(a - 37))
    assert r["calls"][:3] == [(20, 0, 0, 0), (10, 0, 0, 0), (30, 0, 0, 0)]


def test_df_hops_at_finest_resolution_equal_bruteforce(orc):
    """Methods: with omega at the minimal resolution the df search is a brute-
    force search; on a df-only grid ZOOM then equals brute force."""
    seq = I.make_sequence(60, 12)
    grid = I.make_grid([900.0], [80.0], I.grid_arange(-40, 40, 1))
    rng = np.random.default_rng(9)
    D, _ = orc.simulate_grid(seq, grid)
    V = D[rng.integers(0, grid.size, 12)] + 0.05 * (rng.normal(size=(12, 60)) + 1j * rng.normal(size=(12, 60)))
    brute = orc.bruteforce(seq, grid, V)
    for start in (0, 40, 80):
        sched = dict(stages=[dict(kind=orc.SCAN_HOPS, axis0=2, hop=1.0)],
                     starts=[[0, 0, start, 0]])
        z = orc.zoom(seq, grid, sched, V)
        assert np.array_equal(z["idx"], brute["idx"])
        assert np.array_equal(z["cc"], brute["cc"])
    sched = dict(stages=[dict(kind=orc.SCAN_STRIDE, axis0=2, step0=1)], starts=[[0, 0, 0, 0]])
    z = orc.zoom(seq, grid, sched, V)
    assert np.array_equal(z["idx"], brute["idx"])
    assert np.all(z["n_sim"] == grid.size)


def test_physics_zoom_noise_free_truths(orc):
    """On-grid noise-free fingerprints (Experiment 2): wherever the paper
    schedule lands on the truth its CC is 1; wherever it lands it is a local
    maximum of the final unit-step 2-D stencil; it visits a small fraction of
    the grid. How often it lands on the truth depends on how well Properties
    I and III hold for the sequence and tissue values: with T2 near TR the df
    stage at the starting T1/T2 can pick a wrong df (Discussion)."""
    seq, grid = _cfg1()
    D, _ = orc.simulate_grid(seq, grid, threads=4)
    for seed, floor in ((100, 0.1), (102, 0.9)):
        ph = I.phantom_quadrants(grid, 8, seed, snr=np.inf)
        V = D[ph.truth_idx]
        z = orc.zoom(seq, grid, orc.schedule_paper(seq, grid), V, threads=4)
        hit = z["idx"] == ph.truth_idx
        assert hit.mean() >= floor
        assert np.all(np.abs(z["cc"][hit] - 1.0) < 1e-12)
        assert np.all(z["cc"][~hit] < 1.0 - 1e-9)
        assert np.all(z["n_sim"] < grid.size / 20)
        for v in range(len(V)):
            a, b, c, _ = grid.unravel(z["idx"][v])
            for da in (-1, 0, 1):
                for db in (-1, 0, 1):
                    if 0 <= a + da < 60 and 0 <= b + db < 40:
                        k = grid.ravel(a + da, b + db, c)
                        assert orc.cc(V[v], D[k]) <= z["cc"][v] + 1e-15


def test_neighbour_prior_restricts_range(orc):
    """Prior ranges (Experiment 3): the search never leaves init +- half width."""
    sched = dict(stages=[dict(kind=orc.ZOOM2, axis0=0, axis1=1, step0=1, step1=1)],
                 starts=[[0, 0, 0, 0]], prior_half=[3, 2, -1, -1])
    r = orc.zoom_generic(sched, (30, 30, 1, 1), _bowl((25, 25, 0, 0)), init=(10, 10, 0, 0))
    assert r["idx"] == (13, 12, 0, 0)
    assert all(7 <= c[0] <= 13 and 8 <= c[1] <= 12 for c in r["calls"])


def _local_schedule(orc, b1=False):
    st = [dict(kind=orc.ZOOM2, axis0=0, axis1=1, step0=1, step1=1),
          dict(kind=orc.ZOOM1, axis0=2, step0=1)]
    if b1:
        st.append(dict(kind=orc.ZOOM1, axis0=3, step0=1))
    return dict(stages=st, outer=list(st), outer_max=8, starts=[[0, 0, 0, 0]])


def test_local_refine_keeps_the_global_maximum(orc):
    """The global CC maximum is a local one: unit-step refinement started at
    the brute-force argmax never moves, and its value is brute force's."""
    seq, grid = _tiny()
    rng = np.random.default_rng(21)
    D, _ = orc.simulate_grid(seq, grid)
    V = D[rng.integers(0, grid.size, 20)] * np.exp(1j * rng.uniform(0, 6.3, (20, 1)))
    V = V + 0.03 * (rng.normal(size=V.shape) + 1j * rng.normal(size=V.shape))
    brute = orc.bruteforce(seq, grid, V)
    init = np.stack(grid.unravel(brute["idx"]), axis=1).astype(np.int32)
    z = orc.zoom(seq, grid, _local_schedule(orc), V, init=init)
    assert np.array_equal(z["idx"], brute["idx"])
    assert np.allclose(z["cc"], brute["cc"], rtol=0, atol=1e-15)


def test_local_refine_climbs_to_a_local_maximum(orc):
    """From an arbitrary start the refinement ends where no unit neighbour
    (the 8 of the (T1, T2) stencil, df +-1) has a higher CC."""
    seq, grid = _tiny()
    rng = np.random.default_rng(22)
    D, _ = orc.simulate_grid(seq, grid)
    V = D[rng.integers(0, grid.size, 12)]
    V = V + 0.05 * (rng.normal(size=V.shape) + 1j * rng.normal(size=V.shape))
    dims = np.array([len(grid.t1_ms), len(grid.t2_ms), len(grid.df_hz)])
    init = np.zeros((12, 4), np.int32)
    init[:, :3] = rng.integers(0, dims, (12, 3))
    z = orc.zoom(seq, grid, _local_schedule(orc), V, init=init)
    for v in range(12):
        c = np.array(grid.unravel(int(z["idx"][v]))[:3])
        best = orc.cc(V[v], D[int(z["idx"][v])])
        assert abs(best - z["cc"][v]) < 1e-12
        for dl in ([1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [1, 1, 0], [1, -1, 0],
                   [-1, 1, 0], [-1, -1, 0], [0, 0, 1], [0, 0, -1]):
            n = c + np.array(dl)
            if np.any(n < 0) or np.any(n >= dims):
                continue
            assert orc.cc(V[v], D[int((n[0] * dims[1] + n[1]) * dims[2] + n[2])]) <= best


def test_nearest_lattice_voxel_by_hand(orc):
    """Two-pass neighbour prior: the nearest lattice voxel (Chebyshev, ties
    to the lower raster index) on a 6 x 5 slice with stride 4, by hand."""
    near = orc.nearest_lattice(6, 5, 2, 4)
    xy = lambda v: (v % 6, (v // 6) % 5)
    expect = {(0, 0): (0, 0), (1, 0): (0, 0), (2, 0): (0, 0), (3, 0): (4, 0), (5, 0): (4, 0),
              (2, 2): (0, 0), (3, 2): (4, 0), (2, 3): (0, 4), (5, 4): (4, 4), (1, 3): (0, 4),
              (4, 2): (4, 0)}
    for (x, y), (px, py) in expect.items():
        assert xy(near[y * 6 + x]) == (px, py), (x, y)
        assert near[30 + y * 6 + x] == 30 + py * 6 + px  # second slice: its own lattice


def test_lattice_prior_pass_structure(orc):
    """Lattice voxels get exactly the plain search; with whole-axis prior
    ranges every other voxel gets the plain search started at its prior
    centre."""
    seq, grid = _tiny()
    rng = np.random.default_rng(23)
    D, _ = orc.simulate_grid(seq, grid)
    V = D[rng.integers(0, grid.size, 30)]
    V = V + 0.05 * (rng.normal(size=V.shape) + 1j * rng.normal(size=V.shape))
    sched = orc.schedule_paper(seq, grid)
    res = orc.zoom_lattice(seq, grid, sched, V, 6, 5, 1, stride=4)
    lat = res["lattice"]
    plain = orc.zoom(seq, grid, sched, V[lat])
    assert np.array_equal(res["idx"][lat], plain["idx"])
    rest = np.flatnonzero(~lat)
    init = np.stack(grid.unravel(res["idx"][res["prior_voxel"][rest]]), axis=1).astype(np.int32)
    again = orc.zoom(seq, grid, sched, V[rest], init=init)
    assert np.array_equal(res["idx"][rest], again["idx"])
    assert np.array_equal(res["n_sim"][rest], again["n_sim"])


def _calls_of_one_scan(orc, stage, n, centre):
    sched = dict(stages=[stage], starts=[[0, 0, centre, 0]])
    r = orc.zoom_generic(sched, (1, 1, n, 1), lambda a, b, c, d: -abs(c - centre))
    return [c[2] for c in r["calls"]]


def test_scan_hops_non_integer_hop_hand_listed(orc):
    """Methods, Experiment 2 step 1(c): the +-k omega hops land on
    c + round(k * hop) with halves rounded away from zero. Hand-worked point
    lists (the centre is evaluated first, then the targets in increasing
    index order): a floor, a truncation or round-half-even would list other
    points."""
    # hop 23.8 about 50 on 101 values: +-23.8 -> +-24, +-47.6 -> +-48, +-71.4 out
    assert _calls_of_one_scan(orc, dict(kind=orc.SCAN_HOPS, axis0=2, hop=23.8), 101, 50) == \
        [50, 2, 26, 74, 98]
    # hop 2.5 about 10 on 21 values: 2.5 -> 3, 5, 7.5 -> 8, 10, 12.5 -> 13 (out)
    assert _calls_of_one_scan(orc, dict(kind=orc.SCAN_HOPS, axis0=2, hop=2.5), 21, 10) == \
        [10, 0, 2, 5, 7, 13, 15, 18, 20]
    # the targets are offsets from the centre, clipped at each end separately
    assert _calls_of_one_scan(orc, dict(kind=orc.SCAN_HOPS, axis0=2, hop=1.5), 9, 2) == \
        [2, 0, 4, 5, 7, 8]
    # hops below one index step are taken as one step (every index in range)
    assert _calls_of_one_scan(orc, dict(kind=orc.SCAN_HOPS, axis0=2, hop=0.4), 5, 1) == \
        [1, 0, 2, 3, 4]


def test_scan_window_truncation_and_ties(orc):
    """Methods, Experiment 2 step 1(b)/3: a window scan visits c + m s for
    0 < |m s| <= w, so a window of 7 at step 3 reaches +-6 and not +-9; the
    centre is kept on ties, and among equal candidates the lowest index
    wins."""
    st = dict(kind=orc.SCAN_WINDOW, axis0=2, step0=3, window=7)
    assert _calls_of_one_scan(orc, st, 40, 20) == [20, 14, 17, 23, 26]
    # clipped at the low end: 2 - 3 and 2 - 6 are outside
    assert _calls_of_one_scan(orc, st, 40, 2) == [2, 5, 8]
    sched = dict(stages=[st], starts=[[0, 0, 20, 0]])
    run = lambda vals: orc.zoom_generic(sched, (1, 1, 40, 1),
                                        lambda a, b, c, d: vals.get(c, 0.0))["idx"][2]
    assert run({20: 1.0, 23: 1.0}) == 20           # a tie with the centre keeps it
    assert run({20: 0.5, 17: 1.0, 26: 1.0}) == 17  # equal candidates: lowest index
    assert run({20: 0.5, 26: 1.0, 14: 0.9}) == 26
    # a window narrower than the step scans nothing but the centre
    assert _calls_of_one_scan(orc, dict(kind=orc.SCAN_WINDOW, axis0=2, step0=3, window=2),
                              40, 20) == [20]


def test_prior_half_widths_hand_worked(orc):
    """Methods, Experiment 3: ranges T1p +- 3000 ms, T2p +- 800 ms,
    dfp +- 150 Hz around the neighbour's result, in index steps of each
    grid, worked by hand:
      slice grid (T1 step 10, T2 step 5, df step 1): 300, 160, 150;
      volume grid (T1 1, T2 1, df 0.5, B1 0.005 with +- 0.3): 3000, 800, 300, 60;
      small grid (T1 1900/59 = 32.20 ms, T2 380/39 = 9.744 ms, df 4 Hz):
        3000/32.20 = 93.2 -> 93, 800/9.744 = 82.1 -> 82, 150/4 = 37.5 -> 38;
      halves round away from zero: 150 / 60 = 2.5 -> 3, 25 / 10 = 2.5 -> 3;
      a width below half a step still opens one step."""
    from paper_1506_05393_amd import workloads
    assert orc.prior_half(workloads.slice64().grid) == [300, 160, 150, -1]
    assert orc.prior_half(workloads.volume(1, 8).grid) == [3000, 800, 300, 60]
    assert orc.prior_half(workloads.small_dgs().grid) == [93, 82, 38, -1]
    g = I.make_grid([100.0, 160.0, 220.0], [10.0, 20.0], [-60.0, 0.0, 60.0])
    assert orc.prior_half(g, [150.0, 25.0, 150.0, 0.3]) == [3, 3, 3, -1]
    assert orc.prior_half(g, [1.0, -1.0, 0.0, 0.3]) == [1, -1, 1, -1]
    g1 = I.make_grid([100.0], [10.0, 20.0], [0.0])
    assert orc.prior_half(g1) == [-1, 80, -1, -1]


def test_decision_margin_bounds_what_a_perturbation_can_change(orc):
    """The pinning rule of the parity tests: a voxel whose smallest decision
    margin along its path exceeds 2 delta takes the same path, entry for
    entry, under any perturbation of its objective by at most delta (each
    decision compares values at least 2 delta apart). Checked with a
    deterministic per-entry perturbation on noisy small-workload voxels;
    with a perturbation far above the margins some paths do change."""
    from paper_1506_05393_amd import workloads
    w = workloads.small_dgs(False)
    g = w.grid
    sched = orc.schedule_paper(w.seq, g)
    voxels = np.arange(0, w.phantom.n_vox, 23)
    V = []
    for v in voxels:
        d = orc.simulate(w.seq, float(w.phantom.t1[v]), float(w.phantom.t2[v]),
                         float(w.phantom.df[v]))
        V.append(d * np.exp(1j * 0.3 * v) + 0.01 * np.exp(1j * np.arange(len(d))))
    changed_big = 0
    for v in V:
        memo = {}

        def f(i1, i2, i3, i4, delta=0.0):
            k = int(g.ravel(i1, i2, i3, i4))
            if k not in memo:
                memo[k] = orc.cc(v, orc.simulate(w.seq, *map(float, g.values(k))))
            h = (k * 0x9E3779B97F4A7C15) & ((1 << 64) - 1)
            return memo[k] + delta * ((h >> 11) / float(1 << 53) * 2.0 - 1.0)

        r0 = orc.zoom_generic(sched, g.shape, f)
        delta = 0.45 * r0["min_margin"]
        r1 = orc.zoom_generic(sched, g.shape, lambda *i: f(*i, delta=delta))
        assert r1["moves"] == r0["moves"] and r1["idx"] == r0["idx"]
        assert r1["n_eval"] == r0["n_eval"] and r1["calls"] == r0["calls"]
        r2 = orc.zoom_generic(sched, g.shape, lambda *i: f(*i, delta=1e-2))
        changed_big += r2["moves"] != r0["moves"]
    assert changed_big > 0


def test_multistart_schedule_by_hand(orc):
    """The multi-start lattice on a 7 x 5 grid: 3 x 2 starts at T1 indices
    0, 3, 6 and T2 indices 0, 4 (ends included); one start per axis sits at
    the middle; the outer round is the df window, the fine df scan and 2-D
    zooms down to the unit step; the stage list is the paper's."""
    seq = I.make_sequence(20, 2)
    grid = I.make_grid(np.linspace(300, 2100, 7), np.linspace(40, 200, 5), np.arange(-8.0, 9.0, 2.0))
    s = orc.schedule_multistart(seq, grid, 3, 2, 5)
    assert [st[:2] for st in s["starts"]] == [[0, 0], [0, 4], [3, 0], [3, 4], [6, 0], [6, 4]]
    assert all(st[2] == 0 and st[3] == 0 for st in s["starts"])
    paper = orc.schedule_paper(seq, grid)
    assert s["stages"] == paper["stages"] and s["outer_max"] == 5
    kinds = [(o["kind"], o["axis0"], o["step0"], o["step1"]) for o in s["outer"]]
    assert kinds[0] == (1, 2, paper["stages"][1]["step0"], 0)
    assert kinds[1] == (1, 2, 1, 0) and kinds[-1] == (4, 0, 1, 1)
    # T1 step 300 ms: 100 and 50 ms round to index steps 0.33 -> 1; T2 step 40 ms
    assert [k[2:] for k in kinds[2:6]] == [(1, 3), (1, 1), (1, 1), (1, 1)]
    one = orc.schedule_multistart(seq, grid, 1, 1, 0)
    assert [st[:2] for st in one["starts"]] == [[3, 2]]
