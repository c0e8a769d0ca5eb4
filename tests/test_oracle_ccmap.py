"""Pins of the oracle's CC map (Methods and Results, Experiment 1: the CC of
Eq. 1 between a fingerprint and every dictionary entry, written out in full).
"""
import numpy as np

from paper_1506_05393_amd import inputs as I
from tests import bloch_ref


def _tiny():
    seq = I.make_sequence(24, 11)
    grid = I.make_grid([300.0, 700.0, 1200.0, 1900.0, 2600.0], [30.0, 60.0, 120.0, 250.0],
                       np.arange(-12.0, 13.0, 4.0))
    return seq, grid


def test_cc_map_equals_numpy_on_independent_dictionary(orc):
    """Dictionary from the expm integration (tests/bloch_ref), |Vn Dn^H| by NumPy."""
    seq, grid = _tiny()
    D = np.stack([bloch_ref.simulate(seq, *map(float, grid.values(k))) for k in range(grid.size)])
    rng = np.random.default_rng(8)
    V = D[rng.integers(0, grid.size, 3)] * 2.3 * np.exp(0.7j)
    V = V + 0.05 * (rng.normal(size=V.shape) + 1j * rng.normal(size=V.shape))
    V = np.concatenate([V, rng.normal(size=(2, 24)) + 1j * rng.normal(size=(2, 24))])
    m = orc.cc_map(seq, grid, V, threads=3)
    Dn = D / np.linalg.norm(D, axis=1, keepdims=True)
    Vn = V / np.linalg.norm(V, axis=1, keepdims=True)
    assert m.shape == (len(V), grid.size)
    assert np.max(np.abs(m - np.abs(Vn @ Dn.conj().T))) < 1e-13


def test_cc_map_of_entries_is_a_symmetric_gram_matrix(orc):
    """CC(d_a, d_b) = CC(d_b, d_a) and CC(d_a, d_a) = 1: catches an operand
    normalised on one side only or a transposed product."""
    seq, grid = _tiny()
    D, _ = orc.simulate_grid(seq, grid)
    ks = np.array([0, 5, 41, 77, grid.size - 1])
    m = orc.cc_map(seq, grid, D[ks])
    G = m[:, ks]
    assert np.max(np.abs(G - G.T)) < 1e-14
    assert np.max(np.abs(np.diag(G) - 1.0)) < 1e-14
    assert np.all(m <= 1.0 + 1e-14)


def test_cc_map_ranges_and_scale_invariance(orc):
    seq, grid = _tiny()
    D, _ = orc.simulate_grid(seq, grid)
    v = D[[33]] + 0.1
    full = orc.cc_map(seq, grid, v)
    part = orc.cc_map(seq, grid, v, k0=17, count=40)
    assert np.array_equal(part, full[:, 17:57])
    scaled = orc.cc_map(seq, grid, v * (0.01 * np.exp(2.1j)))
    assert np.max(np.abs(scaled - full)) < 1e-14
    zero = orc.cc_map(seq, grid, np.zeros((1, 24), complex))
    assert np.all(zero == 0.0)


def test_cc_map_df_period_constant_tr(orc):
    """Property II in its exact case: constant TR, TE = TR/2 give
    s(df + 1000/TR) = -s(df), so the map repeats along df with that period."""
    n, tr = 80, 12.5
    seq = I.Sequence(10 + 50 * np.abs(np.sin(np.arange(n) / 20.0)),
                     np.where(np.arange(n) % 2 == 0, 0.0, 180.0), np.full(n, tr),
                     np.full(n, tr / 2), 1, 0.0)
    step = 1000.0 / tr / 10  # ten df steps per period
    grid = I.make_grid([600.0, 1400.0], [80.0, 300.0], -40.0 + step * np.arange(30))
    v = bloch_ref.simulate(seq, 1000.0, 150.0, 3.0)[None]
    m = orc.cc_map(seq, grid, v).reshape(2, 2, 30)
    assert np.max(np.abs(m[..., 10:] - m[..., :20])) < 1e-10
