"""Pins of the oracle's temporal smoothing (Methods, Experiment 4; Results,
Fig. 7B): a moving Gaussian of 3 or 5 points along the readouts, applied to
the fingerprints and to the dictionary.

The weights are the binomial ones, (1, 2, 1) / 4 and (1, 4, 6, 4, 1) / 16,
truncated and renormalised at the first and last readouts, applied to the
signal demodulated by each readout's RF phase and modulated back. Checked
against NumPy's convolution, against closed forms (constants and ramps pass,
the alternating signal is removed, 5 points = 3 points twice, a constant in
the demodulated frame passes under any phases), and, for the dictionary side,
against an independent expm dictionary smoothed by NumPy.
"""
import dataclasses

import numpy as np
import pytest

from paper_1506_05393_amd import inputs as I
from tests import bloch_ref

W = {3: np.array([1.0, 2.0, 1.0]), 5: np.array([1.0, 4.0, 6.0, 4.0, 1.0])}


def _np_smooth(x, taps, phase_deg=None):
    """Smoothing along the last axis by np.convolve; edge weights renormalised;
    with phases: M conv(M^H x), M = diag(exp(i phase))."""
    x = np.atleast_2d(np.asarray(x, np.complex128))
    n = x.shape[-1]
    m = np.ones(n) if phase_deg is None else np.exp(1j * np.deg2rad(phase_deg[:n]))
    den = np.convolve(np.ones(n), W[taps], "same")
    return np.stack([m * np.convolve(r * m.conj(), W[taps], "same") / den for r in x])


def _rand(shape, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal(shape) + 1j * r.standard_normal(shape)


@pytest.mark.parametrize("taps", [3, 5])
def test_smooth_equals_numpy_convolution(orc, taps):
    x = _rand((4, 37), taps)
    assert np.max(np.abs(orc.smooth(x, taps) - _np_smooth(x, taps))) < 1e-15


@pytest.mark.parametrize("taps", [3, 5])
def test_smooth_closed_forms(orc, taps):
    """Constants pass everywhere; a ramp passes away from the ends (the
    weights are symmetric); the alternating signal is removed away from the
    ends (the weights sum to 0 with alternating signs)."""
    n, h = 40, taps // 2
    c = np.full(n, 0.3 - 0.7j)
    assert np.max(np.abs(orc.smooth(c, taps) - c)) < 1e-15
    ramp = (2.0 + 1j) * np.arange(n) - 5.0
    assert np.max(np.abs(orc.smooth(ramp, taps)[h:n - h] - ramp[h:n - h])) < 1e-12
    alt = (-1.0) ** np.arange(n) * (1.5 - 0.5j)
    assert np.max(np.abs(orc.smooth(alt, taps)[h:n - h])) < 1e-15


@pytest.mark.parametrize("taps", [3, 5])
def test_smooth_in_the_demodulated_frame(orc, taps):
    """Against M conv(M^H x); a signal constant after demodulation passes
    unchanged whatever the phases (with phases 0/180 it alternates in sign,
    which the plain smoothing would remove); zero phases = plain smoothing."""
    rng = np.random.default_rng(30 + taps)
    ph = rng.choice([0.0, 90.0, 180.0], 41) + rng.uniform(-20, 20, 41)
    x = _rand((3, 41), 31)
    assert np.max(np.abs(orc.smooth(x, taps, ph) - _np_smooth(x, taps, ph))) < 1e-14
    alt = np.tile([0.0, 180.0], 21)[:41]
    c = (0.4 - 1.1j) * np.exp(1j * np.deg2rad(alt))
    assert np.max(np.abs(orc.smooth(c, taps, alt) - c)) < 1e-15
    assert np.max(np.abs(orc.smooth(c, taps)[2:-2])) < 1e-15
    assert np.array_equal(orc.smooth(x, taps, np.zeros(41)), orc.smooth(x, taps))


def test_smooth_five_is_three_twice_in_the_interior(orc):
    """(1, 4, 6, 4, 1) / 16 is (1, 2, 1) / 4 convolved with itself."""
    x = _rand(50, 9)
    a = orc.smooth(x, 5)
    b = orc.smooth(orc.smooth(x, 3), 3)
    assert np.max(np.abs(a[2:-2] - b[2:-2])) < 1e-14
    assert np.max(np.abs(a[:2] - b[:2])) > 1e-3  # the truncations differ at the ends


def test_smooth_commutes_with_reversal_and_edges(orc):
    x = _rand(23, 4)
    for taps in (3, 5):
        assert np.max(np.abs(orc.smooth(x[::-1], taps) - orc.smooth(x, taps)[::-1])) < 1e-15
    # first readout, 3 points: (2 x0 + x1) / 3
    y = orc.smooth(x, 3)
    assert abs(y[0] - (2 * x[0] + x[1]) / 3) < 1e-15
    # second readout, 5 points: (4 x0 + 6 x1 + 4 x2 + x3) / 15
    y = orc.smooth(x, 5)
    assert abs(y[1] - (4 * x[0] + 6 * x[1] + 4 * x[2] + x[3]) / 15) < 1e-15
    # taps 0 and 1 leave the signal alone; other lengths are rejected
    assert np.array_equal(orc.smooth(x, 0), x) and np.array_equal(orc.smooth(x, 1), x)
    with pytest.raises(ValueError):
        orc.smooth(x, 4)


def _tiny(smooth):
    seq = dataclasses.replace(I.make_sequence(24, 11), smooth=smooth)
    grid = I.make_grid([300.0, 700.0, 1200.0, 1900.0, 2600.0], [30.0, 60.0, 120.0, 250.0],
                       np.arange(-12.0, 13.0, 4.0))
    return seq, grid


@pytest.mark.parametrize("taps", [3, 5])
def test_smoothed_dictionary_matches_independent_one(orc, taps):
    """Dictionary entries of a smoothing sequence = the expm dictionary
    smoothed by NumPy; the CC map and brute force follow from it."""
    seq, grid = _tiny(taps)
    D0 = np.stack([bloch_ref.simulate(seq, *map(float, grid.values(k)))
                   for k in range(grid.size)])
    Ds = _np_smooth(D0, taps, seq.phase_deg)
    D, _ = orc.simulate_grid(seq, grid)
    assert np.max(np.abs(D - Ds)) < 1e-12 * np.max(np.abs(Ds))
    rng = np.random.default_rng(12)
    V = _rand((5, 24), 13) * 0.1 + D0[rng.integers(0, grid.size, 5)]
    Vs = _np_smooth(V, taps, seq.phase_deg)
    m = orc.cc_map(seq, grid, Vs)
    Dn = Ds / np.linalg.norm(Ds, axis=1, keepdims=True)
    Vn = Vs / np.linalg.norm(Vs, axis=1, keepdims=True)
    ref = np.abs(Vn @ Dn.conj().T)
    assert np.max(np.abs(m - ref)) < 1e-13
    res = orc.bruteforce(seq, grid, Vs)
    assert np.array_equal(res["idx"], np.argmax(ref, axis=1))


def test_smoothing_changes_the_dictionary(orc):
    """A plausible slip (the flag ignored on the dictionary side) fails here."""
    seq0, grid = _tiny(0)
    seq3, _ = _tiny(3)
    D0, _ = orc.simulate_grid(seq0, grid)
    D3, _ = orc.simulate_grid(seq3, grid)
    assert np.max(np.abs(D3 - D0)) > 1e-3 * np.max(np.abs(D0))
    # fingerprint generation stays raw: smoothing is an explicit step there
    t = tuple(map(float, grid.values(17)))
    assert np.array_equal(orc.simulate(seq3, *t), orc.simulate(seq0, *t))


def test_zoom_on_smoothed_on_grid_fingerprints_is_exact(orc):
    """ZOOM's objective uses the smoothed dictionary: smoothed on-grid
    fingerprints are found with CC = 1 wherever the schedule lands on them,
    and the result never beats brute force."""
    seq, grid = _tiny(3)
    D, _ = orc.simulate_grid(seq, grid)
    ks = np.array([3, 61, 100, grid.size - 2])
    V = orc.smooth(np.stack([orc.simulate(seq, *map(float, grid.values(k))) for k in ks]), 3, seq)
    z = orc.zoom(seq, grid, orc.schedule_paper(seq, grid), V)
    b = orc.bruteforce(seq, grid, V)
    assert np.array_equal(b["idx"], ks)
    assert np.all(z["cc"] <= b["cc"] + 1e-14)
    hit = z["idx"] == ks
    assert hit.any()
    assert np.all(np.abs(z["cc"][hit] - 1.0) < 1e-12)
