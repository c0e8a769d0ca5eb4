"""Pins of the oracle's Bloch simulator and CC against facts outside the oracle.

Appendix Eq. A1/A2 (Bloch model, hard-pulse RF) and Theory Eq. 1 (CC).
"""
import math

import numpy as np
import pytest

from paper_1506_05393_amd import inputs as I
from tests import bloch_ref


def _const_seq(n, fa, tr, phases=None, te=None):
    ph = np.where(np.arange(n) % 2 == 0, 0.0, 180.0) if phases is None else np.asarray(phases, float)
    te = tr / 2 if te is None else te
    return I.Sequence(np.full(n, float(fa)), ph, np.full(n, float(tr)), np.full(n, float(te)), 1, 0.0)


@pytest.mark.parametrize("params", [(1000.0, 100.0, 10.0, 1.0), (300.0, 40.0, -37.5, 0.8),
                                    (2500.0, 1500.0, 55.0, 1.2), (80.0, 20.0, 0.0, 1.0)])
def test_matches_matrix_exponential_integration(orc, params):
    """Independent integration of Eq. A1 (expm of the generator) + Rodrigues RF."""
    seq = I.make_sequence(40, 3)
    seq.ti_ms = 7.0
    a = orc.simulate(seq, *params)
    b = bloch_ref.simulate(seq, *params)
    assert np.max(np.abs(a - b)) < 1e-12


def test_general_rf_phase_matches_reference(orc):
    seq = I.make_sequence(30, 5)
    seq.phase_deg = np.random.default_rng(1).uniform(0, 360, 30)
    a = orc.simulate(seq, 900.0, 70.0, 23.0, 1.0)
    b = bloch_ref.simulate(seq, 900.0, 70.0, 23.0, 1.0)
    assert np.max(np.abs(a - b)) < 1e-12


@pytest.mark.parametrize("t1,t2,df,b1,ti", [(1000.0, 100.0, 10.0, 1.0, 0.0),
                                             (450.0, 60.0, -31.0, 0.9, 12.0)])
def test_first_sample_closed_form(orc, t1, t2, df, b1, ti):
    """s_0 = i Mz(TI) sin(B1 a0) e^{i phi0} e^{-TE0/T2} e^{i 2 pi df TE0/1000}."""
    seq = I.make_sequence(5, 2)
    seq.ti_ms = ti
    seq.phase_deg = np.array([33.0, 0, 0, 0, 0])
    s = orc.simulate(seq, t1, t2, df, b1)
    mz = 1.0 - 2.0 * math.exp(-ti / t1)
    te = seq.te_ms[0]
    want = (1j * mz * math.sin(math.radians(b1 * seq.fa_deg[0])) * np.exp(1j * math.radians(33.0))
            * math.exp(-te / t2) * np.exp(1j * 2 * math.pi * df * te / 1000.0))
    assert abs(s[0] - want) < 1e-14


def test_inversion_recovery_when_flip_angle_zero(orc):
    """FA = 0: Mz(t) = 1 - 2 exp(-t/T1) at every TR boundary and s = 0."""
    seq = I.make_sequence(60, 4)
    seq.fa_deg[:] = 0.0
    t1 = 730.0
    st = orc.trajectory(seq, t1, 80.0, 12.0)
    s = orc.simulate(seq, t1, 80.0, 12.0)
    assert np.max(np.abs(s)) == 0.0
    t_end = np.cumsum(seq.tr_ms)
    want = 1.0 - 2.0 * np.exp(-t_end / t1)
    assert np.max(np.abs(st[:, 2, 2] - want)) < 1e-14
    # B1 = 0 scales every flip angle to zero: same closed form
    seq2 = I.make_sequence(60, 4)
    st2 = orc.trajectory(seq2, t1, 80.0, 12.0, b1=0.0)
    assert np.max(np.abs(st2[:, 2, 2] - want)) < 1e-14


def test_norm_preserved_without_relaxation(orc):
    """T1 = T2 = inf: rotations only, so |M| = 1 after every operation."""
    seq = I.make_sequence(80, 6)
    st = orc.trajectory(seq, math.inf, math.inf, 17.0)
    assert np.max(np.abs(np.linalg.norm(st, axis=2) - 1.0)) < 1e-13


@pytest.mark.parametrize("alpha,tr,t1,t2", [(60.0, 10.0, 1000.0, 100.0),
                                           (30.0, 12.0, 800.0, 300.0),
                                           (45.0, 5.0, 300.0, 30.0)])
def test_bssfp_steady_state(orc, alpha, tr, t1, t2):
    """Constant alpha/TR, alternating phase, df = 0, TE = TR/2: on-resonance
    bSSFP steady state |s| = sin(a)(1-E1) sqrt(E2) / (1 - (E1-E2)cos(a) - E1 E2)."""
    # transient decays roughly as exp(-TR (cos^2(a/2)/T1 + sin^2(a/2)/T2)) per TR
    h = math.radians(alpha) / 2
    rate = tr * (math.cos(h) ** 2 / t1 + math.sin(h) ** 2 / t2)
    n = int(40.0 / rate) + 2
    seq = _const_seq(n, alpha, tr)
    s = orc.simulate(seq, t1, t2, 0.0)
    e1, e2 = math.exp(-tr / t1), math.exp(-tr / t2)
    a = math.radians(alpha)
    want = math.sin(a) * (1 - e1) * math.sqrt(e2) / (1 - (e1 - e2) * math.cos(a) - e1 * e2)
    assert abs(abs(s[-1]) - want) < 1e-9
    assert abs(abs(s[-2]) - want) < 1e-9


def test_mirror_symmetry_in_df(orc):
    """Phases in {0, 180}: s(-df) = -conj(s(df)); Re s = 0 at df = 0."""
    seq = I.make_sequence(120, 7)
    a = orc.simulate(seq, 900.0, 90.0, 23.0)
    b = orc.simulate(seq, 900.0, 90.0, -23.0)
    assert np.max(np.abs(b + np.conj(a))) < 1e-14
    z = orc.simulate(seq, 900.0, 90.0, 0.0)
    assert np.max(np.abs(z.real)) < 1e-15


def test_df_periodicity_constant_tr(orc):
    """Constant TR, TE = TR/2: s(df + 1000/TR) = -s(df) (Property II, exact case)."""
    tr = 12.5
    seq = _const_seq(150, 40.0, tr)
    seq.fa_deg = 10 + 50 * np.abs(np.sin(np.arange(150) / 20.0))
    a = orc.simulate(seq, 1100.0, 120.0, 9.0)
    b = orc.simulate(seq, 1100.0, 120.0, 9.0 + 1000.0 / tr)
    assert np.max(np.abs(a + b)) < 1e-11


def test_alternating_phase_equals_shifted_df(orc):
    """Constant TR, TE = TR/2: s_alt(df) = (-1)^j (-i) s_0(df + 1000/(2 TR))."""
    tr, n = 11.0, 90
    seq_alt = _const_seq(n, 35.0, tr)
    seq_alt.fa_deg = 20 + 30 * np.abs(np.sin(np.arange(n) / 9.0))
    seq0 = _const_seq(n, 35.0, tr, phases=np.zeros(n))
    seq0.fa_deg = seq_alt.fa_deg.copy()
    a = orc.simulate(seq_alt, 700.0, 60.0, 5.0)
    b = orc.simulate(seq0, 700.0, 60.0, 5.0 + 1000.0 / (2 * tr))
    sign = (-1.0) ** np.arange(n)
    assert np.max(np.abs(a - sign * (-1j) * b)) < 1e-12


def test_global_rf_phase_offset(orc):
    """Adding psi to every RF phase multiplies the signal by e^{i psi}."""
    seq = I.make_sequence(70, 8)
    a = orc.simulate(seq, 1200.0, 150.0, -14.0)
    seq.phase_deg = seq.phase_deg + 47.0
    b = orc.simulate(seq, 1200.0, 150.0, -14.0)
    assert np.max(np.abs(b - a * np.exp(1j * math.radians(47.0)))) < 1e-13


def test_b1_one_is_three_parameter_entry(orc):
    seq = I.make_sequence(50, 9)
    g3 = I.make_grid([500.0, 900.0], [50.0, 80.0], [-4.0, 0.0, 4.0])
    g4 = I.make_grid([500.0, 900.0], [50.0, 80.0], [-4.0, 0.0, 4.0], [0.9, 1.0])
    d3, n3 = orc.simulate_grid(seq, g3)
    d4, n4 = orc.simulate_grid(seq, g4)
    assert np.array_equal(d4[1::2], d3)


def test_grid_tables_bitwise_equal_direct(orc):
    """Per-axis factor tables give bit-identical entries to direct evaluation."""
    seq = I.make_sequence(64, 10)
    g = I.make_grid([300.0, 1000.0, 2100.0], [20.0, 90.0], [-12.0, 0.0, 7.5], [0.8, 1.1])
    d, nrm = orc.simulate_grid(seq, g, threads=2)
    for k in range(g.size):
        t1, t2, df, b1 = g.values(k)
        e = orc.simulate(seq, float(t1), float(t2), float(df), float(b1))
        assert np.array_equal(e, d[k])
        acc = 0.0
        for x in e:  # sequential sum, the order the oracle uses
            acc += x.real * x.real + x.imag * x.imag
        assert nrm[k] == math.sqrt(acc)


def test_cc_definition_properties(orc):
    rng = np.random.default_rng(0)
    v = rng.normal(size=50) + 1j * rng.normal(size=50)
    d = rng.normal(size=50) + 1j * rng.normal(size=50)
    c = orc.cc(v, d)
    want = abs(np.sum(v * np.conj(d))) / (np.linalg.norm(v) * np.linalg.norm(d))
    assert abs(c - want) < 1e-15
    assert abs(orc.cc(v, (0.3 - 2.1j) * v) - 1.0) < 1e-14
    assert abs(orc.cc(v * 7.5 * np.exp(0.4j), d) - c) < 1e-14
    assert 0.0 <= c <= 1.0
    assert orc.cc(v, np.zeros(50)) == 0.0
    assert orc.cc(np.zeros(50), d) == 0.0


def test_rejects_bad_timing(orc):
    seq = I.make_sequence(10, 0)
    seq.te_ms = seq.tr_ms.copy()
    with pytest.raises(ValueError):
        orc.simulate(seq, 1000.0, 100.0, 0.0)
