"""The Property I-III checker on maps whose answers are known, and on an
oracle CC map (Theory: empirical properties of CC; Experiment 1)."""
import numpy as np

from paper_1506_05393_amd import inputs as I
from paper_1506_05393_amd import properties as P


def _axes():
    t1 = np.arange(100.0, 2000.0, 50.0)
    t2 = np.arange(20.0, 400.0, 20.0)
    df = np.arange(-60.0, 60.0, 1.0)
    return t1, t2, df


def test_separable_map_has_all_three_properties():
    t1, t2, _ = _axes()
    df = np.arange(-120.0, 120.0, 1.0)
    tr = np.full(10, 12.5)  # period 80 Hz
    w = 1000.0 / 12.5
    a = np.exp(-((t1 - 900.0) / 400.0) ** 2)
    b = np.exp(-((t2 - 120.0) / 90.0) ** 2)
    c = (0.6 + 0.4 * np.cos(2 * np.pi * (df - 5.0) / w)) * np.exp(-np.abs(df - 5.0) / 300.0)
    m = a[:, None, None] * b[None, :, None] * c[None, None, :]
    r = P.check(m.ravel(), m.shape, df, t1, t2, tr)
    assert r["argmax"] == [16, 5, 125]
    assert r["property_I"]["global_max_at_df"]
    assert r["property_I"]["frac_columns_peak_at_df"] == 1.0
    side = r["property_II"]["side_peaks"]
    assert r["property_II"]["side_peaks_below_main"]
    # the side peaks sit one period away on either side (within the decay's shift)
    assert min(abs(abs(s["offset_over_period"]) - 1.0) for s in side) < 0.1
    assert r["property_III"]["frac_t1_profiles_unimodal"] == 1.0
    assert r["property_III"]["frac_t2_profiles_unimodal"] == 1.0
    assert r["property_III"]["t1_peak_spread_ms"] == 0.0


def test_violations_are_reported():
    t1, t2, df = _axes()
    tr = np.full(10, 12.5)
    a = np.exp(-((t1 - 500.0) / 150.0) ** 2) + 0.8 * np.exp(-((t1 - 1600.0) / 150.0) ** 2)
    b = np.exp(-((t2 - 120.0) / 90.0) ** 2)
    c = np.exp(-((df - 5.0) / 10.0) ** 2)
    m = a[:, None, None] * b[None, :, None] * c[None, None, :]
    # T2 columns 0..3 peak at another df (Property I broken there)
    m[:, :4, :] = m[:, :4, ::-1]
    r = P.check(m.ravel(), m.shape, df, t1, t2, tr, truth=(8, 5, 65))
    assert r["property_III"]["frac_t1_profiles_unimodal"] == 0.0  # bimodal along T1
    assert abs(r["property_I"]["frac_columns_peak_at_df"] - (len(t2) - 4) / len(t2)) < 1e-12


def test_oracle_map_of_an_on_grid_fingerprint(orc):
    """Noise-free on-grid fingerprint: the map peaks at the truth with CC = 1
    and Property I holds at the global maximum."""
    seq = I.make_sequence(120, 4)
    grid = I.make_grid(np.arange(300.0, 1800.0, 100.0), np.arange(40.0, 300.0, 20.0),
                       np.arange(-30.0, 31.0, 2.0))
    t = (7, 5, 20)
    k = (t[0] * len(grid.t2_ms) + t[1]) * len(grid.df_hz) + t[2]
    v = orc.simulate(seq, *map(float, grid.values(k)))[None]
    m = orc.cc_map(seq, grid, v)[0]
    r = P.check(m, (len(grid.t1_ms), len(grid.t2_ms), len(grid.df_hz)), grid.df_hz,
                grid.t1_ms, grid.t2_ms, seq.tr_ms)
    assert r["argmax"] == list(t)
    assert abs(r["max_cc"] - 1.0) < 1e-12
    assert r["property_I"]["global_max_at_df"]
    assert r["property_I"]["frac_columns_peak_within_1"] > 0.5
