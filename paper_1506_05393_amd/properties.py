"""Checks of the three empirical CC properties of the Theory section on a CC
map (one fingerprint against a whole grid, as in Experiment 1).

Property I: for every (T1, T2) the CC along df peaks at the fingerprint's df.
Property II: along df the CC is pseudo-periodic with period 1000/TR Hz (TR
in ms): side peaks near multiples of that period, decaying with distance.
Property III: at the fingerprint's df, CC along T1 (for each T2) and along T2
(for each T1) is unimodal, and the peaks line up near one T1 (one T2).

The map is host data (numpy); the functions only locate maxima and count
them, so they apply equally to a GPU map and to the oracle's.
"""
from __future__ import annotations

import numpy as np


def _local_maxima(x: np.ndarray, rel: float) -> np.ndarray:
    """Indices of maxima of a 1-D profile: strictly above both neighbours (an
    end point only needs to beat its one neighbour), ignoring bumps smaller
    than rel * (max - min) of the profile."""
    x = np.asarray(x, np.float64)
    n = x.shape[0]
    if n == 1:
        return np.array([0])
    tol = rel * float(x.max() - x.min())
    left = np.empty(n, bool)
    right = np.empty(n, bool)
    left[0] = True
    right[-1] = True
    left[1:] = x[1:] > x[:-1] + tol
    right[:-1] = x[:-1] > x[1:] + tol
    return np.flatnonzero(left & right)


def check(cc: np.ndarray, dims, df_hz: np.ndarray, t1_ms: np.ndarray, t2_ms: np.ndarray,
          tr_ms: np.ndarray, truth=None, rel: float = 1e-6) -> dict:
    """cc: CC map of one fingerprint, flat in grid order (T1 slowest, then
    T2, df, B1) or shaped dims = (n1, n2, n3[, n4]). truth: grid indices
    (i1, i2, i3[, i4]) of the fingerprint, or None to use the map's argmax.
    tr_ms: the sequence's repetition times (the period of Property II is
    1000 / mean TR)."""
    dims = tuple(int(d) for d in dims)
    m = np.asarray(cc, np.float64).reshape(dims)
    if m.ndim == 4:  # B1 axis: take the slice through the truth / argmax
        b = truth[3] if truth is not None else np.unravel_index(np.argmax(m), m.shape)[3]
        m = m[..., b]
    n1, n2, n3 = m.shape
    top = np.unravel_index(int(np.argmax(m)), m.shape)
    i1, i2, i3 = (truth[:3] if truth is not None else top)
    i1, i2, i3 = int(i1), int(i2), int(i3)

    # Property I
    arg_df = np.argmax(m, axis=2)
    p1 = {"df_index": i3,
          "global_max_at_df": bool(top[2] == i3),
          "frac_columns_peak_at_df": float(np.mean(arg_df == i3)),
          "frac_columns_peak_within_1": float(np.mean(np.abs(arg_df - i3) <= 1)),
          "columns": int(n1 * n2)}

    # Property II
    omega = 1000.0 / float(np.mean(tr_ms))
    prof = m[i1, i2, :]
    peaks = [int(p) for p in _local_maxima(prof, rel) if p != i3]
    peaks.sort(key=lambda p: -prof[p])
    side = []
    for p in peaks[:6]:
        off = float(df_hz[p] - df_hz[i3])
        side.append({"offset_hz": off, "offset_over_period": off / omega, "cc": float(prof[p])})
    near = sorted(side, key=lambda d: abs(d["offset_hz"]))
    heights = [d["cc"] for d in near]
    p2 = {"period_hz": omega, "main_cc": float(prof[i3]), "side_peaks": side,
          "side_peaks_below_main": bool(all(h < prof[i3] for h in heights)),
          "nearest_side_peak_over_period": (abs(near[0]["offset_over_period"]) if near else None)}

    # Property III
    s = m[:, :, i3]  # [n1, n2]
    t1_peaks = [len(_local_maxima(s[:, k], rel)) for k in range(n2)]
    t2_peaks = [len(_local_maxima(s[k, :], rel)) for k in range(n1)]
    arg_t1 = np.argmax(s, axis=0)
    arg_t2 = np.argmax(s, axis=1)
    p3 = {"frac_t1_profiles_unimodal": float(np.mean(np.array(t1_peaks) == 1)),
          "frac_t2_profiles_unimodal": float(np.mean(np.array(t2_peaks) == 1)),
          "t1_peak_spread_ms": float(np.ptp(t1_ms[arg_t1])),
          "t1_peak_median_ms": float(np.median(t1_ms[arg_t1])),
          "t2_peak_spread_ms": float(np.ptp(t2_ms[arg_t2])),
          "t2_peak_median_ms": float(np.median(t2_ms[arg_t2])),
          "t1_at_truth_ms": float(t1_ms[i1]), "t2_at_truth_ms": float(t2_ms[i2])}
    return {"property_I": p1, "property_II": p2, "property_III": p3,
            "argmax": [int(t) for t in top], "max_cc": float(m[top])}
