"""Independent reference integration of the Bloch model for tiny cases.

Free evolution is the matrix exponential of the generator of Eq. A1 in
homogeneous coordinates (precession counter-clockwise about z at 2*pi*df/1000
rad/ms, as R_off of Eq. A2; relaxation toward M0 = 1), and the hard RF pulse is
Rodrigues' rotation by -alpha about the transverse axis at the RF phase, which
is the conjugation Rz(phi) Rx(-alpha) Rz(-phi) of the Appendix. Nothing here
shares code with the oracle; loops are plain Python.
"""
import math

import numpy as np
from scipy.linalg import expm


def free_op(t_ms, t1, t2, df):
    w = 2.0 * math.pi * df / 1000.0
    r1 = 0.0 if math.isinf(t1) else 1.0 / t1
    r2 = 0.0 if math.isinf(t2) else 1.0 / t2
    G = np.array([[-r2, -w, 0.0, 0.0],
                  [w, -r2, 0.0, 0.0],
                  [0.0, 0.0, -r1, r1],
                  [0.0, 0.0, 0.0, 0.0]])
    return expm(G * t_ms)


def rf_op(alpha_deg, phase_deg):
    th = -math.radians(alpha_deg)
    p = math.radians(phase_deg)
    n = np.array([math.cos(p), math.sin(p), 0.0])
    K = np.array([[0.0, -n[2], n[1]], [n[2], 0.0, -n[0]], [-n[1], n[0], 0.0]])
    R = np.eye(3) * math.cos(th) + math.sin(th) * K + (1.0 - math.cos(th)) * np.outer(n, n)
    H = np.eye(4)
    H[:3, :3] = R
    return H


def simulate(seq, t1, t2, df, b1=1.0, n_tr=None):
    n_tr = seq.n if n_tr is None else n_tr
    M = np.array([0.0, 0.0, 1.0, 1.0])
    if seq.inversion:
        M[2] = -1.0
    if seq.ti_ms > 0:
        M = free_op(seq.ti_ms, t1, t2, df) @ M
    out = np.zeros(n_tr, np.complex128)
    for j in range(n_tr):
        M = rf_op(b1 * seq.fa_deg[j], seq.phase_deg[j]) @ M
        M = free_op(seq.te_ms[j], t1, t2, df) @ M
        out[j] = M[0] + 1j * M[1]
        M = free_op(seq.tr_ms[j] - seq.te_ms[j], t1, t2, df) @ M
    return out
