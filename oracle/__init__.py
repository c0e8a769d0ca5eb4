"""ctypes binding of the FP64 CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package. The product path never does; it shares no code with it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Callable, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mrf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

SCAN_STRIDE, SCAN_WINDOW, SCAN_HOPS, ZOOM1, ZOOM2 = range(5)
MAX_STAGES, MAX_STARTS = 64, 16


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (IEEE FP64, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-ffp-contract=off", "-fno-fast-math", "-Wall",
                               "-Wno-unused-function", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Seq(C.Structure):
    _fields_ = [("n", C.c_int32), ("fa_deg", C.POINTER(C.c_double)),
                ("phase_deg", C.POINTER(C.c_double)), ("tr_ms", C.POINTER(C.c_double)),
                ("te_ms", C.POINTER(C.c_double)), ("inversion", C.c_int32),
                ("ti_ms", C.c_double), ("smooth", C.c_int32)]


class GridS(C.Structure):
    _fields_ = [("n1", C.c_int32), ("n2", C.c_int32), ("n3", C.c_int32), ("n4", C.c_int32),
                ("t1", C.POINTER(C.c_double)), ("t2", C.POINTER(C.c_double)),
                ("df", C.POINTER(C.c_double)), ("b1", C.POINTER(C.c_double))]


class Stage(C.Structure):
    _fields_ = [("kind", C.c_int32), ("axis0", C.c_int32), ("axis1", C.c_int32),
                ("step0", C.c_int32), ("step1", C.c_int32), ("window", C.c_int32),
                ("hop", C.c_double), ("objective", C.c_int32)]


OBJ_CC, OBJ_DIST = 0, 1


class Schedule(C.Structure):
    _fields_ = [("n_stages", C.c_int32), ("stages", Stage * MAX_STAGES),
                ("n_outer", C.c_int32), ("outer", Stage * MAX_STAGES),
                ("outer_max", C.c_int32), ("n_starts", C.c_int32),
                ("starts", (C.c_int32 * 4) * MAX_STARTS), ("pruned", C.c_int32),
                ("prior_half", C.c_int32 * 4)]


OBJECTIVE = C.CFUNCTYPE(C.c_double, C.c_void_p, C.POINTER(C.c_int32))
OBJECTIVE2 = C.CFUNCTYPE(None, C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_double))

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        dp, ip, lp = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64)
        L.orc_simulate.argtypes = [C.POINTER(Seq), C.c_int32, C.c_double, C.c_double,
                                   C.c_double, C.c_double, dp, dp]
        L.orc_trajectory.argtypes = [C.POINTER(Seq), C.c_int32, C.c_double, C.c_double,
                                     C.c_double, C.c_double, dp]
        L.orc_simulate_grid.argtypes = [C.POINTER(Seq), C.POINTER(GridS), C.c_int32,
                                        C.c_int64, C.c_int64, dp, dp, dp, C.c_int32]
        L.orc_cc.argtypes = [C.c_int32, dp, dp, dp, dp]
        L.orc_smooth.argtypes = [C.c_int32, C.c_int32, dp, dp, dp]
        L.orc_cc.restype = C.c_double
        L.orc_bruteforce.argtypes = [C.POINTER(Seq), C.POINTER(GridS), C.c_int32, dp, dp,
                                     C.c_int32, C.c_int32, lp, dp, dp, dp, dp, lp, dp,
                                     C.c_int32]
        L.orc_cc_map.argtypes = [C.POINTER(Seq), C.POINTER(GridS), C.c_int32, dp, dp,
                                 C.c_int32, C.c_int64, C.c_int64, dp, C.c_int32]
        L.orc_schedule_paper.argtypes = [C.POINTER(GridS), C.POINTER(Seq),
                                         C.POINTER(Schedule)]
        L.orc_cc_at.argtypes = [C.POINTER(Seq), C.POINTER(GridS), C.c_int32, dp, dp, C.c_int32,
                                C.c_int32, lp, dp, C.c_int32]
        L.orc_prior_half.argtypes = [C.POINTER(GridS), dp, ip]
        L.orc_schedule_finest_objective.argtypes = [C.POINTER(Schedule), C.c_int32]
        L.orc_schedule_multistart.argtypes = [C.POINTER(GridS), C.POINTER(Seq), C.c_int32,
                                              C.c_int32, C.c_int32, C.POINTER(Schedule)]
        L.orc_objectives_at.argtypes = [C.POINTER(Seq), C.POINTER(GridS), C.c_int32, dp, dp,
                                        C.c_int32, C.c_int32, lp, dp, dp, C.c_int32]
        L.orc_zoom_generic.argtypes = [C.POINTER(Schedule), ip, ip, OBJECTIVE, C.c_void_p,
                                       ip, dp, ip, dp, ip, C.c_int32, ip]
        L.orc_zoom_generic2.argtypes = [C.POINTER(Schedule), ip, ip, OBJECTIVE2, C.c_void_p,
                                        ip, dp, ip, dp, ip, C.c_int32, ip]
        L.orc_zoom.argtypes = [C.POINTER(Seq), C.POINTER(GridS), C.c_int32,
                               C.POINTER(Schedule), dp, dp, C.c_int32, ip, lp, dp, dp, ip, dp,
                               C.c_int32]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class _Keep:
    """Holds numpy buffers alive while a ctypes struct points into them."""


def make_seq(seq) -> tuple:
    k = _Keep()
    k.fa = np.ascontiguousarray(seq.fa_deg, np.float64)
    k.ph = np.ascontiguousarray(seq.phase_deg, np.float64)
    k.tr = np.ascontiguousarray(seq.tr_ms, np.float64)
    k.te = np.ascontiguousarray(seq.te_ms, np.float64)
    s = Seq(len(k.fa), _dp(k.fa), _dp(k.ph), _dp(k.tr), _dp(k.te), int(seq.inversion),
            float(seq.ti_ms), int(getattr(seq, "smooth", 0)))
    return s, k


def make_grid(grid) -> tuple:
    k = _Keep()
    k.t1 = np.ascontiguousarray(grid.t1_ms, np.float64)
    k.t2 = np.ascontiguousarray(grid.t2_ms, np.float64)
    k.df = np.ascontiguousarray(grid.df_hz, np.float64)
    k.b1 = np.ascontiguousarray(grid.b1 if len(grid.b1) else np.ones(1), np.float64)
    g = GridS(len(k.t1), len(k.t2), len(k.df), len(grid.b1), _dp(k.t1), _dp(k.t2),
              _dp(k.df), _dp(k.b1))
    return g, k


def _threads(n):
    return int(n) if n else 0


def simulate(seq, t1, t2, df, b1=1.0, n_tr=None) -> np.ndarray:
    """One entry, complex128 [n_tr] (raw, not normalised)."""
    n_tr = seq.n if n_tr is None else n_tr
    s, keep = make_seq(seq)
    re = np.zeros(n_tr)
    im = np.zeros(n_tr)
    rc = lib().orc_simulate(C.byref(s), n_tr, t1, t2, df, b1, _dp(re), _dp(im))
    if rc:
        raise ValueError(f"orc_simulate failed ({rc})")
    return re + 1j * im


def trajectory(seq, t1, t2, df, b1=1.0, n_tr=None) -> np.ndarray:
    """[n_tr, 3, 3]: M after the pulse, at TE and at the end of each TR."""
    n_tr = seq.n if n_tr is None else n_tr
    s, keep = make_seq(seq)
    st = np.zeros(n_tr * 9)
    rc = lib().orc_trajectory(C.byref(s), n_tr, t1, t2, df, b1, _dp(st))
    if rc:
        raise ValueError(f"orc_trajectory failed ({rc})")
    return st.reshape(n_tr, 3, 3)


def simulate_grid(seq, grid, k0=0, count=None, n_tr=None, threads=0):
    """Entries [k0, k0+count): complex128 [count, n_tr] raw, and norms [count]."""
    n_tr = seq.n if n_tr is None else n_tr
    count = grid.size - k0 if count is None else count
    s, ks = make_seq(seq)
    g, kg = make_grid(grid)
    re = np.zeros((count, n_tr))
    im = np.zeros((count, n_tr))
    nrm = np.zeros(count)
    rc = lib().orc_simulate_grid(C.byref(s), C.byref(g), n_tr, k0, count, _dp(re), _dp(im),
                                 _dp(nrm), _threads(threads))
    if rc:
        raise ValueError(f"orc_simulate_grid failed ({rc})")
    return re + 1j * im, nrm


def smooth(x, taps: int, phase_deg=None) -> np.ndarray:
    """Temporal smoothing of complex signals along the last axis (Methods,
    Experiment 4): binomial 3- or 5-point weights, renormalised at the ends,
    applied in the frame demodulated by the RF phases phase_deg (one per
    readout; a sequence, whose phase_deg is taken, or None for zero phases)
    and modulated back; taps 0 or 1 return a copy."""
    if phase_deg is not None and hasattr(phase_deg, "phase_deg"):
        phase_deg = phase_deg.phase_deg
    x = np.asarray(x, np.complex128)
    flat = x.reshape(-1, x.shape[-1]) if x.ndim else x.reshape(1, 1)
    out = np.empty_like(flat)
    n = flat.shape[-1]
    ph = None
    if phase_deg is not None:
        ph = np.ascontiguousarray(np.asarray(phase_deg, np.float64)[:n])
        if ph.shape[0] < n:
            raise ValueError("phase_deg shorter than the signals")
    for r in range(flat.shape[0]):
        re = np.ascontiguousarray(flat[r].real)
        im = np.ascontiguousarray(flat[r].imag)
        rc = lib().orc_smooth(n, int(taps), _dp(ph) if ph is not None else None, _dp(re), _dp(im))
        if rc != 0:
            raise ValueError(f"orc_smooth failed ({rc}): taps must be 0, 1, 3 or 5")
        out[r] = re + 1j * im
    return out.reshape(x.shape)


def cc(v, d) -> float:
    v = np.asarray(v, np.complex128)
    d = np.asarray(d, np.complex128)
    vr, vi = np.ascontiguousarray(v.real), np.ascontiguousarray(v.imag)
    dr, di = np.ascontiguousarray(d.real), np.ascontiguousarray(d.imag)
    return float(lib().orc_cc(len(v), _dp(vr), _dp(vi), _dp(dr), _dp(di)))


def cc_at(seq, grid, vox, idx, n_tr=None, threads=0) -> np.ndarray:
    """CC (Eq. 1) of each voxel against listed entries: vox complex [n_vox,
    n_tr], idx int [n_vox, m] grid indices (negative: 0). float64 [n_vox, m]."""
    vox = np.atleast_2d(np.asarray(vox, np.complex128))
    n_vox = vox.shape[0]
    n_tr = vox.shape[1] if n_tr is None else n_tr
    vox = vox[:, :n_tr]
    idx = np.ascontiguousarray(np.asarray(idx, np.int64).reshape(n_vox, -1))
    m = idx.shape[1]
    s, ks = make_seq(seq)
    g, kg = make_grid(grid)
    vr = np.ascontiguousarray(vox.real)
    vi = np.ascontiguousarray(vox.imag)
    out = np.zeros((n_vox, m))
    rc = lib().orc_cc_at(C.byref(s), C.byref(g), n_tr, _dp(vr), _dp(vi), n_vox, m,
                         idx.ctypes.data_as(C.POINTER(C.c_int64)), _dp(out), _threads(threads))
    if rc:
        raise ValueError(f"orc_cc_at failed ({rc})")
    return out


def objectives_at(seq, grid, vox, idx, n_tr=None, threads=0) -> tuple:
    """(cc, score) float64 [n_vox, m]: both ZOOM objectives of each voxel at
    listed entries idx [n_vox, m] (negative: 0 and -inf)."""
    vox = np.atleast_2d(np.asarray(vox, np.complex128))
    n_vox = vox.shape[0]
    n_tr = vox.shape[1] if n_tr is None else n_tr
    vox = vox[:, :n_tr]
    idx = np.ascontiguousarray(np.asarray(idx, np.int64).reshape(n_vox, -1))
    m = idx.shape[1]
    s, ks = make_seq(seq)
    g, kg = make_grid(grid)
    vr = np.ascontiguousarray(vox.real)
    vi = np.ascontiguousarray(vox.imag)
    cc = np.zeros((n_vox, m))
    sc = np.zeros((n_vox, m))
    rc = lib().orc_objectives_at(C.byref(s), C.byref(g), n_tr, _dp(vr), _dp(vi), n_vox, m,
                                 idx.ctypes.data_as(C.POINTER(C.c_int64)), _dp(cc), _dp(sc),
                                 _threads(threads))
    if rc:
        raise ValueError(f"orc_objectives_at failed ({rc})")
    return cc, sc


def bruteforce(seq, grid, vox, top_k=1, n_tr=None, threads=0) -> dict:
    """vox: complex [n_vox, n_tr]. Returns idx, cc, margin, pd, topk_idx, topk_cc."""
    vox = np.asarray(vox, np.complex128)
    n_vox = vox.shape[0]
    n_tr = vox.shape[1] if n_tr is None else n_tr
    vox = vox[:, :n_tr]
    s, ks = make_seq(seq)
    g, kg = make_grid(grid)
    vr = np.ascontiguousarray(vox.real)
    vi = np.ascontiguousarray(vox.imag)
    idx = np.zeros(n_vox, np.int64)
    ccv = np.zeros(n_vox)
    mg = np.zeros(n_vox)
    pr = np.zeros(n_vox)
    pi = np.zeros(n_vox)
    tki = np.zeros((n_vox, top_k), np.int64)
    tkc = np.zeros((n_vox, top_k))
    lp = lambda a: a.ctypes.data_as(C.POINTER(C.c_int64))
    rc = lib().orc_bruteforce(C.byref(s), C.byref(g), n_tr, _dp(vr), _dp(vi), n_vox, top_k,
                              lp(idx), _dp(ccv), _dp(mg), _dp(pr), _dp(pi), lp(tki), _dp(tkc),
                              _threads(threads))
    if rc:
        raise ValueError(f"orc_bruteforce failed ({rc})")
    return dict(idx=idx, cc=ccv, margin=mg, pd=pr + 1j * pi, topk_idx=tki, topk_cc=tkc)


def cc_map(seq, grid, vox, k0=0, count=None, n_tr=None, threads=0) -> np.ndarray:
    """CC (Eq. 1) of each fingerprint against every entry of [k0, k0 + count)
    of the grid (Experiment 1's CC mapping): float64 [n_vox][count]."""
    vox = np.atleast_2d(np.asarray(vox, np.complex128))
    n_vox = vox.shape[0]
    n_tr = vox.shape[1] if n_tr is None else n_tr
    vox = vox[:, :n_tr]
    s, ks = make_seq(seq)
    g, kg = make_grid(grid)
    count = grid.size - k0 if count is None else count
    vr = np.ascontiguousarray(vox.real)
    vi = np.ascontiguousarray(vox.imag)
    out = np.zeros((n_vox, count))
    rc = lib().orc_cc_map(C.byref(s), C.byref(g), n_tr, _dp(vr), _dp(vi), n_vox, int(k0),
                          int(count), _dp(out), _threads(threads))
    if rc:
        raise ValueError(f"orc_cc_map failed ({rc})")
    return out


def schedule_to_dict(s: Schedule) -> dict:
    st = lambda x: dict(kind=x.kind, axis0=x.axis0, axis1=x.axis1, step0=x.step0,
                        step1=x.step1, window=x.window, hop=x.hop, objective=x.objective)
    return dict(stages=[st(s.stages[i]) for i in range(s.n_stages)],
                outer=[st(s.outer[i]) for i in range(s.n_outer)], outer_max=s.outer_max,
                starts=[list(s.starts[i]) for i in range(s.n_starts)], pruned=s.pruned,
                prior_half=list(s.prior_half))


def schedule_from_dict(d: dict) -> Schedule:
    s = Schedule()
    mk = lambda x: Stage(x["kind"], x["axis0"], x.get("axis1", 0), x.get("step0", 0),
                         x.get("step1", 0), x.get("window", 0), x.get("hop", 0.0),
                         x.get("objective", OBJ_CC))
    s.n_stages = len(d["stages"])
    for i, x in enumerate(d["stages"]):
        s.stages[i] = mk(x)
    s.n_outer = len(d.get("outer", []))
    for i, x in enumerate(d.get("outer", [])):
        s.outer[i] = mk(x)
    s.outer_max = d.get("outer_max", 0)
    starts = d.get("starts", [[0, 0, 0, 0]])
    s.n_starts = len(starts)
    for i, st in enumerate(starts):
        for a in range(4):
            s.starts[i][a] = int(st[a])
    s.pruned = int(d.get("pruned", 0))
    ph = d.get("prior_half", [-1, -1, -1, -1])
    for a in range(4):
        s.prior_half[a] = int(ph[a])
    return s


def schedule_paper(seq, grid) -> dict:
    s, ks = make_seq(seq)
    g, kg = make_grid(grid)
    out = Schedule()
    rc = lib().orc_schedule_paper(C.byref(g), C.byref(s), C.byref(out))
    if rc:
        raise ValueError("orc_schedule_paper failed")
    return schedule_to_dict(out)


def schedule_multistart(seq, grid, k1: int = 4, k2: int = 4, outer_max: int = 8) -> dict:
    """The paper's stages from a k1 x k2 start lattice, then outer rounds."""
    s, ks = make_seq(seq)
    g, kg = make_grid(grid)
    out = Schedule()
    if lib().orc_schedule_multistart(C.byref(g), C.byref(s), k1, k2, outer_max, C.byref(out)):
        raise ValueError("orc_schedule_multistart failed")
    return schedule_to_dict(out)


def schedule_finest_objective(sched: dict, objective: int = OBJ_DIST) -> dict:
    """A copy of the schedule whose unit-step stages use `objective`."""
    s = schedule_from_dict(sched)
    if lib().orc_schedule_finest_objective(C.byref(s), int(objective)):
        raise ValueError("orc_schedule_finest_objective failed")
    return schedule_to_dict(s)


def prior_half(grid, half=None) -> list:
    """Neighbour-prior half widths (Experiment 3) in index steps for physical
    half widths (T1 ms, T2 ms, df Hz, B1); None: 3000, 800, 150, 0.3."""
    g, kg = make_grid(grid)
    out = (C.c_int32 * 4)()
    h = None
    if half is not None:
        kg.half = np.ascontiguousarray(half, np.float64)
        h = _dp(kg.half)
    rc = lib().orc_prior_half(C.byref(g), h, out)
    if rc:
        raise ValueError("orc_prior_half failed")
    return [int(out[a]) for a in range(4)]


def zoom_generic(sched: dict, dims, objective: Callable, init=None) -> dict:
    """Run the ZOOM engine on a Python objective f(i1, i2, i3, i4) -> value,
    or -> (value for CC stages, value for distance stages)."""
    s = schedule_from_dict(sched)
    dims4 = (C.c_int32 * 4)(*[int(x) for x in (list(dims) + [1] * 4)[:4]])
    calls = []

    def cb(_ctx, ip, out):
        i = tuple(ip[a] for a in range(4))
        calls.append(i)
        r = objective(*i)
        a, b = (r, r) if np.isscalar(r) else r
        out[0] = float(a)
        out[1] = float(b)

    f = OBJECTIVE2(cb)
    bi = (C.c_int32 * 4)()
    bvs = (C.c_double * 2)()
    ne = C.c_int32()
    mm = C.c_double()
    ini = None if init is None else (C.c_int32 * 4)(*[int(x) for x in init])
    cap = 4096
    path = (C.c_int32 * (5 * cap))()
    plen = C.c_int32()
    rc = lib().orc_zoom_generic2(C.byref(s), dims4, ini, f, None, bi, bvs,
                                 C.byref(ne), C.byref(mm), path, cap, C.byref(plen))
    if rc:
        raise ValueError("orc_zoom_generic failed")
    moves = [(tuple(path[5 * i + a] for a in range(4)), path[5 * i + 4])
             for i in range(plen.value)]
    return dict(idx=tuple(bi[a] for a in range(4)), val=bvs[0], vals=(bvs[0], bvs[1]),
                n_eval=ne.value, min_margin=mm.value, calls=calls, moves=moves)


def zoom(seq, grid, sched: dict, vox, init=None, n_tr=None, threads=0) -> dict:
    """Physics ZOOM per voxel. init: [n_vox, 4] index tuples (neighbour prior)."""
    vox = np.asarray(vox, np.complex128)
    n_vox = vox.shape[0]
    n_tr = vox.shape[1] if n_tr is None else n_tr
    vox = vox[:, :n_tr]
    s, ks = make_seq(seq)
    g, kg = make_grid(grid)
    sc = schedule_from_dict(sched)
    vr = np.ascontiguousarray(vox.real)
    vi = np.ascontiguousarray(vox.imag)
    idx = np.zeros(n_vox, np.int64)
    ccv = np.zeros(n_vox)
    scv = np.zeros(n_vox)
    ns = np.zeros(n_vox, np.int32)
    mm = np.zeros(n_vox)
    ip = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))
    ini = None
    if init is not None:
        ini_arr = np.ascontiguousarray(init, np.int32).reshape(n_vox, 4)
        ini = ip(ini_arr)
    rc = lib().orc_zoom(C.byref(s), C.byref(g), n_tr, C.byref(sc), _dp(vr), _dp(vi), n_vox,
                        ini, idx.ctypes.data_as(C.POINTER(C.c_int64)), _dp(ccv), _dp(scv),
                        ip(ns), _dp(mm), _threads(threads))
    if rc:
        raise ValueError(f"orc_zoom failed ({rc})")
    return dict(idx=idx, cc=ccv, score=scv, n_sim=ns, min_margin=mm)


def nearest_lattice(width: int, height: int, n_slices: int, stride: int) -> np.ndarray:
    """For every voxel (slice-major raster order) the raster index of the
    nearest lattice voxel (x % stride == 0 and y % stride == 0) of the same
    slice: smallest Chebyshev distance, ties to the lowest raster index.
    Lattice voxels map to themselves. Written as the plain search over all
    lattice voxels of the slice."""
    n = width * height * n_slices
    v = np.arange(n)
    x, y, s = v % width, (v // width) % height, v // (width * height)
    lat = np.flatnonzero((x % stride == 0) & (y % stride == 0))
    out = np.empty(n, np.int64)
    for sl in range(n_slices):
        cand = lat[s[lat] == sl]  # ascending raster order
        mine = np.flatnonzero(s == sl)
        d = np.maximum(np.abs(x[mine][:, None] - x[cand][None, :]),
                       np.abs(y[mine][:, None] - y[cand][None, :]))
        out[mine] = cand[np.argmin(d, axis=1)]  # argmin: first (lowest index) minimiser
    return out


def zoom_lattice(seq, grid, sched: dict, vox, width: int, height: int, n_slices: int,
                 stride: int = 4, n_tr=None, threads=0) -> dict:
    """Neighbour prior as a two-pass lattice (Methods, Experiment 3: each
    voxel starts from a neighbour's result within narrowed ranges). Pass 1:
    the lattice voxels, no prior. Pass 2: every other voxel starts at its
    nearest lattice voxel's result with the schedule's prior half-widths."""
    vox = np.asarray(vox, np.complex128)
    near = nearest_lattice(width, height, n_slices, stride)
    lat = near == np.arange(len(near))
    s1 = dict(sched)
    s1["prior_half"] = [-1, -1, -1, -1]  # without a start the ranges are whole anyway
    r1 = zoom(seq, grid, s1, vox[lat], n_tr=n_tr, threads=threads)
    out = {k: np.empty(len(near), dtype=v.dtype) for k, v in r1.items()}
    for k, v in r1.items():
        out[k][lat] = v
    rest = np.flatnonzero(~lat)
    init = np.stack(grid.unravel(out["idx"][near[rest]]), axis=1).astype(np.int32)
    r2 = zoom(seq, grid, sched, vox[rest], init=init, n_tr=n_tr, threads=threads)
    for k, v in r2.items():
        out[k][rest] = v
    out["lattice"] = lat
    out["prior_voxel"] = near
    return out
