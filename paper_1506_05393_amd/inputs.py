"""Seeded synthetic inputs for MRF dictionary generating and searching.

This module draws random numbers and lays out parameter values; it holds none
of the method's arithmetic (no Bloch simulation, no correlation, no search).
Both the FP64 oracle side and the GPU side take their inputs from here, so the
same seed always means the same sequence, grid, phantom and noise.

What it produces:

* acquisition sequences of the inversion-recovery bSSFP family (Methods,
  Experiment 1 describes the paper's own family; the family used here is a
  fully specified stand-in): flip angle, RF phase, TR and TE per readout;
* parameter grids: one strictly increasing value list per axis
  (T1 ms, T2 ms, df Hz, optional B1 scale);
* phantoms: per-voxel truth parameters, a global complex scale (phase and
  magnitude; the proton-density scale of the Theory section) and complex
  white noise (Experiment 4 adds white noise to the real and imaginary parts).

The noise is drawn from a counter-based generator (Philox) with a fixed stride
per voxel, so voxel v's noise can be reproduced without drawing the others.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

__all__ = [
    "Sequence", "Grid", "Phantom",
    "make_sequence", "make_grid", "grid_linspace", "grid_arange",
    "grid_geomspace", "phantom_quadrants", "phantom_smooth", "phantom_volume",
    "noise_for_voxels", "compose_fingerprints", "nearest_index",
]


@dataclasses.dataclass
class Sequence:
    """One readout per TR. Angles in degrees, times in ms (all float64)."""
    fa_deg: np.ndarray
    phase_deg: np.ndarray
    tr_ms: np.ndarray
    te_ms: np.ndarray
    inversion: int = 1
    ti_ms: float = 0.0
    smooth: int = 0  # dictionary entries smoothed over 3 or 5 readouts (0: none)

    @property
    def n(self) -> int:
        return int(self.fa_deg.shape[0])

    def prefix(self, n: int) -> "Sequence":
        return Sequence(self.fa_deg[:n].copy(), self.phase_deg[:n].copy(),
                        self.tr_ms[:n].copy(), self.te_ms[:n].copy(),
                        self.inversion, self.ti_ms, self.smooth)


@dataclasses.dataclass
class Grid:
    """Cartesian product of per-axis value lists.

    Entry index k = ((i_t1 * n_t2 + i_t2) * n_df + i_df) * max(n_b1, 1) + i_b1.
    An empty b1 axis means B1 = 1 for every entry.
    """
    t1_ms: np.ndarray
    t2_ms: np.ndarray
    df_hz: np.ndarray
    b1: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(0))

    @property
    def shape(self):
        return (len(self.t1_ms), len(self.t2_ms), len(self.df_hz), max(len(self.b1), 1))

    @property
    def size(self) -> int:
        s = self.shape
        return int(s[0]) * int(s[1]) * int(s[2]) * int(s[3])

    def unravel(self, k):
        n1, n2, n3, n4 = self.shape
        k = np.asarray(k, dtype=np.int64)
        i4 = k % n4
        k = k // n4
        i3 = k % n3
        k = k // n3
        i2 = k % n2
        i1 = k // n2
        return i1, i2, i3, i4

    def ravel(self, i1, i2, i3, i4=0):
        n1, n2, n3, n4 = self.shape
        return ((np.asarray(i1, np.int64) * n2 + i2) * n3 + i3) * n4 + i4

    def values(self, k):
        i1, i2, i3, i4 = self.unravel(k)
        b1 = self.b1[i4] if len(self.b1) else np.ones_like(np.asarray(i1, dtype=np.float64))
        return self.t1_ms[i1], self.t2_ms[i2], self.df_hz[i3], b1


def make_sequence(n: int, seed: int) -> Sequence:
    """IR-bSSFP sequence family used by every workload.

    FA_j = 10 + 50*|sin(2*pi*j/250)| + U(0, 5) deg; RF phase alternating
    0/180 deg (0 for even j); TR_j ~ U(10.5, 14) ms; TE_j = TR_j / 2; ideal
    inversion at t = 0 with TI = 0. The jitter and TR use separate child
    streams of PCG64(seed), so the length-n table is the exact prefix of any
    longer one.
    """
    if n <= 0:
        raise ValueError("sequence length must be positive")
    fa_rng, tr_rng = np.random.default_rng(seed).spawn(2)
    j = np.arange(n, dtype=np.float64)
    fa = 10.0 + 50.0 * np.abs(np.sin(2.0 * math.pi * j / 250.0)) + fa_rng.uniform(0.0, 5.0, n)
    phase = np.where(np.arange(n) % 2 == 0, 0.0, 180.0)
    tr = tr_rng.uniform(10.5, 14.0, n)
    te = tr / 2.0
    return Sequence(fa.astype(np.float64), phase.astype(np.float64), tr, te, 1, 0.0)


def _perlin_1d(n: int, spacing: float, rng) -> np.ndarray:
    """1-D gradient (Perlin) noise at x = 0 .. n-1: random gradients in
    [-1, 1] on lattice points `spacing` apart, blended with the quintic fade
    6t^5 - 15t^4 + 10t^3."""
    x = np.arange(n, dtype=np.float64) / spacing
    k = np.floor(x).astype(np.int64)
    t = x - k
    g = rng.uniform(-1.0, 1.0, int(k.max()) + 2)
    fade = t * t * t * (t * (t * 6.0 - 15.0) + 10.0)
    return (1.0 - fade) * g[k] * t + fade * g[k + 1] * (t - 1.0)


def make_sequence_exp1(n: int = 500, seed: int = 0) -> Sequence:
    """IR-bSSFP sequence after the description of Experiment 1: flip angles
    in 0-79 deg from 1-D Perlin noise (lattice spacing 25 readouts, remapped
    to span 0..79), RF phases cycling 0, 90, 180, 90 deg, TR = 14 ms plus
    Gaussian noise remapped to span 0..6 ms; TE = TR / 2 (not stated there),
    ideal inversion, TI = 0."""
    if n <= 0:
        raise ValueError("sequence length must be positive")
    fa_rng, tr_rng = np.random.default_rng(seed).spawn(2)
    p = _perlin_1d(n, 25.0, fa_rng)
    fa = 79.0 * (p - p.min()) / max(float(np.ptp(p)), 1e-300)
    phase = np.array([0.0, 90.0, 180.0, 90.0])[np.arange(n) % 4]
    g = tr_rng.normal(size=n)
    tr = 14.0 + 6.0 * (g - g.min()) / max(float(np.ptp(g)), 1e-300)
    return Sequence(fa, phase, tr, tr / 2.0, 1, 0.0)


def grid_halfopen(lo: float, hi: float, step: float) -> np.ndarray:
    """lo, lo + step, ... below hi (hi excluded)."""
    n = int(math.ceil((hi - lo) / step - 1e-9))
    return lo + step * np.arange(n, dtype=np.float64)


def grid_linspace(lo: float, hi: float, n: int) -> np.ndarray:
    return np.linspace(lo, hi, n, dtype=np.float64)


def grid_arange(lo: float, hi: float, step: float) -> np.ndarray:
    """Closed range lo..hi with the given step (hi included when on the lattice)."""
    n = int(math.floor((hi - lo) / step + 1e-9)) + 1
    return lo + step * np.arange(n, dtype=np.float64)


def grid_geomspace(lo: float, hi: float, n: int) -> np.ndarray:
    return np.geomspace(lo, hi, n, dtype=np.float64)


def make_grid(t1, t2, df, b1=None) -> Grid:
    g = Grid(np.asarray(t1, np.float64), np.asarray(t2, np.float64),
             np.asarray(df, np.float64),
             np.zeros(0) if b1 is None else np.asarray(b1, np.float64))
    for name, ax in (("t1", g.t1_ms), ("t2", g.t2_ms), ("df", g.df_hz), ("b1", g.b1)):
        if name != "b1" and len(ax) == 0:
            raise ValueError(f"axis {name} is empty")
        if len(ax) > 1 and not np.all(np.diff(ax) > 0):
            raise ValueError(f"axis {name} must be strictly increasing")
    return g


def nearest_index(axis: np.ndarray, value: float) -> int:
    """Index of the grid value nearest to `value` (ties go to the lower index)."""
    d = np.abs(np.asarray(axis) - value)
    return int(np.argmin(d))


@dataclasses.dataclass
class Phantom:
    """Per-voxel truths and measurement model draws (voxel-major, raster order).

    t1/t2/df/b1: truth parameter values; truth_idx: the on-grid truth entry
    index or -1 when the truths are off the grid. phase/mag: global complex
    scale per voxel; snr: the white noise level is rms_j|s_j| / snr per voxel.
    noise_key: Philox key for `noise_for_voxels`.
    """
    shape: tuple
    t1: np.ndarray
    t2: np.ndarray
    df: np.ndarray
    b1: np.ndarray
    truth_idx: np.ndarray
    phase: np.ndarray
    mag: np.ndarray
    snr: float
    noise_key: int

    @property
    def n_vox(self) -> int:
        return int(self.t1.shape[0])


def _scale(rng, n):
    phase = rng.uniform(0.0, 2.0 * math.pi, n)
    mag = rng.uniform(0.5, 2.0, n)
    return phase, mag


def _interp_axis(axis: np.ndarray, fidx: np.ndarray) -> np.ndarray:
    """Axis value at a fractional index (linear between neighbouring values)."""
    return np.interp(fidx, np.arange(len(axis), dtype=np.float64), axis)


def phantom_quadrants(grid: Grid, side: int, seed: int, snr: float,
                      on_grid: bool = True) -> Phantom:
    """side x side phantom of 4 tissue classes, one per quadrant.

    Each class draws a centre index uniformly on each axis; each voxel adds a
    uniform jitter of up to +-2 index steps (integer when on_grid, continuous
    otherwise), clipped to the axis. On-grid truths are integer multiples of
    the resolution, as in Experiment 2.
    """
    rng = np.random.default_rng(seed)
    n1, n2, n3, _ = grid.shape
    nv = side * side
    centres = np.stack([rng.integers(0, n, 4) for n in (n1, n2, n3)], axis=1)
    yy, xx = np.divmod(np.arange(nv), side)
    cls = (yy >= side // 2).astype(int) * 2 + (xx >= side // 2).astype(int)
    fidx = np.empty((nv, 3))
    for a, n in enumerate((n1, n2, n3)):
        if on_grid:
            jit = rng.integers(-2, 3, nv).astype(np.float64)
        else:
            jit = rng.uniform(-2.0, 2.0, nv)
        fidx[:, a] = np.clip(centres[cls, a] + jit, 0, n - 1)
    phase, mag = _scale(rng, nv)
    if on_grid:
        ii = fidx.astype(np.int64)
        t1 = grid.t1_ms[ii[:, 0]]
        t2 = grid.t2_ms[ii[:, 1]]
        df = grid.df_hz[ii[:, 2]]
        truth = grid.ravel(ii[:, 0], ii[:, 1], ii[:, 2])
    else:
        t1 = _interp_axis(grid.t1_ms, fidx[:, 0])
        t2 = _interp_axis(grid.t2_ms, fidx[:, 1])
        df = _interp_axis(grid.df_hz, fidx[:, 2])
        truth = np.full(nv, -1, np.int64)
    return Phantom((side, side), t1, t2, df, np.ones(nv), truth, phase, mag,
                   float(snr), int(seed))


def _smooth_map(rng, side: int, lo: float, hi: float) -> np.ndarray:
    """Sum of 3 random 2-D Gaussians plus a linear ramp, rescaled to [lo, hi]."""
    c = (np.arange(side) + 0.5) / side
    y, x = np.meshgrid(c, c, indexing="ij")
    f = np.zeros((side, side))
    for _ in range(3):
        cx, cy = rng.uniform(0.0, 1.0, 2)
        s = rng.uniform(0.15, 0.4)
        a = rng.uniform(0.5, 1.5)
        f += a * np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2.0 * s * s))
    gx, gy = rng.uniform(-0.5, 0.5, 2)
    f += gx * x + gy * y
    f = (f - f.min()) / max(f.max() - f.min(), 1e-12)
    return lo + (hi - lo) * f


def _ellipses(rng, side: int, maps, ranges) -> None:
    """Overlay 3 elliptical regions of constant values (later ones on top)."""
    c = (np.arange(side) + 0.5) / side
    y, x = np.meshgrid(c, c, indexing="ij")
    for _ in range(3):
        cx, cy = rng.uniform(0.25, 0.75, 2)
        ax, ay = rng.uniform(0.08, 0.25, 2)
        th = rng.uniform(0.0, math.pi)
        u = (x - cx) * math.cos(th) + (y - cy) * math.sin(th)
        v = -(x - cx) * math.sin(th) + (y - cy) * math.cos(th)
        inside = (u / ax) ** 2 + (v / ay) ** 2 <= 1.0
        for m, (lo, hi) in zip(maps, ranges):
            m[inside] = rng.uniform(lo, hi)


def phantom_smooth(side: int, seed: int, snr: float,
                   t1_range=(300.0, 3500.0), t2_range=(20.0, 1500.0),
                   df_range=(-35.0, 35.0), b1_range=None,
                   unit_pd: bool = True) -> Phantom:
    """side x side phantom: smooth T1/T2/df maps with 3 elliptical tissue
    regions of constant values on top; continuous (off-grid) truths.

    With unit_pd the magnitude is 1 and only the global phase is random. With
    b1_range a smooth quadratic-bowl B1 field spanning that range is added.
    """
    rng = np.random.default_rng(seed)
    ranges = [t1_range, t2_range, df_range]
    maps = [_smooth_map(rng, side, lo, hi) for lo, hi in ranges]
    _ellipses(rng, side, maps, ranges)
    nv = side * side
    phase, mag = _scale(rng, nv)
    if unit_pd:
        mag = np.ones(nv)
    if b1_range is not None:
        c = (np.arange(side) + 0.5) / side
        y, x = np.meshgrid(c, c, indexing="ij")
        cx, cy = rng.uniform(0.35, 0.65, 2)
        r2 = (x - cx) ** 2 + (y - cy) ** 2
        r2 = r2 / r2.max()
        b1 = (b1_range[0] + (b1_range[1] - b1_range[0]) * r2).reshape(-1)
    else:
        b1 = np.ones(nv)
    return Phantom((side, side), maps[0].reshape(-1), maps[1].reshape(-1),
                   maps[2].reshape(-1), b1, np.full(nv, -1, np.int64), phase,
                   mag, float(snr), int(seed))


def phantom_volume(n_slices: int, side: int, seed: int, snr: float,
                   t1_range=(300.0, 3500.0), t2_range=(20.0, 1500.0),
                   df_range=(-50.0, 50.0), b1_range=(0.75, 1.25)) -> Phantom:
    """A stack of smooth slices (slice s uses seed + s), voxels slice-major."""
    parts = [phantom_smooth(side, seed + s, snr, t1_range, t2_range, df_range,
                            b1_range) for s in range(n_slices)]
    cat = lambda f: np.concatenate([getattr(p, f) for p in parts])
    return Phantom((n_slices, side, side), cat("t1"), cat("t2"), cat("df"),
                   cat("b1"), cat("truth_idx"), cat("phase"), cat("mag"),
                   float(snr), int(seed))


def _noise_stride(n: int) -> int:
    """Uniform draws reserved per voxel: 2n rounded up to a Philox block (4)."""
    return 4 * ((2 * n + 3) // 4)


def noise_for_voxels(key: int, n: int, voxels) -> np.ndarray:
    """Standard complex Gaussian noise, shape [len(voxels), n], complex128.

    Real and imaginary parts are each N(0, 1/2) (Box-Muller on Philox(key)
    uniforms). Voxel v always uses the uniforms at offset v * stride, so any
    subset is reproduced exactly.
    """
    voxels = np.asarray(voxels, dtype=np.int64).reshape(-1)
    stride = _noise_stride(n)
    out = np.empty((len(voxels), n), np.complex128)
    # contiguous runs share one generator
    i = 0
    while i < len(voxels):
        j = i + 1
        while j < len(voxels) and voxels[j] == voxels[j - 1] + 1:
            j += 1
        bg = np.random.Philox(key=key)
        bg.advance(int(voxels[i]) * stride // 4)
        u = np.random.Generator(bg).random((j - i) * stride).reshape(j - i, stride)
        u1 = 1.0 - u[:, 0:2 * n:2]          # (0, 1]
        u2 = u[:, 1:2 * n:2]
        r = np.sqrt(-np.log(u1))
        out[i:j] = r * np.cos(2.0 * math.pi * u2) + 1j * r * np.sin(2.0 * math.pi * u2)
        i = j
    return out


def compose_fingerprints(clean: np.ndarray, ph: Phantom, voxels=None,
                         noise: bool = True) -> np.ndarray:
    """Measurement model: v = mag * exp(i*phase) * s + sigma * z.

    clean: [nv, n] noise-free signals of the chosen voxels (any simulator),
    sigma = mag * rms_j |s_j| / snr, z from `noise_for_voxels`. Returns
    complex128 [nv, n].
    """
    clean = np.asarray(clean)
    nvx, n = clean.shape
    if voxels is None:
        voxels = np.arange(nvx)
    voxels = np.asarray(voxels, np.int64)
    scale = (ph.mag[voxels] * np.exp(1j * ph.phase[voxels]))[:, None]
    out = scale * clean.astype(np.complex128)
    if noise and np.isfinite(ph.snr) and ph.snr > 0:
        rms = np.sqrt(np.mean(np.abs(clean.astype(np.complex128)) ** 2, axis=1))
        sigma = ph.mag[voxels] * rms / ph.snr
        out = out + sigma[:, None] * noise_for_voxels(ph.noise_key, n, voxels)
    return out
