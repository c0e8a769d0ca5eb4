"""Seeded voxel subsets of the 64x64 slice workload (N = 1000, 391 x 399 x 81
grid) whose oracle brute-force results are stored in
tests/golden/slice64_bruteforce_oracle.json.

Three subsets, all built from the oracle simulator and the seeded measurement
model only:

* ``noisy``: 64 voxels of the phantom drawn with PCG64(2024), exactly the
  fingerprints the full-slice tests hand to the GPU (SNR 30, unit PD, random
  global phase);
* ``on_grid``: 16 noise-free fingerprints whose truths are the grid values
  nearest to 16 phantom voxels (PCG64(2025)), scaled by the voxel's global
  phase. Experiment 2's fingerprints are on-grid and noise-free: brute force
  must return the truth entry with CC = 1, and the margin to the runner-up is
  what a 1 ms-scale grid leaves (on this 10 ms / 5 ms / 1 Hz grid every such
  margin is below 1e-5, so none of these is pinned);
* ``short``: 16 noise-free fingerprints at grid points drawn uniformly
  (PCG64(2026)) from the short-relaxation corner T1 in [100, 500] ms, T2 in
  [10, 60] ms (any df), with random global phases. There neighbouring
  entries differ by more than 1e-5 in CC, so the index bar applies.
"""
from __future__ import annotations

import hashlib

import numpy as np

NOISY_SEED, NOISY_COUNT = 2024, 64
ONGRID_SEED, ONGRID_COUNT = 2025, 16
SHORT_SEED, SHORT_COUNT = 2026, 16
SHORT_T1_MS, SHORT_T2_MS = (100.0, 500.0), (10.0, 60.0)


def noisy_voxels(n_vox: int = 4096) -> np.ndarray:
    return np.sort(np.random.default_rng(NOISY_SEED).choice(n_vox, NOISY_COUNT, replace=False))


def ongrid_truths(w) -> tuple:
    """(voxels, truth grid indices) of the on-grid subset."""
    ph, grid = w.phantom, w.grid
    vox = np.sort(np.random.default_rng(ONGRID_SEED).choice(ph.n_vox, ONGRID_COUNT,
                                                            replace=False))
    i1 = np.array([int(np.argmin(np.abs(grid.t1_ms - ph.t1[v]))) for v in vox])
    i2 = np.array([int(np.argmin(np.abs(grid.t2_ms - ph.t2[v]))) for v in vox])
    i3 = np.array([int(np.argmin(np.abs(grid.df_hz - ph.df[v]))) for v in vox])
    return vox, grid.ravel(i1, i2, i3)


def short_truths(w) -> tuple:
    """(truth grid indices, global phases) of the short-relaxation subset."""
    g = w.grid
    rng = np.random.default_rng(SHORT_SEED)
    i1 = np.flatnonzero((g.t1_ms >= SHORT_T1_MS[0]) & (g.t1_ms <= SHORT_T1_MS[1]))
    i2 = np.flatnonzero((g.t2_ms >= SHORT_T2_MS[0]) & (g.t2_ms <= SHORT_T2_MS[1]))
    a = rng.choice(i1, SHORT_COUNT)
    b = rng.choice(i2, SHORT_COUNT)
    c = rng.integers(0, len(g.df_hz), SHORT_COUNT)
    phase = rng.uniform(0.0, 2 * np.pi, SHORT_COUNT)
    return g.ravel(a, b, c), phase


def fingerprints(orc, w):
    """complex64 [96, N]: the 64 noisy fingerprints, the 16 on-grid ones and
    the 16 short-relaxation ones; and the truth indices of the last 32."""
    from tests.gpu_common import oracle_fingerprints
    noisy = oracle_fingerprints(orc, w.seq, w.phantom, voxels=noisy_voxels(w.phantom.n_vox))
    vox, truth = ongrid_truths(w)
    clean = np.stack([orc.simulate(w.seq, *map(float, w.grid.values(int(k)))) for k in truth])
    ong = (np.exp(1j * w.phantom.phase[vox])[:, None] * clean).astype(np.complex64)
    st, sph = short_truths(w)
    clean = np.stack([orc.simulate(w.seq, *map(float, w.grid.values(int(k)))) for k in st])
    short = (np.exp(1j * sph)[:, None] * clean).astype(np.complex64)
    return np.concatenate([noisy, ong, short]), np.concatenate([truth, st])


def digest(V: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(V, np.complex64).tobytes()).hexdigest()
