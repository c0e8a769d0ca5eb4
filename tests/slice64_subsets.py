"""Seeded voxel subsets of the 64x64 slice workload (N = 1000, 391 x 399 x 81
grid) whose oracle brute-force results are stored in
tests/golden/slice64_bruteforce_oracle.json.

Two subsets, both built from the oracle simulator and the seeded measurement
model only:

* ``noisy``: 64 voxels of the phantom drawn with PCG64(2024), exactly the
  fingerprints the full-slice tests hand to the GPU (SNR 30, unit PD, random
  global phase);
* ``on_grid``: 16 noise-free fingerprints whose truths are the grid values
  nearest to 16 phantom voxels (PCG64(2025)), scaled by the voxel's global
  phase. Experiment 2's fingerprints are on-grid and noise-free: brute force
  must return the truth entry with CC = 1, and the margin to the runner-up is
  what a 1 ms-scale grid leaves.
"""
from __future__ import annotations

import hashlib

import numpy as np

NOISY_SEED, NOISY_COUNT = 2024, 64
ONGRID_SEED, ONGRID_COUNT = 2025, 16


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


def fingerprints(orc, w):
    """complex64 [80, N]: the 64 noisy fingerprints, then the 16 on-grid ones,
    and the on-grid truth indices."""
    from tests.gpu_common import oracle_fingerprints
    noisy = oracle_fingerprints(orc, w.seq, w.phantom, voxels=noisy_voxels(w.phantom.n_vox))
    vox, truth = ongrid_truths(w)
    clean = np.stack([orc.simulate(w.seq, *map(float, w.grid.values(int(k)))) for k in truth])
    ong = (np.exp(1j * w.phantom.phase[vox])[:, None] * clean).astype(np.complex64)
    return np.concatenate([noisy, ong]), truth


def digest(V: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(V, np.complex64).tobytes()).hexdigest()
