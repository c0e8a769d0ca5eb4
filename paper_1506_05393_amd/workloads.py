"""The benchmark workloads: sequence, grid and phantom of each, by name.

Every workload is seeded and synthetic. The paper's Experiment 3 maps come
from a structural brain image that is not available; the smooth phantoms with
elliptical tissue regions stand in for those 64x64 slices.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import inputs as I


@dataclasses.dataclass
class Workload:
    name: str
    seq: I.Sequence
    grid: I.Grid
    phantom: I.Phantom
    n_tr: int
    note: str = ""


def small_dgs(on_grid: bool = True) -> Workload:
    """16x16 phantom of 4 tissue classes, N = 200, 60 x 40 x 21 = 50,400 entries,
    SNR 20 (plain DGS: brute force and ZOOM on the same data)."""
    seq = I.make_sequence(200, 0)
    grid = I.make_grid(I.grid_linspace(100, 2000, 60), I.grid_geomspace(20, 400, 40),
                       I.grid_arange(-40, 40, 4))
    ph = I.phantom_quadrants(grid, 16, 100, snr=20.0, on_grid=on_grid)
    return Workload("dgs16x16_N200_E50400", seq, grid, ph, 200)


def slice64() -> Workload:
    """64x64 smooth phantom, N = 1000, 391 x 399 x 81 = 12,636,729 entries, SNR 30."""
    seq = I.make_sequence(1000, 1)
    grid = I.make_grid(I.grid_arange(100, 4000, 10), I.grid_arange(10, 2000, 5),
                       I.grid_arange(-40, 40, 1))
    ph = I.phantom_smooth(64, 101, snr=30.0)
    return Workload("slice64x64_N1000_E12636729", seq, grid, ph, 1000)


def slice64_small_grid(n1: int = 60, n2: int = 60, n3: int = 81) -> Workload:
    """The 64x64 slice against a coarser grid spanning the same ranges (tests)."""
    w = slice64()
    grid = I.make_grid(I.grid_linspace(100, 4000, n1), I.grid_linspace(10, 2000, n2),
                       I.grid_linspace(-40, 40, n3))
    return Workload(f"slice64x64_N1000_E{grid.size}", w.seq, grid, w.phantom, 1000)


def volume(n_slices: int = 8, side: int = 256) -> Workload:
    """8 slices of 256x256, N = 1000, 4 parameters incl. B1 (ZOOM only; the
    3901 x 1991 x 241 x 121 grid is never materialised)."""
    seq = I.make_sequence(1000, 300)
    grid = I.make_grid(I.grid_arange(100, 4000, 1), I.grid_arange(10, 2000, 1),
                       I.grid_arange(-60, 60, 0.5), I.grid_arange(0.7, 1.3, 0.005))
    ph = I.phantom_volume(n_slices, side, 300, snr=25.0)
    return Workload(f"volume{n_slices}x{side}x{side}_N1000_B1", seq, grid, ph, 1000)


def exp3_slice(n_tr: int = 500) -> Workload:
    """Experiment 3's searching ranges at its finest resolution: T1 800-3200 ms
    and T2 50-600 ms at 1 ms, df -48-84 Hz at 1 Hz (the paper's half-open
    ranges; 2401 x 551 x 133 = 175,952,483 entries, never stored), N = 500
    readouts of the sequence family (seed 1). 64x64 smooth phantom (seed 103)
    whose truths are rounded onto that grid; noise-free, unit PD and zero
    phase, as the paper's synthetic fingerprints (ZOOM only)."""
    seq = I.make_sequence(n_tr, 1)
    grid = I.make_grid(I.grid_halfopen(800, 3201, 1), I.grid_halfopen(50, 601, 1),
                       I.grid_halfopen(-48, 85, 1))
    ph = I.phantom_smooth(64, 103, snr=float("inf"), t1_range=(800.0, 3200.0),
                          t2_range=(50.0, 600.0), df_range=(-48.0, 84.0))
    i1 = np.clip(np.rint(ph.t1 - 800.0), 0, len(grid.t1_ms) - 1).astype(np.int64)
    i2 = np.clip(np.rint(ph.t2 - 50.0), 0, len(grid.t2_ms) - 1).astype(np.int64)
    i3 = np.clip(np.rint(ph.df + 48.0), 0, len(grid.df_hz) - 1).astype(np.int64)
    nv = ph.n_vox
    on = I.Phantom(ph.shape, grid.t1_ms[i1], grid.t2_ms[i2], grid.df_hz[i3], np.ones(nv),
                   grid.ravel(i1, i2, i3), np.zeros(nv), np.ones(nv), float("inf"),
                   ph.noise_key)
    return Workload(f"exp3_slice64x64_N{n_tr}_E{grid.size}", seq, grid, on, n_tr)


def exp1_ccmap():
    """CC mapping after Experiment 1: T1 100-5500 ms and T2 50-1200 ms at
    10 ms, df -300-300 Hz at 1 Hz (half-open ranges: 540 x 115 x 600 =
    37,260,000 entries), N = 500, one noise-free fingerprint at T1/T2/df =
    1400 ms / 500 ms / 100 Hz. Returns (name, sequence, grid, truth params,
    truth grid indices)."""
    seq = I.make_sequence_exp1(500, 7)
    grid = I.make_grid(I.grid_halfopen(100, 5500, 10), I.grid_halfopen(50, 1200, 10),
                       I.grid_halfopen(-300, 300, 1))
    truth = (1400.0, 500.0, 100.0)
    idx = (int(np.searchsorted(grid.t1_ms, truth[0])), int(np.searchsorted(grid.t2_ms, truth[1])),
           int(np.searchsorted(grid.df_hz, truth[2])))
    return "exp1_ccmap_E37260000_N500", seq, grid, truth, idx


def serving_grid() -> I.Grid:
    """Resident serving dictionaries: 196 x 200 x 41 = 1,607,200 entries."""
    return I.make_grid(I.grid_arange(100, 4000, 20), I.grid_arange(10, 2000, 10),
                       I.grid_arange(-40, 40, 2))


def phantom_params(ph: I.Phantom) -> np.ndarray:
    """[n_vox, 4] float64 truth parameters (T1, T2, df, B1)."""
    return np.stack([ph.t1, ph.t2, ph.df, ph.b1], axis=1).astype(np.float64)
