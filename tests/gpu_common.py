"""Shared helpers of the GPU parity tests (inputs come from the oracle side)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def oracle_fingerprints(orc, seq, ph, voxels=None, n_tr=None, noise=True):
    """Fingerprints synthesised by the oracle simulator + the measurement model,
    rounded to complex64 (the precision handed to the GPU). Returns the
    complex64 array; the oracle uses exactly these values."""
    from paper_1506_05393_amd import inputs as I
    voxels = np.arange(ph.n_vox) if voxels is None else np.asarray(voxels)
    n_tr = seq.n if n_tr is None else n_tr
    clean = np.stack([orc.simulate(seq, float(ph.t1[v]), float(ph.t2[v]), float(ph.df[v]),
                                   float(ph.b1[v]), n_tr=n_tr) for v in voxels])
    return I.compose_fingerprints(clean, ph, voxels, noise=noise).astype(np.complex64)


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def check_cc_at_index(orc, seq, grid, V, idx, cc, tol, label):
    """Every voxel: the oracle's CC (Eq. 1, FP64) of the entry the GPU
    returned equals the CC the GPU reported, within tol. Returns the oracle
    values."""
    at = orc.cc_at(seq, grid, V, np.asarray(idx, np.int64)[:, None])[:, 0]
    d = np.abs(at - np.asarray(cc, np.float64))
    print(f"{label}: oracle CC at the GPU index vs GPU CC, max |d| {d.max():.2e} "
          f"over {len(d)} voxels")
    assert float(d.max()) < tol, (float(d.max()), int(np.argmax(d)))
    return at


def unit_stencil(grid, idx, axes_steps):
    """Grid indices of the neighbours of each entry along the given
    (axis, step) moves, one column per move; -1 outside the grid."""
    dims = grid.shape
    u = np.stack(grid.unravel(np.asarray(idx, np.int64)), axis=1)
    cols = []
    for move in axes_steps:
        n = u.copy()
        for ax, st in move:
            n[:, ax] += st
        ok = np.all((n >= 0) & (n < np.array(dims)), axis=1)
        cols.append(np.where(ok, grid.ravel(n[:, 0], n[:, 1], n[:, 2], n[:, 3]), -1))
    return np.stack(cols, axis=1)


# the 8 unit neighbours of a 2-D zoom on (T1, T2)
UNIT_T1T2 = [[(0, a), (1, b)] for a in (-1, 0, 1) for b in (-1, 0, 1) if (a, b) != (0, 0)]
