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
