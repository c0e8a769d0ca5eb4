"""GPU parity of dictionary generation (K0 tables + K1) against the FP64 oracle.

Tolerance: entries are compared after dividing each by its own norm; the
L2 distance between the GPU's and the oracle's unit-norm entry bounds the CC
error the dictionary can cause (Cauchy-Schwarz), and must stay below 5e-6 so
that, with the GEMM's own rounding, |CC| stays within 1e-5.
"""
import math

import numpy as np
import pytest

from paper_1506_05393_amd import inputs as I
from tests.gpu_common import need_gpu, to_dev, torch

pytestmark = pytest.mark.gpu

UNIT_L2_TOL = 5e-6


@pytest.fixture(scope="module")
def ctx():
    need_gpu()
    from paper_1506_05393_amd import api
    return api.Context(0)


def _gpu_entries(d, count):
    if d.dtype == "f32":
        re = d.re[:, :count].double().cpu().numpy()
        im = d.im[:, :count].double().cpu().numpy()
        return (re + 1j * im).T
    raw = d.re[:, :count].contiguous().view(torch.bfloat16).float().double().cpu().numpy()
    # [n_tr/4, count, 4, 2] -> [count, n_tr]
    z = raw[..., 0] + 1j * raw[..., 1]
    return z.transpose(1, 0, 2).reshape(count, -1)


def _unit(x):
    n = np.linalg.norm(x, axis=-1, keepdims=True)
    return x / np.where(n > 0, n, 1)


def _cfg1():
    seq = I.make_sequence(200, 0)
    grid = I.make_grid(I.grid_linspace(100, 2000, 60), I.grid_geomspace(20, 400, 40),
                       I.grid_arange(-40, 40, 4))
    return seq, grid


def test_dictionary_f32_matches_oracle_small_workload(ctx, orc):
    from paper_1506_05393_amd import api
    seq, grid = _cfg1()
    sq = api.Sequence(ctx, seq)
    d = api.simulate_dictionary(ctx, sq, grid, dtype="f32")
    torch.cuda.synchronize()
    gpu = _gpu_entries(d, grid.size)
    ref, nref = orc.simulate_grid(seq, grid, threads=8)
    err = np.linalg.norm(_unit(gpu) - _unit(ref), axis=1)
    print(f"max unit-entry L2 error {err.max():.3e}, max raw abs error "
          f"{np.abs(gpu - ref).max():.3e}")
    assert err.max() < UNIT_L2_TOL
    nrm = d.norm.cpu().numpy()
    assert np.max(np.abs(nrm - nref) / nref) < 5e-6


def test_dictionary_ragged_range_prefix_and_ld(ctx, orc):
    """Entry range not a multiple of the block, ld padding, prefix n_tr, B1 axis."""
    from paper_1506_05393_amd import api
    seq = I.make_sequence(77, 5)
    grid = I.make_grid([300.0, 800.0, 1500.0], [25.0, 60.0, 200.0], I.grid_arange(-30, 30, 3),
                       [0.85, 1.0, 1.15])
    sq = api.Sequence(ctx, seq)
    k0, cnt, n_tr = 37, grid.size - 37 - 11, 53
    d = api.alloc_dictionary(n_tr, cnt, "f32", ld=cnt + 29)
    api.simulate_dictionary(ctx, sq, grid, n_tr=n_tr, entry_begin=k0, entry_count=cnt, out=d)
    torch.cuda.synchronize()
    gpu = _gpu_entries(d, cnt)
    ref, nref = orc.simulate_grid(seq, grid, k0=k0, count=cnt, n_tr=n_tr)
    assert np.linalg.norm(_unit(gpu) - _unit(ref), axis=1).max() < UNIT_L2_TOL


def test_dictionary_bf16_is_rounded_f32(ctx, orc):
    from paper_1506_05393_amd import api
    seq, grid = _cfg1()
    sq = api.Sequence(ctx, seq)
    d = api.simulate_dictionary(ctx, sq, grid, dtype="bf16")
    torch.cuda.synchronize()
    gpu = _gpu_entries(d, grid.size)
    ref, _ = orc.simulate_grid(seq, grid, threads=8)
    # bf16 keeps 8 significant bits: relative error <= 2^-8 per component
    tol = np.abs(ref.real) * 2.0 ** -8 + 1e-6
    assert np.all(np.abs(gpu.real - ref.real) <= tol)
    tol = np.abs(ref.imag) * 2.0 ** -8 + 1e-6
    assert np.all(np.abs(gpu.imag - ref.imag) <= tol)


def test_unit_norm_option(ctx, orc):
    from paper_1506_05393_amd import api
    seq, grid = _cfg1()
    sq = api.Sequence(ctx, seq)
    d = api.simulate_dictionary(ctx, sq, grid, dtype="f32", unit_norm=True)
    torch.cuda.synchronize()
    gpu = _gpu_entries(d, grid.size)
    assert np.max(np.abs(np.linalg.norm(gpu, axis=1) - 1.0)) < 1e-5
    ref, _ = orc.simulate_grid(seq, grid, threads=8)
    assert np.linalg.norm(gpu - _unit(ref), axis=1).max() < UNIT_L2_TOL


def test_signals_at_grid_points_equal_entries_and_oracle(ctx, orc):
    from paper_1506_05393_amd import api
    seq, grid = _cfg1()
    sq = api.Sequence(ctx, seq)
    d = api.simulate_dictionary(ctx, sq, grid, dtype="f32")
    ks = np.array([0, 5, 777, 4321, grid.size - 1])
    params = np.stack([np.array(grid.values(k), dtype=np.float64) for k in ks])
    sig = api.simulate_signals(ctx, sq, to_dev(params)).cpu().numpy()
    ent = _gpu_entries(d, grid.size)[ks].astype(np.complex64)
    assert np.array_equal(sig, ent)  # same factors, same FP32 recursion
    off = np.array([[1234.5, 77.7, 3.3, 1.0], [333.3, 29.1, -17.25, 0.93]])
    sig = api.simulate_signals(ctx, sq, to_dev(off)).cpu().numpy().astype(np.complex128)
    for i, p in enumerate(off):
        ref = orc.simulate(seq, *p)
        assert np.linalg.norm(_unit(sig[i]) - _unit(ref)) < UNIT_L2_TOL


def _general_phase_seq(n, seed):
    """Sequence with arbitrary RF phases (pulses not about the x axis)."""
    base = I.make_sequence(n, seed)
    ph = np.random.default_rng(seed + 1000).uniform(0.0, 360.0, n)
    return I.Sequence(base.fa_deg, ph, base.tr_ms, base.te_ms, 1, 0.0)


@pytest.mark.parametrize("n3,b1", [(150, None), (150, [0.9, 1.1]), (21, None), (21, [0.8, 1.0, 1.2])])
def test_dictionary_general_phases_both_df_paths(ctx, orc, n3, b1):
    """General pulse matrices (uniform and per-lane), df axis staged through LDS
    (21 values) and read directly (150), a readout count that is not a multiple
    of the staging chunk; FP32, BF16 and unit-norm outputs; signals at grid
    points equal the entries bit for bit."""
    from paper_1506_05393_amd import api
    seq = _general_phase_seq(62, 7)
    axes = [[300.0, 700.0, 1500.0, 2500.0], [30.0, 80.0, 250.0], I.grid_linspace(-60, 60, n3)]
    grid = I.make_grid(*axes, b1) if b1 else I.make_grid(*axes)
    sq = api.Sequence(ctx, seq)
    d = api.simulate_dictionary(ctx, sq, grid, dtype="f32")
    u = api.simulate_dictionary(ctx, sq, grid, dtype="f32", unit_norm=True)
    d16 = api.simulate_dictionary(ctx, sq, grid, n_tr=60, dtype="bf16")
    torch.cuda.synchronize()
    gpu = _gpu_entries(d, grid.size)
    ref, nref = orc.simulate_grid(seq, grid, threads=8)
    assert np.linalg.norm(_unit(gpu) - _unit(ref), axis=1).max() < UNIT_L2_TOL
    assert np.max(np.abs(d.norm.cpu().numpy() - nref) / nref) < 5e-6
    gu = _gpu_entries(u, grid.size)
    assert np.linalg.norm(gu - _unit(ref), axis=1).max() < UNIT_L2_TOL
    g16 = _gpu_entries(d16, grid.size)
    r60 = ref[:, :60]
    assert np.all(np.abs(g16.real - r60.real) <= np.abs(r60.real) * 2.0 ** -8 + 1e-6)
    assert np.all(np.abs(g16.imag - r60.imag) <= np.abs(r60.imag) * 2.0 ** -8 + 1e-6)
    # the BF16 norm is the norm of the stored values
    assert np.allclose(d16.norm.cpu().numpy(), np.linalg.norm(g16, axis=1), rtol=1e-6)
    ks = np.array([0, 1, grid.size // 2, grid.size - 1])
    params = np.stack([np.array(grid.values(k), dtype=np.float64) for k in ks])
    sig = api.simulate_signals(ctx, sq, to_dev(params)).cpu().numpy()
    assert np.array_equal(sig, gpu[ks].astype(np.complex64))


def test_closed_forms_on_gpu(ctx):
    """Flip angle zero gives no signal; first sample closed form; bSSFP steady state."""
    from paper_1506_05393_amd import api
    seq = I.make_sequence(16, 3)
    seq.fa_deg[:] = 0.0
    sq = api.Sequence(ctx, seq)
    s = api.simulate_signals(ctx, sq, to_dev(np.array([[800.0, 60.0, 5.0, 1.0]]))).cpu().numpy()
    assert np.max(np.abs(s)) == 0.0
    seq = I.make_sequence(8, 3)
    sq = api.Sequence(ctx, seq)
    t1, t2, df = 700.0, 80.0, 12.0
    s = api.simulate_signals(ctx, sq, to_dev(np.array([[t1, t2, df, 1.0]]))).cpu().numpy()[0]
    te = seq.te_ms[0]
    want = (1j * -1.0 * math.sin(math.radians(seq.fa_deg[0])) * math.exp(-te / t2)
            * np.exp(1j * 2 * math.pi * df * te / 1000.0))
    assert abs(s[0] - want) < 1e-6
    n, alpha, tr, t1, t2 = 1200, 50.0, 10.0, 600.0, 60.0
    ph = np.where(np.arange(n) % 2 == 0, 0.0, 180.0)
    seq = I.Sequence(np.full(n, alpha), ph, np.full(n, tr), np.full(n, tr / 2), 1, 0.0)
    sq = api.Sequence(ctx, seq)
    s = api.simulate_signals(ctx, sq, to_dev(np.array([[t1, t2, 0.0, 1.0]]))).cpu().numpy()[0]
    e1, e2, a = math.exp(-tr / t1), math.exp(-tr / t2), math.radians(alpha)
    want = math.sin(a) * (1 - e1) * math.sqrt(e2) / (1 - (e1 - e2) * math.cos(a) - e1 * e2)
    assert abs(abs(s[-1]) - want) < 2e-6


def test_invalid_arguments_are_rejected(ctx):
    from paper_1506_05393_amd import api, _lib
    seq, grid = _cfg1()
    sq = api.Sequence(ctx, seq)
    with pytest.raises(_lib.MRFError, match="n_tr"):
        api.simulate_dictionary(ctx, sq, grid, n_tr=201)
    with pytest.raises(_lib.MRFError, match="n_tr % 4"):
        api.simulate_dictionary(ctx, sq, grid, n_tr=198, dtype="bf16",
                                out=api.alloc_dictionary(200, grid.size, "bf16"))
    bad = I.Sequence(seq.fa_deg, seq.phase_deg, seq.tr_ms, seq.tr_ms.copy(), 1, 0.0)
    with pytest.raises(_lib.MRFError, match="te"):
        api.Sequence(ctx, bad)
    with pytest.raises(_lib.MRFError, match="entry range"):
        api.simulate_dictionary(ctx, sq, grid, entry_begin=grid.size - 10, entry_count=20,
                                out=api.alloc_dictionary(200, 20, "f32"))


def test_full_size_dictionary_sampled(ctx, orc):
    """12,636,729 entries x N = 1000 FP32 (101 GB resident), sampled entries
    checked one by one against the oracle."""
    from paper_1506_05393_amd import api, workloads
    w = workloads.slice64()
    sq = api.Sequence(ctx, w.seq)
    d = api.simulate_dictionary(ctx, sq, w.grid, dtype="f32")
    torch.cuda.synchronize()
    rng = np.random.default_rng(17)
    ks = np.concatenate([[0, w.grid.size - 1], rng.integers(0, w.grid.size, 300)])
    kt = torch.from_numpy(ks).cuda()
    re = d.re.index_select(1, kt).double().cpu().numpy().T
    im = d.im.index_select(1, kt).double().cpu().numpy().T
    gpu = re + 1j * im
    nrm = d.norm.index_select(0, kt).cpu().numpy()
    for i, k in enumerate(ks):
        ref = orc.simulate(w.seq, *map(float, w.grid.values(k)))
        assert np.linalg.norm(_unit(gpu[i]) - _unit(ref)) < UNIT_L2_TOL
        assert abs(nrm[i] - np.linalg.norm(ref)) < 5e-6 * np.linalg.norm(ref)
    del d
    torch.cuda.empty_cache()


@pytest.mark.parametrize("case", ["x_axis", "general_b1_df150", "x_axis_b1_smooth"])
def test_dictionary_pair_equals_both_dictionaries(ctx, case):
    """One pass writing the FP32 planes and the BF16 blocks gives, bit for
    bit, the two dictionaries (and norms) that two separate calls write, over
    a ragged entry range that starts inside the grid."""
    from paper_1506_05393_amd import api
    if case == "x_axis":
        seq = I.make_sequence(64, 5)
        grid = I.make_grid([300.0, 700.0, 1500.0, 2500.0], [30.0, 80.0, 250.0],
                           I.grid_linspace(-60, 60, 41))
    elif case == "general_b1_df150":
        seq = _general_phase_seq(64, 9)
        grid = I.make_grid([300.0, 700.0, 1500.0, 2500.0], [30.0, 80.0, 250.0],
                           I.grid_linspace(-60, 60, 150), [0.9, 1.1])
    else:
        base = I.make_sequence(64, 6)
        seq = I.Sequence(base.fa_deg, base.phase_deg, base.tr_ms, base.te_ms, 1, 0.0, smooth=5)
        grid = I.make_grid([300.0, 700.0, 1500.0, 2500.0], [30.0, 80.0, 250.0],
                           I.grid_linspace(-60, 60, 21), [0.8, 1.0, 1.2])
    sq = api.Sequence(ctx, seq)
    b = 7
    count = grid.size - b - 3  # a ragged block at both ends
    d32, d16 = api.simulate_dictionary_pair(ctx, sq, grid, entry_begin=b, entry_count=count)
    s32 = api.simulate_dictionary(ctx, sq, grid, dtype="f32", entry_begin=b, entry_count=count)
    s16 = api.simulate_dictionary(ctx, sq, grid, dtype="bf16", entry_begin=b, entry_count=count)
    torch.cuda.synchronize()
    assert d32.ld == s32.ld and d16.ld == s16.ld
    assert torch.equal(d32.re[:, :count], s32.re[:, :count])
    assert torch.equal(d32.im[:, :count], s32.im[:, :count])
    assert torch.equal(d16.re[:, :count], s16.re[:, :count])
    assert torch.equal(d32.norm, s32.norm) and torch.equal(d16.norm, s16.norm)
