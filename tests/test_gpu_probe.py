"""Device peak probes (measurement aids of the benchmark): the MFMA-only loops
really run `iters` rounds of four MFMAs per wave, and the write stream writes
exactly the documented pattern. Values are exact (operands 0.5 and 0.25, or
the varied operands' multiples of 1/8 over few rounds: all partial sums
representable), so the checks are equalities."""
import pytest

from tests.gpu_common import need_gpu, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    need_gpu()
    from paper_1506_05393_amd import api
    return api.Context(0)


@pytest.mark.parametrize("dtype,per_lane,per_mfma", [("f32", 16, 4096), ("bf16", 128, 32768)])
@pytest.mark.parametrize("iters", [1, 7, 1000])
def test_mfma_probe_counts_every_round(ctx, dtype, per_lane, per_mfma, iters):
    from paper_1506_05393_amd import api
    out = torch.full((3 * 256,), -1.0, dtype=torch.float32, device="cuda")
    fl = api.probe_mfma(ctx, dtype, iters, out)
    torch.cuda.synchronize()
    assert torch.equal(out, torch.full_like(out, float(per_lane * iters)))
    # 3 workgroups x 4 waves x 4 MFMAs per round
    assert fl == 3 * 4 * 4 * iters * per_mfma


def varied_lane_sums():
    """Each lane's sum of its accumulators after one round of the varied BF16
    loop, from the v_mfma_f32_32x32x16_bf16 operand layout (lane l: A row
    l % 32 and B column l % 32 at k = 8 (l // 32) + e; C rows
    8 (r // 4) + 4 (l // 32) + r % 4 of column l % 32), in float64."""
    import numpy as np
    lane = np.arange(64)[:, None, None]
    f = np.arange(8)[None, :, None]
    e = np.arange(8)[None, None, :]
    val = 0.375 * ((7 * lane + 13 * f + 29 * e) % 61) - 11.0  # exact in BF16
    sums = np.zeros(64)
    for i in range(4):
        a = np.zeros((32, 16))
        b = np.zeros((16, 32))
        for l in range(64):
            k = 8 * (l // 32) + np.arange(8)
            a[l % 32, k] = val[l, 2 * i]
            b[k, l % 32] = val[l, 2 * i + 1]
        c = a @ b
        for l in range(64):
            rows = [8 * (r // 4) + 4 * (l // 32) + r % 4 for r in range(16)]
            sums[l] += c[rows, l % 32].sum()
    return sums


@pytest.mark.parametrize("iters", [1, 3, 7])
def test_varied_mfma_probe_exact(ctx, iters):
    import numpy as np
    from paper_1506_05393_amd import api
    out = torch.full((2 * 256,), -1.0, dtype=torch.float32, device="cuda")
    fl = api.probe_mfma_varied(ctx, iters, out)
    torch.cuda.synchronize()
    want = np.tile(varied_lane_sums() * iters, 8)
    assert np.array_equal(out.cpu().numpy().astype(np.float64), want)
    assert fl == 2 * 4 * 4 * iters * 32768


@pytest.mark.parametrize("nbytes", [16, 4096 * 16 + 48, (1 << 26) + 16])
def test_write_probe_pattern(ctx, nbytes):
    from paper_1506_05393_amd import api
    buf = torch.zeros(nbytes + 64, dtype=torch.uint8, device="cuda")
    api.probe_write(ctx, buf[:nbytes], pattern=0x0BADF00D)
    torch.cuda.synchronize()
    w = buf[:nbytes].view(torch.int32).view(-1, 4).cpu()
    n = w.shape[0]
    i = torch.arange(n, dtype=torch.int64)
    assert torch.all(w[:, 0] == 0x0BADF00D) and torch.all(w[:, 2] == 0x0BADF00D)
    assert torch.all(w[:, 1].to(torch.int64) == i) and torch.all(w[:, 3].to(torch.int64) == i)
    assert torch.all(buf[nbytes:].cpu() == 0)  # nothing past the end


def test_probe_argument_errors(ctx):
    from paper_1506_05393_amd import api
    with pytest.raises(Exception):
        api.probe_mfma(ctx, "f32", 10, torch.empty(100, dtype=torch.float32, device="cuda"))
    with pytest.raises(Exception):
        api.probe_mfma(ctx, "bf16", 0, torch.empty(256, dtype=torch.float32, device="cuda"))
    with pytest.raises(Exception):
        api.probe_write(ctx, torch.empty(24, dtype=torch.uint8, device="cuda"))
    with pytest.raises(Exception):
        api.probe_mfma_varied(ctx, 0, torch.empty(256, dtype=torch.float32, device="cuda"))
