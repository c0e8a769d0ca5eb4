"""Serving scheduler on the host-simulated device (no GPU): admission by
footprint within the budget, first-in first-out order, continuous batching,
rejection, cancellation, injected device failure, draining on destroy.

The fake device runs no kernels and writes no outputs; a batch takes
fake_ns_per_byte x its buffer bytes of wall time."""
import time

import numpy as np
import pytest

from paper_1506_05393_amd import _lib as L
from paper_1506_05393_amd import inputs as I

MB = 1 << 20


def _api():
    from paper_1506_05393_amd import api
    return api


def _grid():
    return I.make_grid(I.grid_linspace(100, 2000, 12), I.grid_geomspace(20, 400, 10),
                       I.grid_arange(-8, 8, 2))


def _server(budget_mb=96, **kw):
    api = _api()
    kw.setdefault("fake_ns_per_byte", 0.05)
    srv = api.Server(None, budget_mb * MB, fake=True, **kw)
    slots = [srv.register(None, _grid(), "bf16", lengths=(500, 1000)) for _ in range(3)]
    return srv, slots


def _trace(n, seed):
    """Seeded request mix: sizes 32^2..128^2 voxels, N in {500, 1000}, both modes."""
    rng = np.random.default_rng(seed)
    sizes = np.array([32, 64, 96, 128]) ** 2
    return [dict(mode=("brute", "zoom")[rng.integers(2)], slot=int(rng.integers(3)),
                 n_tr=int(rng.choice([500, 1000])), n_vox=int(rng.choice(sizes)),
                 gap=float(rng.exponential(0.002))) for _ in range(n)]


def test_budget_fifo_and_batching_under_poisson_load():
    srv, slots = _server(budget_mb=160, n_streams=2, max_inflight=16)
    try:
        tickets, keys = [], []
        for q in _trace(48, 1):
            tickets.append(srv.submit(q["mode"], slots[q["slot"]], q["n_tr"], n_vox=q["n_vox"]))
            keys.append((q["mode"], q["slot"], q["n_tr"]))
            time.sleep(q["gap"])
        srv.wait(tickets, timeout_s=120)
        st = srv.stats()
        polls = [srv.poll(t) for t in tickets]
    finally:
        srv.close()
    assert all(p[0] == "done" for p in polls)
    avail = st["budget_bytes"] - st["resident_bytes"]
    assert 0 < st["peak_reserved_bytes"] <= avail
    assert st["arena_peak_bytes"] <= st["peak_reserved_bytes"]
    assert st["peak_inflight"] <= 16
    assert st["reserved_bytes"] == 0
    assert st["done"] == 48 and st["failed"] == 0
    # continuous batching: some batches held several requests, and batches
    # span readout counts (a batch is keyed by slot and mode only)
    assert st["batches"] < 48 and st["max_batch_requests"] > 1
    assert sum(st["mode_batches"]) == st["batches"]
    assert sum(st["mode_requests"]) == 48 and st["admitted"] == 48
    # first-in first-out within a batch key: a later request never starts first
    keys = [k[:2] for k in keys]
    for k in set(keys):
        starts = [polls[i][2] for i in range(48) if keys[i] == k]
        assert starts == sorted(starts)
    for s, a, b, c in polls:
        assert 0 <= a <= b <= c


def test_strict_fifo_with_one_stream_and_no_batching():
    srv, slots = _server(budget_mb=200, n_streams=1, max_inflight=4, max_batch_vox=1)
    try:
        tickets = [srv.submit(q["mode"], slots[q["slot"]], q["n_tr"], n_vox=q["n_vox"])
                   for q in _trace(20, 2)]
        srv.wait(tickets, timeout_s=60)
        starts = [srv.poll(t)[2] for t in tickets]
        st = srv.stats()
    finally:
        srv.close()
    assert starts == sorted(starts)
    assert st["batches"] == 20


def test_rejects_requests_and_slots_that_can_never_fit():
    api = _api()
    srv = api.Server(None, 8 * MB, fake=True)
    try:
        slot = srv.register(None, _grid(), "bf16", lengths=(1000,))
        with pytest.raises(L.MRFError) as e:
            srv.register(None, I.make_grid(I.grid_linspace(100, 2000, 200),
                                           I.grid_linspace(20, 400, 100), [0.0]), "f32",
                         lengths=(1000,))
        assert e.value.status == 5
        with pytest.raises(L.MRFError) as e:
            srv.submit("brute", slot, 1000, n_vox=128 * 128)  # 128 MB of voxels > 8 MB budget
        assert e.value.status == 5
        t = srv.submit("zoom", slot, 1000, n_vox=64)  # the server keeps serving
        srv.wait([t])
        assert srv.poll(t)[0] == "done"
        assert srv.stats()["rejected"] == 1
    finally:
        srv.close()


def test_invalid_requests_and_registration():
    api = _api()
    srv = api.Server(None, 64 * MB, fake=True)
    try:
        with pytest.raises(L.MRFError, match="multiples of 4"):
            srv.register(None, _grid(), "bf16", lengths=(998,))
        slot = srv.register(None, _grid(), "f32", lengths=(500, 1000))
        with pytest.raises(L.MRFError, match="unknown slot"):
            srv.submit("zoom", slot + 1, 500, n_vox=8)
        with pytest.raises(L.MRFError, match="not a registered length"):
            srv.submit("brute", slot, 700, n_vox=8)
        with pytest.raises(L.MRFError, match="n_tr"):
            srv.submit("zoom", slot, 1001, n_vox=8)
        t = srv.submit("zoom", slot, 700, n_vox=8)  # ZOOM takes any length up to the longest
        z = srv.submit("brute", slot, 500, n_vox=0)  # empty request completes at once
        assert srv.poll(z)[0] == "done"
        with pytest.raises(L.MRFError, match="before the first request"):
            srv.register(None, _grid(), "f32", lengths=(500,))
        with pytest.raises(L.MRFError, match="unknown ticket"):
            srv.poll(10 ** 9)
        srv.wait([t])
    finally:
        srv.close()


def test_cancel_queued_not_running():
    srv, slots = _server(budget_mb=96, n_streams=1, max_inflight=8, fake_ns_per_byte=3.0)
    try:
        t1 = srv.submit("brute", slots[0], 1000, n_vox=64 * 64)   # ~33 MB x 3 ns = ~0.1 s
        t2 = srv.submit("zoom", slots[1], 1000, n_vox=32 * 32)
        t3 = srv.submit("zoom", slots[2], 500, n_vox=32 * 32)
        deadline = time.monotonic() + 10
        while srv.poll(t1)[0] != "running":
            assert time.monotonic() < deadline
            time.sleep(0.0005)
        with pytest.raises(L.MRFError) as e:
            srv.cancel(t1)
        assert e.value.status == 4
        srv.cancel(t2)
        assert srv.poll(t2)[0] == "cancelled"
        srv.wait([t1, t3], timeout_s=30)
        assert srv.poll(t1)[0] == "done" and srv.poll(t3)[0] == "done"
        srv.cancel(t1)  # finished: no-op
        assert srv.poll(t1)[0] == "done"
        st = srv.stats()
        assert st["cancelled"] == 1 and st["done"] == 2 and st["reserved_bytes"] == 0
    finally:
        srv.close()


def test_injected_device_failure_fails_its_batch_and_server_keeps_serving():
    srv, slots = _server(budget_mb=96, n_streams=1, max_batch_vox=1, fake_fail_ticket=3)
    try:
        tickets = [srv.submit("zoom", slots[0], 500, n_vox=256) for _ in range(6)]
        srv.wait(tickets, timeout_s=30)
        states = [srv.poll(t)[0] for t in tickets]
        assert states == ["done", "done", "failed", "done", "done", "done"]
        assert "injected" in srv.failure(tickets[2])
        st = srv.stats()
        assert st["failed"] == 1 and st["done"] == 5 and st["reserved_bytes"] == 0
    finally:
        srv.close()


def test_destroy_drains_inflight_work():
    srv, slots = _server(budget_mb=96, n_streams=1, max_batch_vox=1, fake_ns_per_byte=1.0)
    tickets = [srv.submit("brute", slots[0], 1000, n_vox=32 * 32) for _ in range(5)]
    # each ~8.6 MB batch takes ~8.6 ms of fake device time
    t0 = time.monotonic()
    srv.close()
    assert time.monotonic() - t0 > 0.03
    assert len(tickets) == 5


def test_unknown_ticket_is_an_error():
    """Polling or cancelling a ticket the server never issued fails with
    MRF_ERR_INVALID and names the ticket."""
    srv, slots = _server()
    try:
        t = srv.submit("brute", slots[0], 500, n_vox=64)
        srv.wait([t], timeout_s=60)
        with pytest.raises(L.MRFError, match="unknown ticket"):
            srv.poll(t + 1000)
        with pytest.raises(L.MRFError):
            srv.cancel(t + 1000)
    finally:
        srv.close()


def test_batches_span_readout_counts():
    """Requests of one slot and mode queued behind a busy stream share a
    batch whatever their readout counts (500 and 1000 here), for both modes;
    the reservations (each at the slot's longest count) cover the batch."""
    srv, slots = _server(budget_mb=400, n_streams=1, max_inflight=64, fake_ns_per_byte=0.5)
    try:
        first = srv.submit("brute", slots[0], 1000, n_vox=4096)  # keeps the stream busy
        tickets = [first]
        for mode in ("brute", "zoom"):
            for i in range(6):
                tickets.append(srv.submit(mode, slots[1], (500, 1000)[i % 2], n_vox=1024))
        srv.wait(tickets, timeout_s=120)
        st = srv.stats()
        assert all(srv.poll(t)[0] == "done" for t in tickets)
    finally:
        srv.close()
    assert st["mixed_length_batches"][0] >= 1 and st["mixed_length_batches"][1] >= 1
    assert st["mode_requests"] == [7, 6] and st["batches"] <= 4
    assert st["arena_peak_bytes"] <= st["peak_reserved_bytes"]


def test_batching_window_groups_requests_and_bounds_their_wait():
    """With idle streams, requests arriving 10 ms apart go out one per batch
    without a window; with a 150 ms window they share batches (keyed by slot
    and mode), and no request starts later than its window after submission
    (plus the scheduler's wake-up), unless its batch was full."""
    def run(window):
        srv, slots = _server(budget_mb=400, n_streams=2, max_inflight=64,
                             fake_ns_per_byte=0.0005, batch_window_ms=window)
        try:
            tickets = []
            for i in range(12):
                tickets.append(srv.submit("zoom", slots[0], (500, 1000)[i % 2], n_vox=1024))
                time.sleep(0.010)
            srv.wait(tickets, timeout_s=60)
            polls = [srv.poll(t) for t in tickets]
            st = srv.stats()
        finally:
            srv.close()
        assert all(p[0] == "done" for p in polls)
        return st, polls

    st0, _ = run(0.0)
    st1, polls = run(150.0)
    assert st0["mode_batches"][1] >= 10  # one request per batch (each stream idle)
    assert st1["mode_batches"][1] <= 3 and st1["max_batch_requests"] >= 4
    for _, t_sub, t_start, _ in polls:
        assert t_start - t_sub <= 150.0 + 50.0


def test_batching_window_does_not_hold_a_draining_server():
    """Closing the server launches a waiting batch at once."""
    srv, slots = _server(budget_mb=400, n_streams=1, batch_window_ms=60_000.0)
    t = srv.submit("brute", slots[0], 1000, n_vox=1024)
    t0 = time.perf_counter()
    srv.close()
    assert time.perf_counter() - t0 < 30.0
