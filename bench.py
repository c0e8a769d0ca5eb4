"""Benchmark of the MRF dictionary generating and searching hot path on one GPU.

One step = one pass of the whole hot path over one 64x64 slice (N = 1000,
12,636,729-entry grid): FP32 dictionary generation, FP32 brute-force
matching (MFMA GEMM + fused top-k), and the further paths as they exist.
Prints one JSON line (see README/DESIGN for the fields).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
# multi-start ZOOM lattice (T1 starts, T2 starts, outer rounds): the cheapest
# one found to agree with brute force on every pinned voxel of both small
# workloads (searched with the oracle over 1x4 ... 4x4; 4x4 costs twice the
# entries for the same agreement)
MULTISTART = (2, 3, 8)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK = {"fp32_mfma_tflops": 157.3, "bf16_mfma_tflops": 2500.0, "hbm_gbps": 8000.0}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="slice64", choices=["slice64", "small"])
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=20.0,
                   help="target CPU time of the oracle sample")
    p.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    p.add_argument("--no-volume", action="store_true",
                   help="skip the 8 x 256 x 256 four-parameter ZOOM volume")
    p.add_argument("--copy-probe-gb", type=float, default=0.0,
                   help="only run a plain device copy of this size (3 times), the reference "
                        "for scaling HBM byte counters, and exit")
    p.add_argument("--no-ccmap", action="store_true",
                   help="skip the CC map of Experiment 1 and its Property I-III checks")
    p.add_argument("--no-smooth", action="store_true",
                   help="skip the temporal smoothing measurement")
    p.add_argument("--no-zoom-dict", action="store_true",
                   help="skip ZOOM over a resident dictionary")
    p.add_argument("--no-peaks", action="store_true",
                   help="skip the measured device peaks (MFMA-only loops, write and copy streams)")
    p.add_argument("--serve-seconds", type=float, default=60.0,
                   help="length of the serving stream (arrival times)")
    p.add_argument("--serve-requests", type=int, default=0,
                   help="cap on the requests of the serving stream (0: none)")
    p.add_argument("--serve-rate", type=float, default=20.0, help="Poisson arrivals per second")
    p.add_argument("--serve-window-ms", type=float, default=750.0,
                   help="batching window of the second serving run (0: skip it)")
    return p.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_inputs(api, ctx, sq, w, torch):
    """Fingerprints of the phantom: GPU-simulated clean signals, then the
    measurement model (global phase/magnitude, complex white noise)."""
    from paper_1506_05393_amd import inputs as I
    from paper_1506_05393_amd import workloads as W
    params = torch.from_numpy(W.phantom_params(w.phantom)).cuda()
    clean = api.simulate_signals(ctx, sq, params, n_tr=w.n_tr)
    ph = w.phantom
    nv = ph.n_vox
    noise = torch.from_numpy(I.noise_for_voxels(ph.noise_key, w.n_tr, np.arange(nv))
                             .astype(np.complex64)).cuda()
    scale = torch.from_numpy((ph.mag * np.exp(1j * ph.phase)).astype(np.complex64)).cuda()
    rms = clean.abs().pow(2).mean(dim=1).sqrt()
    sigma = torch.from_numpy(ph.mag.astype(np.float32)).cuda() * rms / ph.snr
    return (scale[:, None] * clean + sigma[:, None] * noise).contiguous()


COUNTERS = os.path.join(ROOT, "profiles", "hbm_counters__slice64x64_N1000_E12636729.md")


def counted_traffic(kernel: str, source: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary (copy-calibrated), or None when the kernel's source has
    changed since the counters were taken (or no summary exists)."""
    import hashlib
    try:
        text = open(COUNTERS).read()
    except OSError:
        return None
    now = hashlib.sha256(open(os.path.join(ROOT, "paper_1506_05393_amd", "csrc", source),
                              "rb").read()).hexdigest()
    if f"csrc/{source}: {now}" not in text:
        return None
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip("|").split("|")]
        if len(cells) == 7 and cells[0] == kernel:
            return float(cells[6])
    return None


def volume_bench(api, ctx, torch, n_slices: int = 8, side: int = 256):
    """MRF-ZOOM over 8 slices of 256 x 256 voxels, N = 1000, on the virtual
    3901 x 1991 x 241 x 121 (T1, T2, df, B1) grid: the paper schedule with B1
    stages, without and with the two-pass lattice neighbour prior (Experiment
    3 ranges: +-3000 ms, +-800 ms, +-150 Hz, +-0.3). Fingerprints: GPU-simulated
    phantom truths, random global phase and magnitude, SNR 25 noise."""
    from paper_1506_05393_amd import workloads as W
    w = W.volume(n_slices, side)
    sq = api.Sequence(ctx, w.seq)
    ga = api.GridArg(w.grid)
    ph = w.phantom
    clean = api.simulate_signals(ctx, sq, torch.from_numpy(W.phantom_params(ph)).cuda())
    g = torch.Generator(device="cuda").manual_seed(ph.noise_key)
    noise = torch.randn(clean.shape, dtype=torch.complex64, device="cuda", generator=g)
    scale = torch.from_numpy((ph.mag * np.exp(1j * ph.phase)).astype(np.complex64)).cuda()
    sigma = (clean.abs().pow(2).mean(dim=1).sqrt() * torch.from_numpy(ph.mag.astype(np.float32))
             .cuda() / ph.snr)
    vox = (scale[:, None] * clean + sigma[:, None] * noise).contiguous()
    del clean, noise
    sched = api.schedule_paper(ctx, sq, ga)
    sched_p = dict(sched)
    sched_p["prior_half"] = api.prior_half_widths(ga)
    ws = api.Workspace(ctx.device)
    ev = lambda: torch.cuda.Event(enable_timing=True)
    out = {}
    for name, fn in (("plain", lambda: api.zoom_search(ctx, sq, ga, vox, sched=sched, workspace=ws)),
                     ("lattice", lambda: api.zoom_search_lattice(ctx, sq, ga, vox, side, side,
                                                                 n_slices, sched=sched_p,
                                                                 workspace=ws))):
        a, b = ev(), ev()
        a.record()
        r = fn()
        b.record()
        torch.cuda.synchronize()
        out[name] = (a.elapsed_time(b), r)
        log(f"volume {name}: {out[name][0]:.0f} ms")
    per_slice = []
    nv = side * side
    for s in range(n_slices):
        a, b = ev(), ev()
        a.record()
        api.zoom_search_lattice(ctx, sq, ga, vox[s * nv:(s + 1) * nv], side, side, 1,
                                sched=sched_p, workspace=ws)
        b.record()
        per_slice.append((a, b))
    torch.cuda.synchronize()
    per_slice = [a.elapsed_time(b) for a, b in per_slice]
    n = vox.shape[0]
    res = {"workload": f"{w.name}: {n} voxels, grid {len(w.grid.t1_ms)} x {len(w.grid.t2_ms)} x "
                       f"{len(w.grid.df_hz)} x {len(w.grid.b1)} (never stored)",
           "prior_half_idx": sched_p["prior_half"]}
    for name, (ms, r) in out.items():
        ns = r["n_sim"].cpu().numpy()
        res[name] = {"ms": ms, "voxels_per_s": n / (ms * 1e-3), "n_sim_mean": float(ns.mean()),
                     "n_sim_p50": float(np.percentile(ns, 50)),
                     "n_sim_p99": float(np.percentile(ns, 99)), "n_sim_max": int(ns.max()),
                     "n_sim_hist": np.histogram(ns, bins=[0, 100, 200, 300, 400, 600, 800,
                                                          1200, 1 << 30])[0].tolist()}
    res["lattice_speedup"] = out["plain"][0] / out["lattice"][0]
    res["index_agreement_lattice_vs_plain"] = float(
        (out["plain"][1]["idx"] == out["lattice"][1]["idx"]).double().mean().item())
    res["cc_mean"] = {k: float(v[1]["cc"].double().mean().item()) for k, v in out.items()}
    res["slice_ms_lattice"] = {"p50": float(np.percentile(per_slice, 50)),
                               "p99": float(np.percentile(per_slice, 99))}
    return res


def serve_bench(api, ctx, torch, seconds: float, rate: float, seed: int = 4,
                max_requests: int = 0, window_ms: float = 0.0):
    """Request stream through the server: Poisson arrivals at `rate`/s for
    `seconds` (rate x seconds arrival times, uniform over the span: a Poisson
    process conditioned on its count), with the server's batching window
    `window_ms`, slices of 32^2, 64^2, 96^2 or 128^2 voxels, N in {500, 1000},
    three sequences (seeds 2-4) with resident BF16 dictionaries over a
    1.6M-entry grid, half brute force (BF16 + FP32 re-scoring), half
    MRF-ZOOM (simulated on the fly). Latency = completion observed by the
    server - submission. Returns the summary and, per request type (mode,
    N), a seeded 1% of the distinct voxels it served with their parameters,
    noise draws and served results, for the oracle re-check."""
    from paper_1506_05393_amd import inputs as I
    from paper_1506_05393_amd import workloads as W
    grid = W.serving_grid()
    seqs_h = [I.make_sequence(1000, s) for s in (2, 3, 4)]
    seqs = [api.Sequence(ctx, q) for q in seqs_h]
    sizes = [32, 64, 96, 128]
    rng = np.random.default_rng(seed)
    # voxel pools: in-grid parameters, GPU-simulated signals, SNR 30 noise
    pools, params, noises = {}, {}, {}
    for si, sq in enumerate(seqs):
        for n in sizes:
            nv = n * n
            p = np.stack([rng.uniform(120, 3900, nv), rng.uniform(12, 1900, nv),
                          rng.uniform(-39, 39, nv), np.ones(nv)], axis=1)
            sig = api.simulate_signals(ctx, sq, torch.tensor(p, device="cuda"))
            g = torch.Generator(device="cuda").manual_seed(seed * 1000 + si * 10 + n)
            noise = torch.randn(sig.shape, dtype=torch.complex64, device="cuda", generator=g)
            sigma = sig.abs().pow(2).mean(dim=1, keepdim=True).sqrt() / 30
            pools[(si, n)] = (sig + sigma * noise).contiguous()
            params[(si, n)] = p
            noises[(si, n)] = noise
    resident = 3 * ((grid.size + 255) // 256 * 256 * 250 * 16 + 2 * grid.size * 8)
    budget = resident + 24 * (1 << 30)
    srv = api.Server(ctx, budget, max_inflight=64, n_streams=2, refine_bf16=True,
                     batch_window_ms=window_ms)
    try:
        slots = [srv.register(sq, grid, "bf16", lengths=(500, 1000)) for sq in seqs]
        warm = [srv.submit(m, s, n, pools[(s, 32)]) for m in ("brute", "zoom") for s in slots
                for n in (500, 1000)]
        srv.wait(warm, timeout_s=120)
        st0 = srv.stats()
        n_arr = int(round(rate * seconds))
        if max_requests:
            n_arr = min(n_arr, max_requests)
        times = np.sort(rng.uniform(0.0, seconds, n_arr))
        trace = [(float(t), ("brute", "zoom")[rng.integers(2)], int(rng.integers(3)),
                  int(rng.choice([500, 1000])), int(rng.choice(sizes))) for t in times]
        tickets, meta, rejected = [], [], 0
        t0 = time.perf_counter()
        last_log = t0
        for at, mode, s, n_tr, n in trace:
            d = at - (time.perf_counter() - t0)
            if d > 0:
                time.sleep(d)
            try:
                tickets.append(srv.submit(mode, slots[s], n_tr, pools[(s, n)]))
                meta.append((mode, s, n_tr, n))
            except Exception:
                rejected += 1
            if time.perf_counter() - last_log > 15:
                last_log = time.perf_counter()
                log(f"serving: {len(tickets)} requests submitted")
        srv.wait(tickets, timeout_s=900)
        polls = [srv.poll(tk) for tk in tickets]
        st = srv.stats()
        # per request type, the first served result of every pool it used
        recheck = {}
        rs = np.random.default_rng(seed + 1)
        for i, (mode, s, n_tr, n) in enumerate(meta):
            key = f"{mode}_N{n_tr}"
            pool = recheck.setdefault(key, {"mode": mode, "n_tr": n_tr, "items": {}})["items"]
            if (s, n) in pool or polls[i][0] != "done":
                continue
            nv = n * n
            pick = np.sort(rs.choice(nv, max(1, nv // 100), replace=False))
            r = srv.result(tickets[i])
            pick_t = torch.from_numpy(pick).cuda()
            pool[(s, n)] = {"seq": s, "voxels": pick, "params": params[(s, n)][pick],
                            "noise": noises[(s, n)][pick_t, :n_tr].cpu().numpy(),
                            "idx": r["idx"][pick_t].cpu().numpy(),
                            "cc": r["cc"][pick_t].cpu().numpy()}
    finally:
        srv.close()
    n_req = len(tickets)
    lat = np.array([p[3] - p[1] for p in polls])
    span_s = (max(p[3] for p in polls) - min(p[1] for p in polls)) * 1e-3
    vox = sum(m[3] * m[3] for m in meta)
    by_mode = {m: np.array([lat[i] for i in range(n_req) if meta[i][0] == m]) for m in ("brute", "zoom")}
    mb = [st["mode_batches"][k] - st0["mode_batches"][k] for k in (0, 1)]
    mr = [st["mode_requests"][k] - st0["mode_requests"][k] for k in (0, 1)]
    mx = [st["mixed_length_batches"][k] - st0["mixed_length_batches"][k] for k in (0, 1)]
    summary = {
        "workload": f"Poisson {rate:g} req/s for {seconds:g} s ({len(trace)} arrivals, uniform "
                    f"over the span), sizes 32^2..128^2, N in {{500,1000}}, 3 sequences, grid "
                    f"{grid.size} entries, BF16 resident, half brute / half ZOOM",
        "batch_window_ms": window_ms,
        "brute_force": "BF16 GEMM, top-8 FP32 re-scoring, unit-step FP32 refinement",
        "offered_requests": len(trace),
        "submitted": int(st["submitted"] - st0["submitted"]),
        "admitted": int(st["admitted"] - st0["admitted"]),
        "rejected": int(st["rejected"] - st0["rejected"]) + rejected,
        "done": int(sum(p[0] == "done" for p in polls)),
        "failed": int(sum(p[0] != "done" for p in polls)),
        "latency_ms_p50": float(np.percentile(lat, 50)),
        "latency_ms_p99": float(np.percentile(lat, 99)),
        "latency_ms_p50_by_mode": {m: float(np.percentile(v, 50)) for m, v in by_mode.items() if len(v)},
        "latency_ms_p99_by_mode": {m: float(np.percentile(v, 99)) for m, v in by_mode.items() if len(v)},
        "voxels_per_s": vox / span_s,
        "requests_per_s": n_req / span_s,
        "offered_requests_per_s": rate,
        "span_s": span_s,
        "batches": int(st["batches"] - st0["batches"]),
        "batches_by_mode": {"brute": mb[0], "zoom": mb[1]},
        "requests_per_batch_by_mode": {"brute": mr[0] / max(mb[0], 1), "zoom": mr[1] / max(mb[1], 1)},
        "mixed_count_batches_by_mode": {"brute": mx[0], "zoom": mx[1]},
        "max_batch_requests": int(st["max_batch_requests"]),
        "resident_GB": st["resident_bytes"] / 1e9,
        "peak_reserved_GB": st["peak_reserved_bytes"] / 1e9,
        "budget_GB": st["budget_bytes"] / 1e9,
    }
    return summary, {"grid": grid, "seqs": seqs_h, "types": recheck}


def serve_recheck(sample) -> dict:
    """The oracle re-check of the served results: for each request type, the
    sampled voxels' fingerprints are synthesised by the oracle from the same
    parameters and noise draws (SNR 30); the oracle's CC of the served entry
    must equal the served CC within 1e-5; a brute-force result must be a
    maximum of its 26 unit neighbours under the oracle within 1e-5, and on 8
    voxels per type within 1e-5 of the oracle's own brute force over the
    whole grid; a ZOOM result must equal the oracle's ZOOM (paper schedule)
    on voxels whose oracle decision margins exceed 1e-5."""
    import oracle
    grid, seqs = sample["grid"], sample["seqs"]
    th = host_threads()
    out = {}
    moves = [[(0, a), (1, b), (2, c)] for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)
             if (a, b, c) != (0, 0, 0)]
    dims = np.array(grid.shape)
    for key, t in sample["types"].items():
        n_tr = t["n_tr"]
        res = {"voxels": 0, "cc_at_index_max_abs_d": 0.0}
        worst_local, eps_ok, eps_n, pin_n, pin_ok = -np.inf, 0, 0, 0, 0
        for (s, n), it in t["items"].items():
            # the pool's signals span the whole sequence (its noise level too);
            # a request uses their first n_tr readouts
            seq = seqs[s]
            p = it["params"]
            clean = np.stack([oracle.simulate(seq, *map(float, q)) for q in p])
            sigma = np.sqrt(np.mean(np.abs(clean) ** 2, axis=1, keepdims=True)) / 30.0
            V = (clean[:, :n_tr] + sigma * it["noise"]).astype(np.complex64)
            idx, cc = it["idx"], it["cc"].astype(np.float64)
            at = oracle.cc_at(seq, grid, V, idx[:, None], n_tr=n_tr, threads=th)[:, 0]
            res["voxels"] += len(idx)
            res["cc_at_index_max_abs_d"] = max(res["cc_at_index_max_abs_d"], float(np.abs(at - cc).max()))
            if t["mode"] == "brute":
                u = np.stack(grid.unravel(idx), 1)
                cols = []
                for mv in moves:
                    q = u.copy()
                    for ax, d in mv:
                        q[:, ax] += d
                    ok = np.all((q >= 0) & (q < dims), axis=1)
                    cols.append(np.where(ok, grid.ravel(q[:, 0], q[:, 1], q[:, 2], q[:, 3]), -1))
                nb = oracle.cc_at(seq, grid, V, np.stack(cols, 1), n_tr=n_tr, threads=th)
                worst_local = max(worst_local, float((nb.max(axis=1) - at).max()))
                if eps_n < 8:
                    k = min(8 - eps_n, len(idx))
                    bf = oracle.bruteforce(seq, grid, V[:k], n_tr=n_tr, threads=th)
                    eps_ok += int(np.sum(at[:k] >= bf["cc"] - 1e-5))
                    eps_n += k
            else:
                # the slot's schedule: the paper's for the whole sequence
                z = oracle.zoom(seq, grid, oracle.schedule_paper(seq, grid), V, n_tr=n_tr,
                                threads=th)
                pinned = z["min_margin"] > 1e-5
                pin_n += int(pinned.sum())
                pin_ok += int(np.sum(idx[pinned] == z["idx"][pinned]))
        if t["mode"] == "brute":
            res["local_max_excess_max"] = worst_local
            res["oracle_bruteforce_voxels"] = eps_n
            res["within_1e-5_of_oracle_best"] = eps_ok / max(eps_n, 1)
            res["pass"] = bool(res["cc_at_index_max_abs_d"] < 1e-5 and worst_local <= 1e-5
                               and eps_ok == eps_n)
        else:
            res["pinned"] = pin_n
            res["agreement_pinned"] = pin_ok / max(pin_n, 1)
            res["pass"] = bool(res["cc_at_index_max_abs_d"] < 1e-5 and pin_ok == pin_n)
        out[key] = res
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads() -> int:
    """The host threads this process may use (affinity), capped by OMP_NUM_THREADS."""
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():
        threads = max(1, min(threads, int(os.environ["OMP_NUM_THREADS"])))
    return threads


def cpu_baseline(w, target_s: float):
    """The FP64 oracle's brute force on a bounded sample: a few voxels against
    a leading slab of T1 rows of the grid, extrapolated to the whole grid."""
    import oracle
    from paper_1506_05393_amd import inputs as I
    oracle.build(force=False)
    nv = 8
    ph = w.phantom
    vox = np.linspace(0, ph.n_vox - 1, nv).astype(np.int64)
    clean = np.stack([oracle.simulate(w.seq, ph.t1[v], ph.t2[v], ph.df[v], ph.b1[v])
                      for v in vox])
    V = I.compose_fingerprints(clean, ph, vox).astype(np.complex64)
    threads = host_threads()
    # calibrate on 2 T1 rows, then size the sample to about target_s
    rows = 2
    sub = I.make_grid(w.grid.t1_ms[:rows], w.grid.t2_ms, w.grid.df_hz)
    t = time.perf_counter()
    oracle.bruteforce(w.seq, sub, V, threads=threads)
    dt = time.perf_counter() - t
    rows = int(min(len(w.grid.t1_ms), max(rows, target_s / max(dt / rows, 1e-6))))
    sub = I.make_grid(w.grid.t1_ms[:rows], w.grid.t2_ms, w.grid.df_hz)
    t = time.perf_counter()
    oracle.bruteforce(w.seq, sub, V, threads=threads)
    dt = time.perf_counter() - t
    full_s = dt * w.grid.size / sub.size
    # the same oracle on one core, on one T1 row
    sub1 = I.make_grid(w.grid.t1_ms[:1], w.grid.t2_ms, w.grid.df_hz)
    t = time.perf_counter()
    oracle.bruteforce(w.seq, sub1, V, threads=1)
    dt1 = time.perf_counter() - t
    return {"value": nv / full_s, "unit": "voxels/s", "cores": threads, "kind": "oracle",
            "sample": f"{nv} voxels x {sub.size} entries ({rows} of {len(w.grid.t1_ms)} T1 rows) "
                      f"in {dt:.1f} s, extrapolated to {w.grid.size} entries",
            "one_core": {"value": nv / (dt1 * w.grid.size / sub1.size), "unit": "voxels/s",
                         "sample": f"{nv} voxels x {sub1.size} entries (1 T1 row) in {dt1:.1f} s"},
            "nproc": os.cpu_count(), "cpu_model": cpu_model()}


def _param_errors(grid, idx, ref_idx):
    """Mean and max |dT1| (ms), |dT2| (ms), |ddf| (Hz) between grid entries."""
    a = np.stack(grid.values(np.asarray(idx, np.int64))[:3], axis=1)
    b = np.stack(grid.values(np.asarray(ref_idx, np.int64))[:3], axis=1)
    d = np.abs(a - b)
    return {k: {"mean": float(d[:, i].mean()), "max": float(d[:, i].max())}
            for i, k in enumerate(("T1_ms", "T2_ms", "df_Hz"))}


def _agreement(idx, ref_idx, pinned):
    same = np.asarray(idx) == np.asarray(ref_idx)
    return {"pinned": int(pinned.sum()), "voxels": int(len(same)),
            "agreement_pinned": float(same[pinned].mean()) if pinned.any() else None,
            "agreement_all": float(same.mean())}


def oracle_agreement(api, ctx, torch, threads: int):
    """The small workload (16x16 phantom, N = 200, 50,400 entries; on-grid and
    off-grid truths) with fingerprints synthesised by the oracle: the FP64
    oracle's brute force and ZOOM (paper schedule and the 2 x 3 multi-start
    schedule), timed on all host threads and on one, against the library's
    FP32 brute force, BF16 + re-scoring, and both ZOOM schedules on the same
    fingerprints. Agreement on pinned voxels (oracle margin > 1e-5) and on
    all, and the T1/T2/df errors against the oracle."""
    import oracle
    from paper_1506_05393_amd import inputs as I
    from paper_1506_05393_amd import workloads as W
    out = {}
    for on_grid in (True, False):
        w = W.small_dgs(on_grid)
        ph = w.phantom
        clean = np.stack([oracle.simulate(w.seq, ph.t1[v], ph.t2[v], ph.df[v], ph.b1[v])
                          for v in range(ph.n_vox)])
        V = I.compose_fingerprints(clean, ph).astype(np.complex64)
        s_paper = oracle.schedule_paper(w.seq, w.grid)
        s_multi = oracle.schedule_multistart(w.seq, w.grid, *MULTISTART)
        t = time.perf_counter()
        bf = oracle.bruteforce(w.seq, w.grid, V, top_k=2, threads=threads)
        t_bf = time.perf_counter() - t
        t = time.perf_counter()
        zp = oracle.zoom(w.seq, w.grid, s_paper, V, threads=threads)
        t_zp = time.perf_counter() - t
        t = time.perf_counter()
        zm = oracle.zoom(w.seq, w.grid, s_multi, V, threads=threads)
        t_zm = time.perf_counter() - t
        sub = np.arange(0, ph.n_vox, 16)  # one core: every 16th voxel
        t = time.perf_counter()
        oracle.bruteforce(w.seq, w.grid, V[sub], threads=1)
        t_bf1 = (time.perf_counter() - t) * ph.n_vox / len(sub)
        t = time.perf_counter()
        oracle.zoom(w.seq, w.grid, s_multi, V[sub], threads=1)
        t_zm1 = (time.perf_counter() - t) * ph.n_vox / len(sub)
        # the library on the same fingerprints
        sq = api.Sequence(ctx, w.seq)
        Vd = torch.from_numpy(V).cuda()
        d32 = api.simulate_dictionary(ctx, sq, w.grid, dtype="f32")
        d16 = api.simulate_dictionary(ctx, sq, w.grid, dtype="bf16")
        gpu = {"fp32": api.match_bruteforce(ctx, d32, Vd, top_k=2),
               "bf16_rescore": api.match_bruteforce(ctx, d16, Vd, top_k=8, seq=sq, grid=w.grid),
               "zoom_paper": api.zoom_search(ctx, sq, w.grid, Vd, sched=s_paper),
               "zoom_multistart_2x3": api.zoom_search(ctx, sq, w.grid, Vd, sched=s_multi)}
        torch.cuda.synchronize()
        pin_bf = bf["margin"] > 1e-5
        res = {"oracle_seconds": {"bruteforce": t_bf, "zoom_paper": t_zp,
                                  "zoom_multistart_2x3": t_zm, "threads": threads,
                                  "bruteforce_one_core": t_bf1,
                                  "zoom_multistart_2x3_one_core": t_zm1,
                                  "one_core_sample": f"every 16th voxel ({len(sub)}), scaled"},
               "oracle_zoom_vs_bruteforce": {
                   "paper": _agreement(zp["idx"], bf["idx"], pin_bf),
                   "multistart_2x3": _agreement(zm["idx"], bf["idx"], pin_bf),
                   "n_sim_mean": {"paper": float(zp["n_sim"].mean()),
                                  "multistart_2x3": float(zm["n_sim"].mean())}}}
        for name, r in gpu.items():
            idx = r["idx"].cpu().numpy()
            cc = r["cc"].cpu().numpy().astype(np.float64)
            ref = bf if not name.startswith("zoom") else (zp if name == "zoom_paper" else zm)
            pin = pin_bf if ref is bf else ref["min_margin"] > 1e-5
            e = {"vs": "oracle brute force" if ref is bf else "oracle ZOOM, same schedule",
                 **_agreement(idx, ref["idx"], pin),
                 "max_abs_dCC": float(np.abs(cc - ref["cc"]).max()),
                 "param_error_vs_oracle": _param_errors(w.grid, idx, ref["idx"])}
            if on_grid:
                e["param_error_vs_truth"] = _param_errors(w.grid, idx, ph.truth_idx)
            if name.startswith("zoom"):
                e["agreement_with_oracle_bruteforce"] = _agreement(idx, bf["idx"], pin_bf)
                e["n_sim_mean"] = float(r["n_sim"].double().mean().item())
            res[name] = e
        out["on_grid" if on_grid else "off_grid"] = res
        del d32, d16
    return out


def slice_epsilon_agreement(w, gpu: dict):
    """The slice workload against the stored oracle brute force of its seeded
    64-voxel subset (tests/golden/slice64_bruteforce_oracle.json, written by
    the oracle alone): for each GPU path the fraction of subset voxels whose
    returned entry's oracle CC, against the oracle's own fingerprint, is
    within 1e-5 of the oracle's best, and index agreement on pinned ones."""
    import oracle
    from paper_1506_05393_amd import inputs as I
    path = os.path.join(ROOT, "tests", "golden", "slice64_bruteforce_oracle.json")
    with open(path) as f:
        G = json.load(f)
    vox = np.array(G["noisy_voxels"])
    n = len(vox)
    ph = w.phantom
    clean = np.stack([oracle.simulate(w.seq, ph.t1[v], ph.t2[v], ph.df[v], ph.b1[v])
                      for v in vox])
    V = I.compose_fingerprints(clean, ph, vox).astype(np.complex64)
    best = np.array(G["cc"][:n])
    pinned = np.array(G["margin"][:n]) > 1e-5
    ref_idx = np.array(G["idx"][:n])
    out = {"subset": f"{n} phantom voxels (PCG64(2024)), oracle brute force over the full grid",
           "pinned": int(pinned.sum())}
    for name, idx in gpu.items():
        at = oracle.cc_at(w.seq, w.grid, V, idx[vox][:, None])[:, 0]
        out[name] = {"eps_agreement_1e-5": float(np.mean(at >= best - 1e-5)),
                     "index_agreement": float(np.mean(idx[vox] == ref_idx)),
                     "index_agreement_pinned": (float(np.mean(idx[vox][pinned] == ref_idx[pinned]))
                                                if pinned.any() else None),
                     "max_shortfall": float(np.max(best - at))}
    return out


def slice_zoom_oracle_timing(w, threads: int):
    """The oracle's ZOOM (paper schedule) on every voxel of the slice, all host
    threads, and on every 16th voxel on one core (scaled)."""
    import oracle
    from paper_1506_05393_amd import inputs as I
    ph = w.phantom
    clean = np.stack([oracle.simulate(w.seq, ph.t1[v], ph.t2[v], ph.df[v], ph.b1[v])
                      for v in range(ph.n_vox)])
    V = I.compose_fingerprints(clean, ph).astype(np.complex64)
    s = oracle.schedule_paper(w.seq, w.grid)
    t = time.perf_counter()
    z = oracle.zoom(w.seq, w.grid, s, V, threads=threads)
    t_all = time.perf_counter() - t
    sub = np.arange(0, ph.n_vox, 16)
    t = time.perf_counter()
    oracle.zoom(w.seq, w.grid, s, V[sub], threads=1)
    t_one = (time.perf_counter() - t) * ph.n_vox / len(sub)
    return {"value": ph.n_vox / t_all, "unit": "voxels/s", "cores": threads,
            "seconds": t_all, "n_sim_mean": float(z["n_sim"].mean()),
            "one_core": {"value": ph.n_vox / t_one, "unit": "voxels/s",
                         "sample": f"every 16th voxel ({len(sub)}) on one core, scaled"}}


# Flops per simulated readout of a ZOOM candidate with pulses about x (RF
# phases 0/180 deg, the benchmark sequences): pulse 6, two free-evolution
# intervals 2 x 15, the voxel scaling 2 and v conj(d) 8 in FP32, |d|^2 4 in
# FP64; rated against the FP32 VALU peak without packed FP32.
ZOOM_FLOPS_PER_STEP = 50.0

# FP32 flops per entry and readout of the CC-map recursion with general RF
# pulses: 3x3 rotation (15), two precession + relaxation intervals (2 x 10),
# |d|^2 (4), v conj(d) (8), |v|^2 shared by two entries (2), counted from the
# kernel's 28 FMA-class instructions per entry and readout.
CC_MAP_FLOPS_PER_STEP = 56.0
# FP32 VALU peak without packed FP32: 256 CUs x 4 SIMDs x 16 lanes x 2 flops
# (FMA) x 2.4 GHz (the published 157.3 TFLOP/s counts packed FP32 pairs)
FP32_VALU_UNPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12


def cc_map_bench(api, ctx, torch, repeats: int = 5):
    """CC mapping after Experiment 1 (37,260,000 entries, N = 500): the map of
    one fingerprint, simulated on the fly, and the Property I-III checks."""
    from paper_1506_05393_amd import properties, workloads as W
    name, seq, grid, truth, ti = W.exp1_ccmap()
    sq = api.Sequence(ctx, seq)
    params = torch.tensor([[truth[0], truth[1], truth[2], 1.0]], dtype=torch.float64,
                          device=ctx.device)
    v = api.simulate_signals(ctx, sq, params)
    out = torch.empty((1, grid.size), dtype=torch.float32, device=ctx.device)
    api.cc_map(ctx, sq, grid, v, out=out)
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_read("k_cc_map", reset=True)
    for _ in range(repeats):
        api.cc_map(ctx, sq, grid, v, out=out)
    torch.cuda.synchronize()
    ms, n = ctx.profile_read("k_cc_map")
    ctx.profile(False)
    ms /= max(n, 1)
    m = out[0].cpu().numpy()
    E, N = grid.size, seq.n
    kt = (ti[0] * len(grid.t2_ms) + ti[1]) * len(grid.df_hz) + ti[2]
    props = properties.check(m, (len(grid.t1_ms), len(grid.t2_ms), len(grid.df_hz)), grid.df_hz,
                             grid.t1_ms, grid.t2_ms, seq.tr_ms, truth=ti)
    tflops = E * N * CC_MAP_FLOPS_PER_STEP / (ms * 1e-3) / 1e12
    return {"workload": name, "entries": E, "n_tr": N, "truth_T1_T2_df": list(truth),
            "kernel": "k_cc_map", "ms": ms, "launches": n,
            "entries_per_s": E / (ms * 1e-3), "readout_steps_per_s": E * N / (ms * 1e-3),
            "roofline": {"bound": "alu", "achieved": tflops,
                         "peak": FP32_VALU_UNPACKED_TFLOPS, "unit": "TFLOP/s",
                         "frac": tflops / FP32_VALU_UNPACKED_TFLOPS,
                         "flops_per_entry_readout": CC_MAP_FLOPS_PER_STEP},
            "argmax_is_truth": bool(int(np.argmax(m)) == kt), "max_cc": float(m.max()),
            "properties": props,
            "paper_context": "Experiment 1: 4 h 35 min to generate the dictionary and the CC "
                             "maps (C++, 2.0 GHz dual-core laptop)"}


def smoothing_bench(api, ctx, torch, w, vox, d32, ws, wsz, base, repeats: int = 3):
    """Temporal 3-point smoothing (Methods, Experiment 4; Fig. 7B) on the
    slice: the fingerprints smoothed by mrf_smooth_signals, the dictionary
    smoothed by K1's delay line, then brute force and ZOOM; times beside the
    unsmoothed ones (`base`) and T1/T2/df errors against the phantom's truth."""
    import dataclasses
    seq3 = dataclasses.replace(w.seq, smooth=3)
    sq3 = api.Sequence(ctx, seq3)
    ga = api.GridArg(w.grid)
    sched = api.schedule_paper(ctx, sq3, ga)
    n_vox = vox.shape[0]
    vs = torch.empty_like(vox)
    out = api._result_tensors(n_vox, ctx.device)
    outz = api._result_tensors(n_vox, ctx.device, with_nsim=True)
    ev = lambda: torch.cuda.Event(enable_timing=True)
    t = {"smooth_signals": [], "dict_f32": [], "match_f32": [], "zoom": []}
    for r in range(repeats + 1):
        e = [ev() for _ in range(5)]
        e[0].record()
        api.smooth_signals(ctx, vox, 3, out=vs, seq=sq3)
        e[1].record()
        api.simulate_dictionary(ctx, sq3, ga, dtype="f32", out=d32)
        e[2].record()
        api.match_bruteforce(ctx, d32, vs, top_k=2, workspace=ws, out=out)
        e[3].record()
        api.zoom_search(ctx, sq3, ga, vs, sched=sched, workspace=wsz, out=outz)
        e[4].record()
        torch.cuda.synchronize()
        if r:
            for k, a_, b_ in zip(t, e[:-1], e[1:]):
                t[k].append(a_.elapsed_time(b_))
    med = {k: float(np.median(v)) for k, v in t.items()}
    ph = w.phantom

    def err(idx):
        t1, t2, df, _ = w.grid.values(idx)
        return {"T1_ms": float(np.mean(np.abs(t1 - ph.t1))),
                "T2_ms": float(np.mean(np.abs(t2 - ph.t2))),
                "df_Hz": float(np.mean(np.abs(df - ph.df)))}

    idx_b = out["idx"].cpu().numpy()
    idx_z = outz["idx"].cpu().numpy()
    return {"taps": 3, "ms": med,
            "dict_f32_ratio_vs_unsmoothed": med["dict_f32"] / base["dict_f32"],
            "zoom_ratio_vs_unsmoothed": med["zoom"] / base["zoom"],
            "zoom_index_agreement_vs_brute": float(np.mean(idx_z == idx_b)),
            "mean_abs_error_brute_smoothed": err(idx_b),
            "mean_abs_error_brute_unsmoothed": err(base["idx_f32"]),
            "mean_abs_error_zoom_smoothed": err(idx_z),
            "mean_abs_error_zoom_unsmoothed": err(base["idx_zoom"])}


def zoom_dict_bench(api, ctx, torch, w, sq, vox, sched, base, repeats: int = 50):
    """MRF-ZOOM over a resident dictionary (the paper's MZfulldict): the slice's
    whole grid as entry-major FP32 rows (K1), then the gathering engine; its
    time per slice beside the simulating engine's (`base`)."""
    ga = api.GridArg(w.grid)
    N, E = w.n_tr, w.grid.size
    d = api.alloc_dictionary(N, E, "f32rows")
    ev = lambda: torch.cuda.Event(enable_timing=True)
    gen = []
    for r in range(3):
        a_, b_ = ev(), ev()
        a_.record()
        api.simulate_dictionary(ctx, sq, ga, dtype="f32rows", out=d)
        b_.record()
        torch.cuda.synchronize()
        gen.append(a_.elapsed_time(b_))
    n_vox = vox.shape[0]
    ws = api.Workspace(ctx.device)
    out = api._result_tensors(n_vox, ctx.device, with_nsim=True)
    api.zoom_search_dict(ctx, d, ga, vox, sched, workspace=ws, out=out)
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_read("k_zoom", reset=True)
    zl = []
    for _ in range(repeats):
        a_, b_ = ev(), ev()
        a_.record()
        api.zoom_search_dict(ctx, d, ga, vox, sched, workspace=ws, out=out)
        b_.record()
        zl.append((a_, b_))
    torch.cuda.synchronize()
    kms, kn = ctx.profile_read("k_zoom")
    ctx.profile(False)
    zl = [a_.elapsed_time(b_) for a_, b_ in zl]
    nsim = out["n_sim"].cpu().numpy()
    idx = out["idx"].cpu().numpy()
    kavg = kms / max(kn, 1)
    read_bytes = float(np.abs(nsim).sum()) * N * 8  # each visited entry's row, once
    gen_ms = float(np.median(gen[1:]))
    del d
    torch.cuda.empty_cache()
    return {"what": "ZOOM reading visited entries from a resident entry-major FP32 dictionary "
                    "(paper: MZfulldict)",
            "dict_rows_gen_ms": gen_ms,
            "dict_rows_gen_GB_per_s": E * N * 8 / (gen_ms * 1e-3) / 1e9,
            "slice_ms_p50": float(np.percentile(zl, 50)),
            "slice_ms_p99": float(np.percentile(zl, 99)),
            "voxels_per_s": n_vox / (float(np.median(zl)) * 1e-3),
            "kernel": "k_zoom (gathering)", "kernel_avg_ms": kavg,
            "n_sim_mean": float(np.abs(nsim).mean()),
            "roofline": {"bound": "hbm", "achieved": read_bytes / (kavg * 1e-3) / 1e9,
                         "peak": PEAK["hbm_gbps"], "unit": "GB/s",
                         "frac": read_bytes / (kavg * 1e-3) / 1e9 / PEAK["hbm_gbps"],
                         "algorithmic_bytes": read_bytes,
                         "bytes_per_unit": "8 N per visited entry (its row, read once)"},
            "speedup_vs_simulating_zoom": base["zoom_ms"] / float(np.median(zl)),
            "speedup_vs_f32_brute": base["brute_ms"] / float(np.median(zl)),
            "index_agreement_vs_simulating_zoom": float(np.mean(idx == base["idx_zoom"]))}


def device_peaks(api, ctx, torch, write_gb: float = 16.0):
    """Measured device peaks: MFMA-only loops per dtype and a non-temporal
    write stream (libmrf probe kernels, timed by HIP events on their launch
    stream), and a plain copy (torch, timed by events on the same stream)."""
    n_cu = torch.cuda.get_device_properties(ctx.device).multi_processor_count
    out = torch.empty(n_cu * 2 * 256, dtype=torch.float32, device=ctx.device)
    res = {"what": "MFMA-only loops (4 independent 32x32 accumulators per wave, 2 waves per "
                   "SIMD; operands constant, and for bf16_varied varying by lane and element, "
                   "which lowers the clock); write = one 16 B store per thread, 4 KB per "
                   "workgroup; copy = torch copy_"}
    ctx.profile(True)
    for dt, iters, per_lane in (("f32", 120000, 16), ("bf16", 240000, 128)):
        name = "k_probe_mfma_" + dt
        api.probe_mfma(ctx, dt, 1000, out)
        torch.cuda.synchronize()
        ctx.profile_read(name, reset=True)
        fl = 0.0
        for _ in range(3):
            fl = api.probe_mfma(ctx, dt, iters, out)
        torch.cuda.synchronize()
        ms, n = ctx.profile_read(name)
        res[f"mfma_{dt}_tflops"] = fl / (ms / n * 1e-3) / 1e12
        res[f"mfma_{dt}_output_exact"] = bool((out == float(per_lane * iters)).all().item())
    api.probe_mfma_varied(ctx, 1000, out)
    torch.cuda.synchronize()
    ctx.profile_read("k_probe_mfma_bf16_varied", reset=True)
    fl = 0.0
    for _ in range(3):
        fl = api.probe_mfma_varied(ctx, 240000, out)
    torch.cuda.synchronize()
    ms, n = ctx.profile_read("k_probe_mfma_bf16_varied")
    res["mfma_bf16_varied_tflops"] = fl / (ms / n * 1e-3) / 1e12
    res["mfma_bf16_varied_output_finite"] = bool(torch.isfinite(out).all().item())
    nb = int(write_gb * 1e9) // 32 * 32
    buf = torch.empty(nb, dtype=torch.uint8, device=ctx.device)
    api.probe_write(ctx, buf)
    torch.cuda.synchronize()
    ctx.profile_read("k_probe_write", reset=True)
    for _ in range(3):
        api.probe_write(ctx, buf, pattern=0x1234567)
    torch.cuda.synchronize()
    ms, n = ctx.profile_read("k_probe_write")
    ctx.profile(False)
    res["write_GB_per_s"] = nb / (ms / n * 1e-3) / 1e9
    w4 = buf.view(torch.int32).view(-1, 4)
    res["write_output_exact"] = bool(int(w4[0, 0]) == 0x1234567 and int(w4[-1, 0]) == 0x1234567
                                     and int(w4[-1, 1]) == (w4.shape[0] - 1) % (1 << 32))
    half = nb // 2
    x, y = buf[:half], buf[half:]
    a_, b_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    y.copy_(x)
    a_.record()
    for _ in range(3):
        y.copy_(x)
    b_.record()
    torch.cuda.synchronize()
    res["copy_GB_per_s"] = 2 * half / (a_.elapsed_time(b_) / 3 * 1e-3) / 1e9
    del buf, x, y, w4
    torch.cuda.empty_cache()
    return res


def vendor_gemm(torch, m: int, k: int, n: int, reps: int = 10):
    """torch.matmul (hipBLASLt) on a BF16 GEMM of the brute-force shape (M = 2
    rows per voxel, K = the packed readouts, N a slice of the entries), on
    random data, timed by events: the vendor library's rate on this shape,
    beside which the fused GEMM + top-k kernel is read."""
    g = torch.Generator(device="cuda").manual_seed(1)
    a = torch.randn(m, k, device="cuda", dtype=torch.bfloat16, generator=g)
    b = torch.randn(k, n, device="cuda", dtype=torch.bfloat16, generator=g)
    for _ in range(3):
        c = a @ b
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        c = a @ b
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b, c
    torch.cuda.empty_cache()
    return {"shape_mkn": [m, k, n], "ms": ms, "TFLOP_per_s": 2.0 * m * n * k / (ms * 1e-3) / 1e12}


def copy_probe(gb: float):
    """y = x * 1 over `gb` GB of float32: an elementwise kernel that reads and
    writes exactly gb GB, to scale FETCH_SIZE / WRITE_SIZE counter readings."""
    import torch
    n = int(gb * 1e9) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4}))


def main():
    args = parse()
    if args.copy_probe_gb > 0:
        copy_probe(args.copy_probe_gb)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    from paper_1506_05393_amd import api, workloads as W

    w = W.slice64() if args.workload == "slice64" else W.small_dgs(False)
    ctx = api.Context(0)
    sq = api.Sequence(ctx, w.seq)
    log(f"workload {w.name}: {w.phantom.n_vox} voxels, {w.grid.size} entries, N={w.n_tr}")
    vox = make_inputs(api, ctx, sq, w, torch)
    n_vox, N, E = vox.shape[0], w.n_tr, w.grid.size
    d32 = api.alloc_dictionary(N, E, "f32")
    d16 = api.alloc_dictionary(N, E, "bf16")
    ws = api.Workspace(ctx.device)
    wsz = api.Workspace(ctx.device)
    out32 = api._result_tensors(n_vox, ctx.device)
    out16 = api._result_tensors(n_vox, ctx.device)
    outz = api._result_tensors(n_vox, ctx.device, with_nsim=True)
    ga = api.GridArg(w.grid)
    sched = api.schedule_paper(ctx, sq, ga)
    sched_loc = api.schedule_local(ga)
    ref32 = api._result_tensors(n_vox, ctx.device, with_nsim=True)
    ref16 = api._result_tensors(n_vox, ctx.device, with_nsim=True)
    torch.cuda.synchronize()

    ev = lambda: torch.cuda.Event(enable_timing=True)
    rows = {}

    def step(record):
        marks = [("t0", ev())]
        marks[-1][1].record()
        # the FP32 planar and the BF16 dictionary from one simulation pass
        api.simulate_dictionary_pair(ctx, sq, ga, out=(d32, d16))
        marks.append(("dict_pair", ev()))
        marks[-1][1].record()
        api.match_bruteforce(ctx, d32, vox, top_k=2, workspace=ws, out=out32)
        marks.append(("match_f32", ev()))
        marks[-1][1].record()
        api.match_bruteforce(ctx, d16, vox, top_k=8, seq=sq, grid=ga, workspace=ws, out=out16)
        marks.append(("match_bf16_rescore", ev()))
        marks[-1][1].record()
        api.zoom_search(ctx, sq, ga, vox, sched=sched, workspace=wsz, out=outz)
        marks.append(("zoom", ev()))
        marks[-1][1].record()
        # unit-step local refinement from each brute-force result (ZOOM engine,
        # init = the brute-force entry)
        api.zoom_search(ctx, sq, ga, vox, sched=sched_loc, start=out32["idx"], workspace=wsz,
                        out=ref32)
        marks.append(("refine_f32", ev()))
        marks[-1][1].record()
        api.zoom_search(ctx, sq, ga, vox, sched=sched_loc, start=out16["idx"], workspace=wsz,
                        out=ref16)
        marks.append(("refine_bf16", ev()))
        marks[-1][1].record()
        if record:
            rows.setdefault("_marks", []).append(marks)

    for i in range(args.warmup):
        step(False)
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")
    ctx.profile(True)
    for k in ("k_match_f32", "k_sim_dict", "k_match_bf16", "k_rescore"):
        ctx.profile_read(k, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.profile(False)
    log(f"timed {args.steps} steps in {wall:.2f} s")

    # single-slice ZOOM latency over 50 repeated calls
    zl = []
    for _ in range(50):
        a_, b_ = ev(), ev()
        a_.record()
        api.zoom_search(ctx, sq, ga, vox, sched=sched, workspace=wsz, out=outz)
        b_.record()
        zl.append((a_, b_))
    torch.cuda.synchronize()
    zl = [a_.elapsed_time(b_) for a_, b_ in zl]
    nsim = outz["n_sim"].cpu().numpy()
    # the multi-start schedule on the same slice
    sched_ms = api.schedule_multistart(ctx, sq, ga, *MULTISTART)
    outzm = api._result_tensors(n_vox, ctx.device, with_nsim=True)
    zm = []
    for _ in range(10):
        a_, b_ = ev(), ev()
        a_.record()
        api.zoom_search(ctx, sq, ga, vox, sched=sched_ms, workspace=wsz, out=outzm)
        b_.record()
        zm.append((a_, b_))
    torch.cuda.synchronize()
    zm = [a_.elapsed_time(b_) for a_, b_ in zm]
    ccm = None
    if not args.no_ccmap:
        log("cc map (Experiment 1) ...")
        ccm = cc_map_bench(api, ctx, torch)
    peaks = None
    if not args.no_peaks:
        log("device peaks ...")
        peaks = device_peaks(api, ctx, torch)
    vendor = None
    if not args.no_peaks:
        # the BF16 GEMM's packed shape: 2 rows per voxel, 8 values per
        # 4-readout block with the blocks padded to 4, a 65536-entry slice
        kb = 8 * (((w.n_tr + 3) // 4 + 3) // 4 * 4)
        log("vendor BF16 GEMM on the same shape ...")
        vendor = vendor_gemm(torch, 2 * n_vox, kb, 65536)

    per_row = {}
    step_ms = []
    for marks in rows["_marks"]:
        step_ms.append(marks[0][1].elapsed_time(marks[-1][1]))
        for (n0, e0), (n1, e1) in zip(marks[:-1], marks[1:]):
            per_row.setdefault(n1, []).append(e0.elapsed_time(e1))
    gemm_ms, gemm_n = ctx.profile_read("k_match_f32")
    sim_ms, sim_n = ctx.profile_read("k_sim_dict")
    gemm_avg = gemm_ms / max(gemm_n, 1)
    sim_avg = float(np.median(per_row["dict_pair"]))
    # each dictionary alone, for comparison (outside the timed steps)
    sep = {"f32": [], "bf16": []}
    for _ in range(3):
        for dt, d in (("f32", d32), ("bf16", d16)):
            a_, b_ = ev(), ev()
            a_.record()
            api.simulate_dictionary(ctx, sq, ga, dtype=dt, out=d)
            b_.record()
            torch.cuda.synchronize()
            sep[dt].append(a_.elapsed_time(b_))
    sep = {k: float(np.median(v)) for k, v in sep.items()}
    b16_ms, b16_n = ctx.profile_read("k_match_bf16")
    rs_ms, rs_n = ctx.profile_read("k_rescore")
    b16_avg = b16_ms / max(b16_n, 1)
    idx32 = out32["idx"].cpu().numpy()
    idx16 = out16["idx"].cpu().numpy()
    idxz = outz["idx"].cpu().numpy()
    rf32 = ref32["idx"].cpu().numpy()
    rf16 = ref16["idx"].cpu().numpy()
    flops = 8.0 * n_vox * N * E
    achieved = flops / (gemm_avg * 1e-3) / 1e12
    dict_bytes = E * N * 8 + E * N * 4 + 2 * E * 8  # FP32 planes, BF16 blocks, two norms
    ms_per_step = wall * 1e3 / args.steps
    res = {
        "metric": "voxels/s at 64x64 N=1000: brute vs ZOOM, FP32 vs BF16; p99 slice latency",
        "value": n_vox / (ms_per_step * 1e-3),
        "unit": "voxels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "voxels": n_vox, "n_tr": N, "entries": E,
                   "step": "dictionary generation (FP32 and BF16, one pass) + brute-force FP32 "
                           "+ brute-force BF16 with top-8 FP32 re-scoring + MRF-ZOOM + local "
                           "refinement of both brute-force results"},
        "roofline": {"bound": "mfma", "kernel": "k_match_f32_3m", "achieved": achieved,
                     "peak": PEAK["fp32_mfma_tflops"], "unit": "TFLOP/s",
                     "frac": achieved / PEAK["fp32_mfma_tflops"],
                     "traffic": counted_traffic("mrf::k_match_f32_3m<16>", "match.hip"),
                     "avg_ms": gemm_avg, "launches": gemm_n,
                     "algorithmic_flops_per_launch": flops,
                     "flops_note": "achieved counts 8 V N E (a complex MAC as 4 real MACs); the "
                                   "kernel's three-product form issues 6 V N E MFMA flops, so frac can "
                                   "exceed 1; issued_frac is the MFMA utilisation",
                     "issued_frac": 0.75 * achieved / PEAK["fp32_mfma_tflops"],
                     "peak_measured": peaks["mfma_f32_tflops"] if peaks else None,
                     "frac_measured": achieved / peaks["mfma_f32_tflops"] if peaks else None},
        "rows_ms": {k: float(np.median(v)) for k, v in per_row.items()},
        "brute_f32_voxels_per_s": n_vox / (float(np.median(per_row["match_f32"])) * 1e-3),
        "brute_bf16_rescore_voxels_per_s":
            n_vox / (float(np.median(per_row["match_bf16_rescore"])) * 1e-3),
        "bf16": {"kernel": "k_match_bf16", "avg_ms": b16_avg,
                 "TFLOP_per_s": flops / (b16_avg * 1e-3) / 1e12,
                 "frac_bf16_peak": flops / (b16_avg * 1e-3) / 1e12 / PEAK["bf16_mfma_tflops"],
                 "frac_bf16_measured": (flops / (b16_avg * 1e-3) / 1e12 / peaks["mfma_bf16_tflops"]
                                        if peaks else None),
                 "frac_bf16_varied_peak": (flops / (b16_avg * 1e-3) / 1e12 /
                                           peaks["mfma_bf16_varied_tflops"] if peaks else None),
                 "vendor_gemm_same_shape": vendor,
                 "ratio_vs_vendor_gemm": (flops / (b16_avg * 1e-3) / 1e12 / vendor["TFLOP_per_s"]
                                          if vendor else None),
                 "rescore_ms": rs_ms / max(rs_n, 1),
                 "index_agreement_vs_f32": float(np.mean(idx16 == idx32)),
                 "speedup_vs_f32": float(np.median(per_row["match_f32"]) /
                                         np.median(per_row["match_bf16_rescore"]))},
        "zoom_vs_brute": {"index_agreement_vs_f32": float(np.mean(idxz == idx32)),
                          "speedup_vs_f32": float(np.median(per_row["match_f32"]) / np.median(zl)),
                          "speedup_vs_bf16": float(np.median(per_row["match_bf16_rescore"]) /
                                                   np.median(zl))},
        "refined": {"what": "unit-step local refinement (ZOOM engine started at each "
                            "brute-force result) to the local CC maximum",
                    "f32_ms": float(np.median(per_row["refine_f32"])),
                    "bf16_ms": float(np.median(per_row["refine_bf16"])),
                    "f32_moved": float(np.mean(rf32 != idx32)),
                    "bf16_moved": float(np.mean(rf16 != idx16)),
                    "index_agreement_f32_bf16": float(np.mean(rf32 == rf16)),
                    "index_agreement_zoom_vs_f32": float(np.mean(idxz == rf32)),
                    "n_sim_mean_bf16": float(ref16["n_sim"].double().mean().item())},
        "dict_gen": {"kernel": "k_sim_dict (FP32 planes and BF16 blocks from one recursion pass)",
                     "ms": sim_avg, "bytes": dict_bytes,
                     "GB_per_s": dict_bytes / (sim_avg * 1e-3) / 1e9,
                     "frac_hbm": dict_bytes / (sim_avg * 1e-3) / 1e9 / PEAK["hbm_gbps"],
                     "frac_write_measured": (dict_bytes / (sim_avg * 1e-3) / 1e9 /
                                             peaks["write_GB_per_s"] if peaks else None),
                     "traffic": counted_traffic("mrf::k_sim_dict<5, 1, true, false>", "sim.hip"),
                     "separate_ms": {"f32": sep["f32"], "bf16": sep["bf16"],
                                     "sum": sep["f32"] + sep["bf16"]}},
        "zoom_multistart": {
            "schedule": "paper stages from a 2 x 3 start lattice over T1/T2 (ends included), "
                        "outer rounds [df window, fine df, 2-D zooms 100/50/20/10/1 ms] <= 8; "
                        "the cheapest lattice whose oracle ZOOM matched the oracle brute force "
                        "on every pinned voxel of both small workloads",
            "slice_ms_p50": float(np.percentile(zm, 50)),
            "slice_ms_p99": float(np.percentile(zm, 99)), "repeats": len(zm),
            "voxels_per_s": n_vox / (float(np.median(zm)) * 1e-3),
            "n_sim_mean": float(outzm["n_sim"].double().mean().item()),
            "speedup_vs_f32": float(np.median(per_row["match_f32"]) / np.median(zm)),
            "speedup_vs_bf16": float(np.median(per_row["match_bf16_rescore"]) / np.median(zm)),
            "index_agreement_vs_f32": float(np.mean(outzm["idx"].cpu().numpy() == idx32))},
        "zoom_voxels_per_s": n_vox / (float(np.median(zl)) * 1e-3),
        "zoom": {"schedule": "paper (Methods, Experiment 2 steps 1-5)",
                 "n_sim_mean": float(nsim.mean()), "n_sim_max": int(nsim.max()),
                 "slice_ms_p50": float(np.percentile(zl, 50)),
                 "slice_ms_p99": float(np.percentile(zl, 99)), "repeats": len(zl),
                 "roofline": {
                     "bound": "alu", "kernel": "k_zoom",
                     "achieved": float(nsim.sum()) * N * ZOOM_FLOPS_PER_STEP /
                                 (float(np.median(zl)) * 1e-3) / 1e12,
                     "peak": FP32_VALU_UNPACKED_TFLOPS, "unit": "TFLOP/s",
                     "frac": float(nsim.sum()) * N * ZOOM_FLOPS_PER_STEP /
                             (float(np.median(zl)) * 1e-3) / 1e12 / FP32_VALU_UNPACKED_TFLOPS,
                     "flops_per_readout": ZOOM_FLOPS_PER_STEP,
                     "algorithmic_flops_per_launch": float(nsim.sum()) * N * ZOOM_FLOPS_PER_STEP,
                     "note": "sum over voxels of entries simulated x readouts x flops per "
                             "readout, over the slice's median call time"}},
        "slice_latency_ms": {"p50": float(np.percentile(step_ms, 50)),
                             "p99": float(np.percentile(step_ms, 99))},
        "device_peaks": peaks,
        "cc_map": ccm,
        "paper_context": "paper: 116.72 s per 1731-voxel 64x64 slice (ZOOM, df dictionary) on a "
                         "2.0 GHz dual-core laptop, C++",
    }
    if not args.no_smooth:
        log("smoothing ...")
        res["smoothing"] = smoothing_bench(
            api, ctx, torch, w, vox, d32, ws, wsz,
            {"dict_f32": sep["f32"], "zoom": res["zoom"]["slice_ms_p50"],
             "idx_f32": idx32, "idx_zoom": idxz})
    del d32, d16
    torch.cuda.empty_cache()
    if not args.no_zoom_dict:
        log("zoom over a resident dictionary ...")
        res["zoom_dict"] = zoom_dict_bench(
            api, ctx, torch, w, sq, vox, sched,
            {"zoom_ms": res["zoom"]["slice_ms_p50"], "brute_ms": res["rows_ms"]["match_f32"],
             "idx_zoom": idxz})
        log(f"zoom dict: {res['zoom_dict']['slice_ms_p50']:.2f} ms per slice")
    if not args.no_volume:
        log("volume ...")
        res["volume"] = volume_bench(api, ctx, torch)
    serve_sample = None
    if not args.no_serve:
        log("serving ...")
        res["serving"], serve_sample = serve_bench(api, ctx, torch, args.serve_seconds,
                                                   args.serve_rate,
                                                   max_requests=args.serve_requests)
        log(f"serving done: {res['serving']['done']} requests, p50 "
            f"{res['serving']['latency_ms_p50']:.1f} ms, p99 {res['serving']['latency_ms_p99']:.1f} ms")
        if args.serve_window_ms > 0:
            log(f"serving with a {args.serve_window_ms:g} ms batching window ...")
            res["serving_batched"], _ = serve_bench(api, ctx, torch, args.serve_seconds,
                                                    args.serve_rate,
                                                    max_requests=args.serve_requests,
                                                    window_ms=args.serve_window_ms)
            rb = res["serving_batched"]["requests_per_batch_by_mode"]
            log(f"batched serving done: {res['serving_batched']['done']} requests, "
                f"{rb['brute']:.2f} / {rb['zoom']:.2f} requests per brute / ZOOM batch")
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cb = cpu_baseline(w, args.cpu_seconds)
        if args.workload == "slice64":
            th = host_threads()
            log("oracle ZOOM on the slice ...")
            cb["zoom"] = slice_zoom_oracle_timing(w, th)
            log("agreement with the oracle (small workload, slice subset) ...")
            res["agreement_vs_oracle"] = {
                "small_dgs": oracle_agreement(api, ctx, torch, th),
                "slice64_subset": slice_epsilon_agreement(
                    w, {"fp32": idx32, "bf16_rescore": idx16, "zoom_paper": idxz,
                        "zoom_multistart_2x3": outzm["idx"].cpu().numpy(),
                        "fp32_refined": rf32})}
        res["cpu_baseline"] = cb
        if serve_sample is not None:
            log("oracle re-check of served results ...")
            res["serving"]["oracle_recheck"] = serve_recheck(serve_sample)
        if "agreement_vs_oracle" in res:
            ag = res["agreement_vs_oracle"]
            small = ag["small_dgs"]
            sl = ag["slice64_subset"]
            pin = lambda k: min(small[g][k]["agreement_pinned"] for g in ("on_grid", "off_grid"))
            pin_bf = lambda k: min(small[g][k]["agreement_with_oracle_bruteforce"]
                                   ["agreement_pinned"] for g in ("on_grid", "off_grid"))
            res["speedups_at_agreement"] = {
                "what": "speedup on the 64x64 slice; agreement with the FP64 oracle's brute force "
                        "on pinned voxels (margin > 1e-5) of the small workload (on- and off-grid, "
                        "the lower) and the fraction of the slice's stored 64-voxel oracle subset "
                        "within 1e-5 of the best CC",
                "bf16_rescore_vs_fp32": {"speedup": res["bf16"]["speedup_vs_f32"],
                                         "agreement_pinned_small": pin("bf16_rescore"),
                                         "eps_agreement_slice": sl["bf16_rescore"]["eps_agreement_1e-5"]},
                "zoom_multistart_2x3_vs_fp32": {
                    "speedup": res["zoom_multistart"]["speedup_vs_f32"],
                    "agreement_pinned_small": pin_bf("zoom_multistart_2x3"),
                    "eps_agreement_slice": sl["zoom_multistart_2x3"]["eps_agreement_1e-5"]},
                "zoom_paper_vs_fp32": {
                    "speedup": res["zoom_vs_brute"]["speedup_vs_f32"],
                    "agreement_pinned_small": pin_bf("zoom_paper"),
                    "eps_agreement_slice": sl["zoom_paper"]["eps_agreement_1e-5"]}}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
