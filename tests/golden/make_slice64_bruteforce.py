"""Writes slice64_bruteforce_oracle.json: the FP64 oracle's streaming brute
force (Theory Eq. 1 over every entry of the 391 x 399 x 81 grid, N = 1000)
for the seeded voxel subsets of tests/slice64_subsets.py.

It calls only the oracle and the seeded input generators; no value in the
file comes from the GPU library. Run from the repository root:

    python tests/golden/make_slice64_bruteforce.py [threads]

(about 4 minutes on 8 cores).
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as orc  # noqa: E402
from paper_1506_05393_amd import workloads  # noqa: E402
from tests import slice64_subsets as S  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "slice64_bruteforce_oracle.json")
TOP_K = 8


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else 0
    orc.build(force=False)
    w = workloads.slice64()
    V, truth = S.fingerprints(orc, w)
    t0 = time.time()
    r = orc.bruteforce(w.seq, w.grid, V, top_k=TOP_K, threads=threads)
    dt = time.time() - t0
    doc = {
        "_about": ("FP64 oracle brute force (Theory Eq. 1, every entry) on the 64x64 slice "
                   "workload's grid (T1 100:10:4000, T2 10:5:2000, df -40:1:40; N = 1000, "
                   "sequence seed 1). Rows 0-63: the noisy subset (phantom seed 101, SNR 30, "
                   "voxels drawn with PCG64(2024)); rows 64-79: noise-free fingerprints at the "
                   "grid values nearest to 16 phantom voxels (PCG64(2025)); rows 80-95: "
                   "noise-free fingerprints at grid points of the short-relaxation corner "
                   "T1 100-500 ms, T2 10-60 ms (PCG64(2026)). Written by "
                   "tests/golden/make_slice64_bruteforce.py from the oracle only."),
        "workload": w.name,
        "inputs_sha256": S.digest(V),
        "noisy_voxels": [int(x) for x in S.noisy_voxels(w.phantom.n_vox)],
        "ongrid_voxels": [int(x) for x in S.ongrid_truths(w)[0]],
        "truth_idx": [int(x) for x in truth],
        "top_k": TOP_K,
        "idx": [int(x) for x in r["idx"]],
        "cc": [float(x) for x in r["cc"]],
        "margin": [float(x) for x in r["margin"]],
        "topk_idx": [[int(y) for y in x] for x in r["topk_idx"]],
        "topk_cc": [[float(y) for y in x] for x in r["topk_cc"]],
        "pd_re": [float(x) for x in r["pd"].real],
        "pd_im": [float(x) for x in r["pd"].imag],
        "oracle_seconds": dt,
    }
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=1)
    print(f"wrote {OUT} ({dt:.0f} s)")


if __name__ == "__main__":
    main()
