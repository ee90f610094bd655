"""Host-side inputs of the full-size parity tests, built in a process of its own.

    python tests/fullsize_prep.py --out DIR [--workers W] [--grid G --obstacles n --lo a --hi b]

Writes to DIR:
  P32.raw     the FP32 kernel matrix the library loads ([N, K] row-major), from
              the workload's five-point harmonic-measure build
  rows.npy    int64 ids of the rows the oracle solved: a seeded 1% vertex
              sample and the 256 seeded targets
  rows64.npy  FP64 [len(rows), K]: those rows of P_IB from the oracle's row
              solves on the cotangent Laplacian (Section IV, eqs. 32-33; row x
              is (L_II^{-1} e_x)^T (-L_IB) for the symmetric L^c)
  meta.json   N, K, sample size, targets

Both builds fork worker pools, so they run here, in a process that never
touches the GPU; the test process that holds the GPU only reads the files.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

_SOLVER = {}


def _solve_rows(rows):
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)
    return _SOLVER["s"].rows(rows)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--workers", type=int, default=min(16, len(os.sched_getaffinity(0))))
    ap.add_argument("--grid", type=int, default=0, help="grid size override (tests of this script)")
    ap.add_argument("--obstacles", type=int, default=3)
    ap.add_argument("--lo", type=float, default=0.05)
    ap.add_argument("--hi", type=float, default=0.2)
    ap.add_argument("--sample-frac", type=float, default=0.01)
    ap.add_argument("--targets", type=int, default=256)
    a = ap.parse_args()

    from oracle import fem
    from oracle.poisson import RowSolver
    from workloads import build_config, grid_domain
    from workloads.grid import harmonic_measure_5pt
    from workloads.seeds import rng, targets_sources

    t0 = time.perf_counter()

    def say(msg):
        print(f"[prep {time.perf_counter() - t0:6.1f} s] {msg}", flush=True)

    if a.grid:
        g = grid_domain(a.grid, a.obstacles, (a.lo, a.hi), seed_id=2)
    else:
        g = build_config("grid1025")
    N, K = g.N, g.K
    say(f"domain N={N} K={K}; kernel matrix with {a.workers} workers")
    last = [0.0]

    def prog(done, k):
        if time.perf_counter() - last[0] > 10 or done == k:
            last[0] = time.perf_counter()
            say(f"kernel matrix: {done}/{k} columns")
    P = harmonic_measure_5pt(g, dtype=np.float32, workers=a.workers, progress=prog,
                             out_path=os.path.join(a.out, "P32.raw"))
    del P

    ts = targets_sources(2, N, a.targets)[0]
    sample = np.sort(rng(2, "sample").choice(N, size=max(1, int(N * a.sample_frac)),
                                              replace=False))
    rows = np.unique(np.concatenate([sample, ts]))
    say(f"oracle: cotangent Laplacian and LU of L_II; {len(rows)} row solves")
    Lc = fem.cotan_laplacian(g.xy(), g.triangles, n=g.G * g.G)
    _SOLVER["s"] = RowSolver(Lc, g.interior, g.boundary)
    del Lc
    chunks = [rows[i:i + 32] for i in range(0, len(rows), 32)]
    out = np.empty((len(rows), K))
    pos = 0
    import multiprocessing as mp
    with mp.get_context("fork").Pool(max(1, a.workers)) as pool:
        for i, r in enumerate(pool.imap(_solve_rows, chunks)):
            out[pos:pos + len(r)] = r
            pos += len(r)
            if time.perf_counter() - last[0] > 10 or i == len(chunks) - 1:
                last[0] = time.perf_counter()
                say(f"oracle rows: {pos}/{len(rows)}")
    np.save(os.path.join(a.out, "rows.npy"), rows)
    np.save(os.path.join(a.out, "rows64.npy"), out)
    with open(os.path.join(a.out, "meta.json"), "w") as f:
        json.dump({"N": N, "K": K, "sample": int(len(sample)), "targets": int(a.targets)}, f)
    say("done")


if __name__ == "__main__":
    main()
