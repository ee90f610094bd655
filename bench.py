"""Throughput of the divergence-distance path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload (the 257x257 grid, 3 seeded rectangular obstacles, FP32 dense
Poisson kernel, CSR truncation at 1e-6 row-relative, one seeded target and
source).  One step is one pass of the whole path for that query:

  dense TV field, dense KL field            (streaming over N x B FP32 rows)
  truncated TV and KL fields                (streaming over the CSR rows)
  steepest-descent paths on the dense KL and TV fields

Inputs are resident in HBM before the timed region.  Prints one JSON line.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "kernel entries/sec (N·B·targets/s)"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--max-steps", type=int, default=4000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--setup-workers", type=int, default=None,
                    help="processes that build the kernel matrix (1 = in-process; use 1 "
                         "under a profiler that initialises the GPU before main)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a plain 1 GiB device copy first (calibrates HBM byte counters)")
    return ap.parse_args()


def cpu_baseline(P32, Pt_tau, t, s, adj, max_steps, entries_per_step):
    """The FP64 oracle doing the same step on the host (single-threaded NumPy)."""
    from oracle import divergence as dv
    from oracle import path as op
    P64 = P32.astype(np.float64)
    Pt, thr = dv.truncate(P64, Pt_tau)
    reps = 0
    t0 = time.perf_counter()
    while True:
        tv = dv.tv_field(P64, t)
        kl = dv.kl_field(P64, t)
        dv.tv_trunc_field(Pt, t)
        dv.kl_trunc_field(Pt, t, thr)
        op.steepest_descent_path(kl, adj[0], adj[1], s, t, max_steps)
        op.steepest_descent_path(tv, adj[0], adj[1], s, t, max_steps)
        reps += 1
        el = time.perf_counter() - t0
        if el >= 10.0 or reps >= 3:
            break
    return {"value": entries_per_step * reps / el, "unit": "entries/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{reps} full step(s) of this workload (4 fields + 2 paths), FP64 NumPy, "
                      f"{el:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the path shards by rows, see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1708_02845_amd import Context, Kernel
    from workloads import build_config
    from workloads.seeds import targets_sources

    tau = 1e-6
    g = build_config("c2")
    P = g.poisson_kernel(dtype=np.float32, workers=args.setup_workers)
    t_arr, s_arr = targets_sources(1, g.N, 1)
    t, s = int(t_arr[0]), int(s_arr[0])
    adj = (g.adj_ptr, g.adj_idx)

    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    ctx = Context(0)
    kd = Kernel.load_dense(ctx, P, adjacency=adj)
    kc = Kernel.load_dense(ctx, P, adjacency=adj, tau=tau)
    N, B = kd.N, kd.B
    dev = "cuda:0"
    f = torch.empty((4, N), dtype=torch.float32, device=dev)

    names = ["dense_tv", "dense_kl", "csr_tv", "csr_kl", "paths"]
    ev = {n: [] for n in names}

    def step(timed):
        evs = {}
        for n in names:
            evs[n] = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) \
                if timed else None
        def rec(n, i):
            if timed:
                evs[n][i].record()
        rec("dense_tv", 0); _, b_tv = kd.field(t, "tv", out=f[0]); rec("dense_tv", 1)
        rec("dense_kl", 0); _, b_kl = kd.field(t, "kl", out=f[1]); rec("dense_kl", 1)
        rec("csr_tv", 0); kc.field(t, "tv", out=f[2]); rec("csr_tv", 1)
        rec("csr_kl", 0); kc.field(t, "kl", out=f[3]); rec("csr_kl", 1)
        rec("paths", 0)
        res_kl = kd.trace_paths([s], [t], "kl", f[1].view(1, -1), [b_kl], args.max_steps)
        res_tv = kd.trace_paths([s], [t], "tv", f[0].view(1, -1), [b_tv], args.max_steps)
        rec("paths", 1)
        if timed:
            for n in names:
                ev[n].append(evs[n])
        return res_kl, res_tv

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    t0.record()
    for _ in range(args.steps):
        res_kl, res_tv = step(True)
    t1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_per_step = t0.elapsed_time(t1) / args.steps

    avg_us = {n: 1000.0 * float(np.mean([a.elapsed_time(b) for a, b in ev[n]])) for n in names}
    # algorithmic bytes per launch
    nnz = kc.nnz
    traffic = {
        "dense_tv": N * B * 4 + N * 4,
        "dense_kl": N * B * 4 + N * 4,
        "csr_tv": nnz * 6 + N * (8 + 4 + 4),
        "csr_kl": nnz * 6 + N * (8 + 4 + 8 + 4),
    }
    kernels = {}
    for n in names:
        kernels[n] = {"avg_us": round(avg_us[n], 3)}
        if n in traffic:
            gbs = traffic[n] / (avg_us[n] * 1e-6) / 1e9
            kernels[n].update({"alg_bytes": traffic[n], "GB/s": round(gbs, 1),
                               "frac": round(gbs / HBM_PEAK_GBS, 4)})
    dom = max(traffic, key=lambda n: avg_us[n])
    path_len = int(res_kl[1][0].item())
    rechecks = [int(res_kl[3][0].item()), int(res_tv[3][0].item())]
    entries_per_step = 4 * N * B
    value = entries_per_step / (ms_per_step * 1e-3)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "entries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "grid 257x257, 3 rectangular obstacles, dense + CSR tau=1e-6, "
                               "1 target: TV, KL, TV_tau, KL_tau fields + 2 paths",
                   "N": N, "B": B, "csr_nnz": nnz, "targets": 1, "fields_per_step": 4,
                   "kl_path_vertices": path_len, "fp64_rechecks_kl_tv": rechecks,
                   "cache": "warm (no flush between steps)"},
        "roofline": {"bound": "hbm", "kernel": dom,
                     "achieved": round(traffic[dom] / (avg_us[dom] * 1e-6) / 1e9, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(traffic[dom] / (avg_us[dom] * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": None},
        "kernels": kernels,
        "wall_s_timed": round(wall, 3),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(P, tau, t, s, adj, args.max_steps, entries_per_step)
    kd.free()
    kc.free()
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
