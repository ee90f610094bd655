"""Throughput of the divergence-distance path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload: the 257x257 grid with 3 seeded rectangular obstacles (N = 60,695
interior rows, B = 1,478 non-zero boundary columns), FP32 dense Poisson
kernel, its CSR truncation at 1e-6 row-relative, one seeded (source, target)
query.  One step is one pass of the whole path for that query:

  dense TV field and dense KL field          streaming over the N x B rows
  truncated TV and KL fields                 streaming over the CSR rows
  KL field through the contraction (f16x3)   log-kernel operand, T = 1
  steepest-descent paths on the KL and TV fields

The value is kernel entries per second, N*B per field, 5 fields per step.
Inputs are resident in HBM before the timed region.  After the timed steps
the batched forms are measured on the same domain with 64 targets (the
contraction in both forms, and 64 paths in one launch); those figures are
reported under "rows" and are not part of the value.  Prints one JSON line.
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
MFMA_PEAK_TFLOPS = {"f16x3": 2500.0, "bf16x3": 2500.0, "f32": 157.3}
# source file of each measured kernel, for matching counter records to the code
KERNEL_SOURCE = {"dense_tv": "stream.hip", "dense_kl": "stream.hip", "csr_tv": "stream.hip",
                 "csr_kl": "stream.hip", "gemm_kl_T1": "gemm.hip", "kl_gemm_f16x3": "gemm.hip"}


def measured_traffic(workload, kernel):
    """HBM bytes per launch (fetched + written) from the rocprofv3 counter record in
    profiles/hbm_traffic.txt, or None when there is none for this kernel or the
    kernel's source has changed since the counters were taken."""
    import hashlib
    src = KERNEL_SOURCE.get(kernel)
    path = os.path.join(ROOT, "profiles", "hbm_traffic.txt")
    if src is None or not os.path.exists(path):
        return None
    with open(os.path.join(ROOT, "paper_1708_02845_amd", "csrc", src), "rb") as f:
        sha = hashlib.sha1(f.read()).hexdigest()[:12]
    with open(path) as f:
        for line in f:
            t = line.split()
            if len(t) == 5 and t[0] == workload and t[1] == kernel and t[4] == sha:
                return int(t[2]) + int(t[3])
    return None


METRIC = "kernel entries/sec (N·B·targets/s)"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--max-steps", type=int, default=4000)
    ap.add_argument("--batch", type=int, default=64, help="targets of the batched rows")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-rows", action="store_true", help="skip the batched-row measurements")
    ap.add_argument("--setup-workers", type=int, default=None,
                    help="processes that build the kernel matrix (1 = in-process; use 1 "
                         "under a profiler that initialises the GPU before main)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a plain 1 GiB device copy first (calibrates HBM byte counters)")
    ap.add_argument("--kernel-cache", default=None,
                    help=".npy path: load the kernel matrix from it if present, else build and "
                         "save it there (lets a profiled run skip the build)")
    ap.add_argument("--qps", type=float, default=200.0, help="serving: arrival rate")
    ap.add_argument("--duration", type=float, default=30.0, help="serving: seconds of arrivals")
    ap.add_argument("--slots", type=int, default=1,
                    help="serving: batch slots (streams) per domain; keep domains x slots within "
                         "the process's hardware queues, or short batches queue behind long ones")
    ap.add_argument("--serving-grids", default="129,257,513,1025",
                    help="serving: grid sizes of the resident domains")
    ap.add_argument("--workload", default="grid257", choices=["grid257", "grid1025", "serving"],
                    help="grid1025: the 1025x1025, 20-obstacle domain (32 GB kernel), batched KL "
                         "at 64 targets, single-target and truncated streaming")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_matrix(g, args, progress=None):
    """FP32 kernel matrix of a grid workload, optionally through an .npy cache."""
    path = args.kernel_cache
    if path and os.path.exists(path):
        P = np.load(path, mmap_mode="r")
        if P.shape == (g.N, g.K) and P.dtype == np.float32:
            log(f"kernel matrix from {path}")
            return P
    P = g.poisson_kernel(dtype=np.float32, workers=args.setup_workers, progress=progress)
    if path:
        np.save(path, P)
        log(f"kernel matrix saved to {path}")
    return P


def run_grid1025(args):
    """Full-size measurements on the 1025x1025 domain (N = 992,998, B = 8,150).

    The 64- and 256-target contraction in both forms, the single-target TV/KL streams,
    and the truncated (tau = 1e-5) TV/KL streams with their local-minimum
    census.  Parity at this size is checked by tests/test_gpu_full_size.py.
    """
    import torch

    from paper_1708_02845_amd import Context, Kernel
    from workloads import build_config
    from workloads.seeds import targets_sources

    g = build_config("grid1025")
    log(f"grid1025: N={g.N} K={g.K}; building the kernel matrix")
    t0 = time.perf_counter()
    last = [0.0]

    def prog(done, k):
        if time.perf_counter() - last[0] > 10 or done == k:
            last[0] = time.perf_counter()
            log(f"kernel matrix: {done}/{k} columns, {last[0] - t0:.0f} s")
    P = kernel_matrix(g, args, progress=prog)
    build_s = time.perf_counter() - t0
    T = 64
    ts_all = targets_sources(2, g.N, 256)[0]
    ts = ts_all[:T]
    ctx = Context(0)
    res = {}
    for form in ("f16x3", "bf16x3", "f32"):
        log(f"loading with the {form} operand")
        t1 = time.perf_counter()
        k = Kernel.load_dense(ctx, P, gemm_form=form)
        load_s = time.perf_counter() - t1
        N, B = k.N, k.B
        lda = (B + 63) // 64 * 64
        reps = 5
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        for TT in (64, 256):
            tsT = ts_all[:TT]
            D = torch.empty((TT, N), dtype=torch.float32, device="cuda:0")
            k.batch_fields(tsT, "kl", out=D)
            torch.cuda.synchronize()
            a.record()
            for _ in range(reps):
                _, bounds = k.batch_fields(tsT, "kl", out=D)
            b.record()
            torch.cuda.synchronize()
            us = 1000.0 * a.elapsed_time(b) / reps
            flops = 2.0 * N * B * TT * (1 if form == "f32" else 3)
            byts = N * lda * 4 + TT * lda * 4 + TT * N * 4 + N * 4
            tf = flops / (us * 1e-6) / 1e12
            res[f"a5_batched_kl_{form}_T{TT}"] = {
                "avg_us": round(us, 1), "entries_per_s": N * B * TT / (us * 1e-6),
                "alg_bytes": byts, "GB/s": round(gbs(byts, us), 1),
                "hbm_frac": round(gbs(byts, us) / HBM_PEAK_GBS, 4), "mfma_TFLOP/s": round(tf, 1),
                "mfma_frac": round(tf / MFMA_PEAK_TFLOPS[form], 4), "load_s": round(load_s, 1)}
            log(f"{form}: {us:.0f} us per {TT}-target launch")
            del D
            torch.cuda.empty_cache()
        if form == "f16x3":
            f = torch.empty((k.N,), dtype=torch.float32, device="cuda:0")
            for kind in ("tv", "kl"):
                k.field(int(ts[0]), kind, out=f)
                torch.cuda.synchronize()
                a.record()
                for _ in range(reps):
                    _, bd = k.field(int(ts[0]), kind, out=f)
                b.record()
                torch.cuda.synchronize()
                us = 1000.0 * a.elapsed_time(b) / reps
                byts = N * B * 4 + N * 4
                res[f"a{2 if kind == 'tv' else 3}_stream_{kind}"] = {
                    "avg_us": round(us, 1), "alg_bytes": byts, "GB/s": round(gbs(byts, us), 1),
                    "hbm_frac": round(gbs(byts, us) / HBM_PEAK_GBS, 4)}
                log(f"stream {kind}: {us:.0f} us")
        k.free()
        torch.cuda.empty_cache()
    # the truncated kernel (tau = 1e-5 row-relative): streams and local-minimum census
    tau = 1e-5
    log(f"loading the tau={tau:g} truncation")
    kc = Kernel.load_dense(ctx, P, tau=tau, adjacency=(g.adj_ptr, g.adj_idx))
    N, B, nnz = kc.N, kc.B, kc.nnz
    f = torch.empty((1, N), dtype=torch.float32, device="cuda:0")
    t0_ = int(ts[0])
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    for kind in ("tv", "kl"):
        kc.field(t0_, kind, out=f[0])
        torch.cuda.synchronize()
        reps = 5
        a.record()
        for _ in range(reps):
            _, bd = kc.field(t0_, kind, out=f[0])
        b.record()
        torch.cuda.synchronize()
        us = 1000.0 * a.elapsed_time(b) / reps
        byts = nnz * 6 + N * (16 if kind == "tv" else 24)
        cls, counts = kc.local_minima([t0_], f, [bd])
        cert, und = int(counts[0, 0].item()), int(counts[0, 1].item())
        resolved, res_ms = resolve_census(kc, [t0_], kind, cls, counts)
        res[f"a4_csr_{kind}_tau1e-5"] = {
            "avg_us": round(us, 1), "nnz": nnz, "nnz_frac": round(nnz / (N * B), 4),
            "alg_bytes": byts, "GB/s": round(gbs(byts, us), 1),
            "hbm_frac": round(gbs(byts, us) / HBM_PEAK_GBS, 4),
            "local_minima_certain": cert, "local_minima_undecided": und,
            "local_minima_fp64": resolved[0], "fp64_census_ms": res_ms}
        log(f"csr {kind}: {us:.0f} us, minima {counts[0].tolist()}")
    res.update(csr_batch_rows(kc, ts_all, "tau1e-5"))
    kc.free()
    torch.cuda.empty_cache()
    # the same truncation with FP16 stored values (4 bytes per stored entry)
    log(f"loading the tau={tau:g} truncation with FP16 values")
    kc = Kernel.load_dense(ctx, P, tau=tau, adjacency=(g.adj_ptr, g.adj_idx), csr_values="f16")
    for kind in ("tv", "kl"):
        kc.field(t0_, kind, out=f[0])
        torch.cuda.synchronize()
        reps = 5
        a.record()
        for _ in range(reps):
            _, bd = kc.field(t0_, kind, out=f[0])
        b.record()
        torch.cuda.synchronize()
        us = 1000.0 * a.elapsed_time(b) / reps
        byts = nnz * 4 + N * (20 if kind == "tv" else 28)
        cls, counts = kc.local_minima([t0_], f, [bd])
        res[f"a4_csr_{kind}_tau1e-5_f16"] = {
            "avg_us": round(us, 1), "nnz": nnz, "alg_bytes": byts, "GB/s": round(gbs(byts, us), 1),
            "hbm_frac": round(gbs(byts, us) / HBM_PEAK_GBS, 4), "bound_abs": bd[0],
            "local_minima_certain": int(counts[0, 0].item()),
            "local_minima_undecided": int(counts[0, 1].item())}
        log(f"csr f16 {kind}: {us:.0f} us, minima {counts[0].tolist()}")
    res.update(csr_batch_rows(kc, ts_all, "tau1e-5_f16"))
    kc.free()
    torch.cuda.empty_cache()
    # the same truncation with the floored log-kernel operand: KL_tau of 256
    # targets as one f16x3 contraction
    log(f"loading the tau={tau:g} truncation with the floored contraction operand")
    kg = Kernel.load_dense(ctx, P, tau=tau, gemm_form="f16x3")
    lda = (kg.B + 63) // 64 * 64
    D = torch.empty((len(ts_all), kg.N), dtype=torch.float32, device="cuda:0")
    kg.batch_fields(ts_all, "kl", out=D)
    torch.cuda.synchronize()
    reps = 5
    a.record()
    for _ in range(reps):
        kg.batch_fields(ts_all, "kl", out=D)
    b.record()
    torch.cuda.synchronize()
    us = 1000.0 * a.elapsed_time(b) / reps
    TT = len(ts_all)
    flops = 2.0 * kg.N * kg.B * TT * 3
    byts = kg.N * lda * 4 + TT * lda * 4 + TT * kg.N * 4 + kg.N * 4
    tf = flops / (us * 1e-6) / 1e12
    res[f"a4_trunc_kl_contraction_f16x3_tau{tau:g}_T{TT}"] = {
        "avg_us": round(us, 1), "entries_per_s": kg.N * kg.B * TT / (us * 1e-6),
        "alg_bytes": byts, "GB/s": round(gbs(byts, us), 1),
        "hbm_frac": round(gbs(byts, us) / HBM_PEAK_GBS, 4), "mfma_TFLOP/s": round(tf, 1),
        "mfma_frac": round(tf / MFMA_PEAK_TFLOPS["f16x3"], 4)}
    log(f"floored KL contraction: {us:.0f} us for {TT} targets")
    del D
    kg.free()
    torch.cuda.empty_cache()
    # second truncation point: an absolute threshold that keeps about 5% of the entries
    tau_abs = 4e-4
    log(f"loading the absolute tau={tau_abs:g} truncation")
    kc = Kernel.load_dense(ctx, P, tau=tau_abs, tau_relative=False,
                           adjacency=(g.adj_ptr, g.adj_idx))
    res.update(csr_batch_rows(kc, ts_all, f"abs{tau_abs:g}"))
    kc.free()
    torch.cuda.empty_cache()
    res["a0_grid_poisson_kernel"] = grid_poisson_row(ctx, g, P, build_s)
    ctx.close()
    main_row = res["a5_batched_kl_f16x3_T64"]
    out = {"metric": METRIC, "value": main_row["entries_per_s"], "unit": "entries/s",
           "n_gpus": 1, "steps": 5, "warmup": 1, "ms_per_step": main_row["avg_us"] / 1000.0,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f16x3",
           "data": "synthetic",
           "config": {"workload": "grid 1025x1025, 20 rectangular obstacles (sides U[0.025,0.075]); "
                                  "64 targets per launch, KL via contraction",
                      "N": g.N, "B": int(P.shape[1]) - 4, "targets": T,
                      "kernel_matrix_build_s": round(build_s, 1)},
           "roofline": {"bound": "hbm", "kernel": "kl_gemm_f16x3", "achieved": main_row["GB/s"],
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": main_row["hbm_frac"],
                        "traffic": measured_traffic("grid1025_T64", "kl_gemm_f16x3")},
           "rows": res}
    print(json.dumps(out), flush=True)


def grid_poisson_row(ctx, g, P_host, build_s, batch=1024):
    """The whole P_IB of a grid domain solved on the device (FP64 multigrid-
    preconditioned CG, FP32 output), timed against the host build of the same
    matrix, and compared with it on sampled rows."""
    import torch
    out = torch.empty((g.N, g.K), dtype=torch.float32, device="cuda:0")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st = ctx.grid_poisson_kernel(g.node_type(), out=out, tol=1e-12, batch=batch)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    # algorithmic bytes of one iteration over a batch: 13 passes over the fine
    # level (product 2, residual update 3, restriction 1, prolongation and
    # smoothing 2, direction with the solution update 5), 4 over each coarser level
    G, levels = g.G, []
    Gl = G
    for _ in range(st["levels"]):
        levels.append(Gl)
        Gl = Gl // 2 + 1
    per_iter = 8 * batch * (13 * G * G + sum(4 * x * x for x in levels[1:]))
    byts = st["total_iterations"] * per_iter + 4 * g.N * g.K
    rows = np.random.default_rng(5).choice(g.N, size=64, replace=False)
    diff = float(np.abs(out[torch.as_tensor(rows, device="cuda:0")].cpu().numpy() -
                        np.asarray(P_host[rows, :g.K], dtype=np.float32)).max())
    del out
    torch.cuda.empty_cache()
    gbs_ = byts / secs / 1e9
    log(f"grid Poisson kernel on the device: {secs:.2f} s, {st}, max |diff| {diff:.2e}")
    return {"seconds": round(secs, 3), "host_build_s": round(build_s, 1),
            "speedup_vs_host": round(build_s / secs, 2), "iterations_max": st["iterations"],
            "iterations_total": st["total_iterations"], "batches": st["batches"],
            "levels": st["levels"], "max_rel_residual": st["max_rel_residual"],
            "alg_bytes": byts, "GB/s": round(gbs_, 1), "hbm_frac": round(gbs_ / HBM_PEAK_GBS, 4),
            "max_abs_diff_vs_host_64_rows": diff}


def resolve_census(k, targets, kind, cls, counts):
    """FP64 re-decision of a census: (minima per field, milliseconds)."""
    import torch
    if counts is None:
        counts = torch.zeros((len(targets), 2), dtype=torch.int32, device=cls.device)
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    k.resolve_minima(targets, kind, cls, counts)
    b.record()
    torch.cuda.synchronize()
    return [int(x) for x in counts[:, 0].cpu().tolist()], round(a.elapsed_time(b), 2)


def csr_batch_rows(kc, ts_all, label):
    """The many-target pass over the truncated rows at T = 256 (TV and KL),
    with the local-minimum census of the 256 fields.

    Per stored entry and target it reads 4 bytes of target weights from LDS
    (peak 128 B per clock per CU: 78.6 TB/s at 256 CUs and 2.4 GHz) and issues
    1.5 (TV in fixed point: a min, and half of a three-way add) or 1 (KL: an
    FMA) VALU operations (peak 256 x 64 lanes x 2.4 GHz = 39.3e12 per second)."""
    import torch
    N, B, nnz = kc.N, kc.B, kc.nnz
    T = 256
    ts = ts_all[:T]
    D = torch.empty((T, N), dtype=torch.float32, device="cuda:0")
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    out = {}
    for kind in ("tv", "kl"):
        kc.batch_fields(ts, kind, out=D)
        torch.cuda.synchronize()
        reps = 3
        a.record()
        for _ in range(reps):
            _, bounds = kc.batch_fields(ts, kind, out=D)
        b.record()
        torch.cuda.synchronize()
        us = 1000.0 * a.elapsed_time(b) / reps
        upd = nnz * T / (us * 1e-6)
        byts = nnz * 6 + N * 16 + T * N * 4
        ops = 1.5 if kind == "tv" else 1
        cls, counts = kc.local_minima(ts, D, bounds)
        c = counts.cpu().numpy()
        # the FP64 re-decision on the first 8 fields (it costs 1 + degree FP64 rows
        # per undecided vertex)
        resolved, res_ms = resolve_census(kc, ts[:8], kind, cls[:8].contiguous(), None)
        out[f"a4_csr_batch_{kind}_{label}_T{T}"] = {
            "avg_us": round(us, 1), "nnz": nnz, "nnz_frac": round(nnz / (N * B), 4),
            "entry_updates_per_s": upd, "entries_per_s": N * B * T / (us * 1e-6),
            "lds_frac": round(upd * 4 / 78.6e12, 4),
            "valu_frac": round(upd * ops / 39.3e12, 4),
            "GB/s": round(gbs(byts, us), 1),
            "local_minima_per_field": {"certain_mean": float(c[:, 0].mean()),
                                       "certain_max": int(c[:, 0].max()),
                                       "undecided_mean": float(c[:, 1].mean()),
                                       "fp64_first8": resolved, "fp64_census_ms": res_ms}}
        log(f"csr batch {kind} {label}: {us:.0f} us for {T} targets")
    del D
    return out


def cpu_baseline(P32, tau, t, s, adj, max_steps, entries_per_step):
    """The FP64 oracle doing the same step on the host (single-threaded NumPy)."""
    from oracle import divergence as dv
    from oracle import path as op
    P64 = P32.astype(np.float64)
    Pt, thr = dv.truncate(P64, tau)
    reps = 0
    t0 = time.perf_counter()
    while True:
        tv = dv.tv_field(P64, t)
        kl = dv.kl_field(P64, t)
        dv.tv_trunc_field(Pt, t)
        dv.kl_trunc_field(Pt, t, thr)
        dv.kl_field(P64, t)          # the fifth field: KL again (the contraction's definition)
        op.steepest_descent_path(kl, adj[0], adj[1], s, t, max_steps)
        op.steepest_descent_path(tv, adj[0], adj[1], s, t, max_steps)
        reps += 1
        el = time.perf_counter() - t0
        if el >= 10.0 or reps >= 4:
            break
    # the paper's CPU mode: KL distances only at the vertices the path needs
    t1 = time.perf_counter()
    path, _, n_eval = op.steepest_descent_path_lazy(
        lambda xs: dv.distances(P64, t, xs, "kl"), adj[0], adj[1], s, t, max_steps)
    lazy_ms = 1000.0 * (time.perf_counter() - t1)
    return {"value": entries_per_step * reps / el, "unit": "entries/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{reps} full step(s) of this workload (5 fields + 2 paths), FP64 NumPy "
                      f"on one core, {el:.1f} s",
            "path_only_kl": {"ms_per_query": round(lazy_ms, 2), "rows_evaluated": n_eval,
                             "path_vertices": len(path)}}


class Timer:
    """HIP-event timing of one labelled launch group on torch's current stream."""

    def __init__(self, torch):
        self.torch = torch
        self.pairs = {}

    def run(self, name, fn, timed):
        if not timed:
            return fn()
        a = self.torch.cuda.Event(enable_timing=True)
        b = self.torch.cuda.Event(enable_timing=True)
        a.record()
        out = fn()
        b.record()
        self.pairs.setdefault(name, []).append((a, b))
        return out

    def avg_us(self, name):
        return 1000.0 * float(np.mean([a.elapsed_time(b) for a, b in self.pairs[name]]))


def gbs(nbytes, us):
    return nbytes / (us * 1e-6) / 1e9


def run_serving(args):
    """Open-loop serving over resident grid domains (2/5/10/20 obstacles)."""
    import torch

    from paper_1708_02845_amd import Context
    from paper_1708_02845_amd.serve import Server, latency_summary
    from workloads import CONFIGS, grid_domain
    from workloads.serving import poisson_arrivals

    c = CONFIGS["serving4"]
    sizes = [int(x) for x in args.serving_grids.split(",")]
    ctx = Context(0)
    srv = Server(ctx, max_batch=c["max_batch"], slots_per_domain=args.slots,
                 max_steps=c["max_steps"])
    doms = []
    for (G, k, sides) in c["domains"]:
        if G not in sizes:
            continue
        g = grid_domain(G, k, sides, seed_id=c["seed_id"] + G)
        log(f"serving: building {G}x{G} ({g.N} x {g.K})")
        t0 = time.perf_counter()
        last = [0.0]

        def prog(done, kk):
            if time.perf_counter() - last[0] > 10:
                last[0] = time.perf_counter()
                log(f"  {done}/{kk} columns")
        P = g.poisson_kernel(dtype=np.float32, workers=args.setup_workers, progress=prog)
        ok = srv.add_domain(f"grid{G}", P, (g.adj_ptr, g.adj_idx))
        log(f"  built in {time.perf_counter() - t0:.0f} s, admitted={ok}")
        if ok:
            doms.append((f"grid{G}", g.N, srv.domains[f"grid{G}"].kernel.B))
        del P
    # warm every domain once
    for name, n, _ in doms:
        srv.submit(name, 0, n - 1)
    srv.drain()
    srv.completed.clear()
    srv.batch_sizes.clear()
    arr = poisson_arrivals(c["seed_id"], [(nm, n) for nm, n, _ in doms], args.qps, args.duration)
    log(f"serving: {len(arr)} arrivals over {args.duration:.0f} s at {args.qps:.0f} QPS")
    t0 = time.perf_counter()
    qs = srv.run_open_loop(arr, timeout=args.duration * 10 + 60)
    wall = time.perf_counter() - t0
    summ = latency_summary(qs)
    entries = sum(next(n * b for nm, n, b in doms if nm == q.domain) for q in qs)
    per_dom = {}
    for nm, n, b in doms:
        sel = [q for q in qs if q.domain == nm]
        if sel:
            per_dom[nm] = {"N": n, "B": b, **latency_summary(sel),
                           "reached": sum(q.status == "reached" for q in sel)}
    out = {"metric": METRIC, "value": entries / wall, "unit": "entries/s", "n_gpus": 1,
           "steps": len(qs), "warmup": len(doms), "ms_per_step": 1000.0 * wall / len(qs),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f16x3",
           "data": "synthetic",
           "config": {"workload": "serving: resident grid domains, open-loop Poisson arrivals, "
                                  "KL field (f16x3 contraction) + path per query, continuous "
                                  "batching",
                      "domains": [nm for nm, _, _ in doms], "refused": [r[0] for r in srv.refused],
                      "qps_offered": args.qps, "qps_achieved": len(qs) / wall,
                      "max_batch": c["max_batch"], "slots_per_domain": args.slots},
           "latency": summ, "per_domain": per_dom,
           "batch_size_hist": dict(sorted(srv.batch_sizes.items())),
           "hbm_admitted_bytes": srv.hbm_used}
    srv.close()
    ctx.close()
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the path shards by rows)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "grid1025":
        run_grid1025(args)
        return
    if args.workload == "serving":
        run_serving(args)
        return

    import torch

    from paper_1708_02845_amd import Context, Kernel
    from workloads import build_config
    from workloads.seeds import targets_sources

    tau = 1e-6
    g = build_config("grid257")
    P = kernel_matrix(g, args)
    t_arr, s_arr = targets_sources(1, g.N, max(1, args.batch))
    t, s = int(t_arr[0]), int(s_arr[0])
    adj = (g.adj_ptr, g.adj_idx)

    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    ctx = Context(0)
    kd = Kernel.load_dense(ctx, P, adjacency=adj, gemm_form="f16x3")
    kc = Kernel.load_dense(ctx, P, adjacency=adj, tau=tau)
    N, B = kd.N, kd.B
    f = torch.empty((5, N), dtype=torch.float32, device="cuda:0")
    tm = Timer(torch)

    # The two walks of a step are latency-bound chains on one CU each; each
    # runs on a stream of its own as soon as its field is ready, overlapped
    # with the step's remaining field kernels (whose grids leave one workgroup
    # slot per CU free for such work).  The step ends when all three streams
    # have finished.
    main = torch.cuda.current_stream()
    side = [torch.cuda.Stream(), torch.cuda.Stream()]

    def step(timed):
        res = []
        for st, kind, fi in ((side[0], "kl", 1), (side[1], "tv", 0)):
            _, bd = tm.run(f"dense_{kind}", lambda: kd.field(t, kind, out=f[fi]), timed)
            ready = torch.cuda.Event()
            ready.record(main)
            st.wait_event(ready)
            with torch.cuda.stream(st):
                res.append(tm.run(f"path_{kind}", lambda: kd.trace_paths(
                    [s], [t], kind, f[fi].view(1, -1), [bd], args.max_steps), timed))
        tm.run("csr_tv", lambda: kc.field(t, "tv", out=f[2]), timed)
        tm.run("csr_kl", lambda: kc.field(t, "kl", out=f[3]), timed)
        tm.run("gemm_kl_T1", lambda: kd.batch_fields([t], "kl", out=f[4]), timed)
        for st in side:
            main.wait_stream(st)
        return res

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        res_kl, res_tv = step(True)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_per_step = e0.elapsed_time(e1) / args.steps

    nnz = kc.nnz
    lda = (B + 63) // 64 * 64
    traffic = {   # algorithmic bytes per launch
        "dense_tv": N * B * 4 + N * 4,
        "dense_kl": N * B * 4 + N * 4,
        "csr_tv": nnz * 6 + N * (8 + 4 + 4),
        "csr_kl": nnz * 6 + N * (8 + 4 + 8 + 4),
        "gemm_kl_T1": N * B * 4 + N * 4 + N * 4,
    }
    kernels = {}
    for n in ["dense_tv", "dense_kl", "csr_tv", "csr_kl", "gemm_kl_T1", "path_kl", "path_tv"]:
        us = tm.avg_us(n)
        kernels[n] = {"avg_us": round(us, 3)}
        if n in traffic:
            kernels[n].update({"alg_bytes": traffic[n], "GB/s": round(gbs(traffic[n], us), 1),
                               "frac": round(gbs(traffic[n], us) / HBM_PEAK_GBS, 4)})
    dom = max(traffic, key=lambda n: kernels[n]["avg_us"])
    path_len = int(res_kl[1][0].item())
    rechecks = [int(res_kl[3][0].item()), int(res_tv[3][0].item())]
    entries_per_step = 5 * N * B
    value = entries_per_step / (ms_per_step * 1e-3)

    rows = {}
    if not args.no_rows and args.batch > 0:
        T = args.batch
        ts, ss = t_arr[:T], s_arr[:T]
        kf = Kernel.load_dense(ctx, P, gemm_form="f32")
        kb = Kernel.load_dense(ctx, P, gemm_form="bf16x3")
        D = torch.empty((T, N), dtype=torch.float32, device="cuda:0")
        reps = 20
        for form, kern in (("f16x3", kd), ("bf16x3", kb), ("f32", kf)):
            for _ in range(3):
                kern.batch_fields(ts, "kl", out=D)
            torch.cuda.synchronize()
            for _ in range(reps):
                tm.run(f"gemm_{form}", lambda: kern.batch_fields(ts, "kl", out=D), True)
            torch.cuda.synchronize()
            us = tm.avg_us(f"gemm_{form}")
            flops = 2.0 * N * B * T * (1 if form == "f32" else 3)
            byts = N * lda * 4 + T * lda * 4 + T * N * 4 + N * 4
            tf = flops / (us * 1e-6) / 1e12
            rows[f"a5_batched_kl_{form}_T{T}"] = {
                "avg_us": round(us, 2), "fields_per_s": round(T / (us * 1e-6), 1),
                "entries_per_s": N * B * T / (us * 1e-6),
                "alg_bytes": byts, "GB/s": round(gbs(byts, us), 1),
                "hbm_frac": round(gbs(byts, us) / HBM_PEAK_GBS, 4),
                "mfma_TFLOP/s": round(tf, 1),
                "mfma_frac": round(tf / MFMA_PEAK_TFLOPS[form], 4)}
        kf.free()
        kb.free()
        _, bounds = kd.batch_fields(ts, "kl", out=D)
        for _ in range(2):
            kd.trace_paths(ss, ts, "kl", D, bounds, args.max_steps)
        torch.cuda.synchronize()
        for _ in range(10):
            res = tm.run("paths_T", lambda: kd.trace_paths(ss, ts, "kl", D, bounds, args.max_steps),
                         True)
        torch.cuda.synchronize()
        us = tm.avg_us("paths_T")
        lens = res[1].cpu().numpy()
        rows[f"a6_paths_kl_T{T}"] = {"avg_us": round(us, 2), "paths_per_s": round(T / (us * 1e-6), 1),
                                     "mean_vertices": float(lens.mean()),
                                     "fp64_rechecks": int(res[3].sum().item())}
        # triangle-based paths (the method of the paper's figures) on the same fields
        kd.attach_mesh(*g.interior_mesh())
        for _ in range(2):
            kd.trace_paths_triangles(ss, ts, D, 20000)
        torch.cuda.synchronize()
        for _ in range(5):
            res = tm.run("tri_T", lambda: kd.trace_paths_triangles(ss, ts, D, 20000), True)
        torch.cuda.synchronize()
        us = tm.avg_us("tri_T")
        rows[f"triangle_paths_kl_T{T}"] = {
            "avg_us": round(us, 2), "paths_per_s": round(T / (us * 1e-6), 1),
            "mean_points": float(res[2].float().mean().item()),
            "reached": int((res[3] == 0).sum().item())}
        # on-demand walks: FP64 distances only where the path needs them
        for TT in (1, T):
            for _ in range(2):
                kd.trace_paths_on_demand(ss[:TT], ts[:TT], "kl", args.max_steps)
            torch.cuda.synchronize()
            for _ in range(5):
                res = tm.run(f"ondemand_T{TT}",
                             lambda: kd.trace_paths_on_demand(ss[:TT], ts[:TT], "kl",
                                                              args.max_steps), True)
            torch.cuda.synchronize()
            us = tm.avg_us(f"ondemand_T{TT}")
            rows[f"on_demand_paths_kl_T{TT}"] = {
                "avg_us": round(us, 2), "paths_per_s": round(TT / (us * 1e-6), 1),
                "mean_vertices": float(res[1].float().mean().item()),
                "rows_evaluated": int(res[3].sum().item())}
        # KL over the truncated target support (rows of x exact)
        prow = np.asarray(P[t], dtype=np.float64)[np.asarray(P.max(axis=0) > 0)]
        for tau_s in (1e-3, 1e-6):
            kd.support_kl_field(t, tau_s, out=f[0])
            torch.cuda.synchronize()
            for _ in range(20):
                tm.run(f"support_{tau_s}", lambda: kd.support_kl_field(t, tau_s, out=f[0]), True)
            torch.cuda.synchronize()
            us = tm.avg_us(f"support_{tau_s}")
            keep = (prow > 0) & (prow >= tau_s * prow.max())
            pieces = np.zeros((B + 3) // 4 * 4, dtype=bool)
            pieces[:B] = keep
            npieces = int(pieces.reshape(-1, 4).any(axis=1).sum())
            byts = N * npieces * 16 + N * 4
            rows[f"support_kl_tau{tau_s:g}"] = {
                "avg_us": round(us, 3), "support_frac": round(float(keep.mean()), 4),
                "alg_bytes": byts, "GB/s": round(gbs(byts, us), 1),
                "frac": round(gbs(byts, us) / HBM_PEAK_GBS, 4)}
        # more f-divergences on the same streaming pass (chi-squared, Hellinger)
        for kind in ("chi2", "hellinger"):
            kd.field(t, kind, out=f[0])
            torch.cuda.synchronize()
            for _ in range(20):
                tm.run(f"dense_{kind}", lambda: kd.field(t, kind, out=f[0]), True)
            torch.cuda.synchronize()
            us = tm.avg_us(f"dense_{kind}")
            byts = N * B * 4 + N * 4
            rows[f"f_divergence_{kind}_dense"] = {
                "avg_us": round(us, 3), "alg_bytes": byts, "GB/s": round(gbs(byts, us), 1),
                "frac": round(gbs(byts, us) / HBM_PEAK_GBS, 4)}

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
        "config": {"workload": "grid 257x257, 3 rectangular obstacles; 1 query: TV, KL, TV_tau, "
                               "KL_tau (tau=1e-6) streaming fields, KL via f16x3 contraction, "
                               "KL and TV paths",
                   "N": N, "B": B, "csr_nnz": nnz, "targets": 1, "fields_per_step": 5,
                   "kl_path_vertices": path_len, "fp64_rechecks_kl_tv": rechecks,
                   "cache": "warm (no flush between steps)"},
        "roofline": {"bound": "hbm", "kernel": dom,
                     "achieved": round(gbs(traffic[dom], kernels[dom]["avg_us"]), 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs(traffic[dom], kernels[dom]["avg_us"]) / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic("grid257", dom)},
        "kernels": kernels,
        "rows": rows,
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
