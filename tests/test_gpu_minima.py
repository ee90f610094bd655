"""GPU local-minimum census against the oracle's spurious-minimum count (Section V)."""

import numpy as np
import pytest

from oracle import divergence as dv
from oracle import path as op
from workloads import build_config, grid_domain
from workloads.seeds import targets_sources

pytestmark = pytest.mark.gpu


def check_against_oracle(cls, ref_field, adj_ptr, adj_idx, t):
    ref = set(op.spurious_minima(ref_field, adj_ptr, adj_idx, t))
    certain = set(np.nonzero(cls == 1)[0].tolist())
    undecided = set(np.nonzero(cls == 2)[0].tolist())
    assert certain <= ref <= certain | undecided
    return len(ref), len(certain), len(undecided)


@pytest.mark.parametrize("kind", ["kl", "tv"])
def test_disk_fields_have_no_minima(gpu_ctx, kind):
    from paper_1708_02845_amd import Kernel
    inst = build_config("disk4096")
    k = Kernel.load_dense(gpu_ctx, inst.P, adjacency=(inst.adj_ptr, inst.adj_idx))
    try:
        ts = targets_sources(0, inst.N, 3)[0]
        D, bounds = k.batch_fields(ts, kind)
        cls, counts = k.local_minima(ts, D, bounds)
        cls, counts = cls.cpu().numpy(), counts.cpu().numpy()
        for i, t in enumerate(ts):
            ref = (dv.kl_field if kind == "kl" else dv.tv_field)(inst.P, int(t))
            n_ref, n_cert, n_und = check_against_oracle(cls[i], ref, inst.adj_ptr, inst.adj_idx, int(t))
            assert n_ref == 0 and counts[i, 0] == n_cert == 0 and counts[i, 1] == n_und
    finally:
        k.free()


@pytest.mark.parametrize("kind", ["kl", "tv"])
def test_truncated_grid_fields(gpu_ctx, kind):
    from paper_1708_02845_amd import Kernel
    g = grid_domain(97, 3, (0.1, 0.25), seed_id=71)
    P = g.poisson_kernel().astype(np.float32)
    tau = 1e-3
    k = Kernel.load_dense(gpu_ctx, P, tau=tau, adjacency=(g.adj_ptr, g.adj_idx))
    try:
        ts = targets_sources(71, g.N, 4)[0]
        D, bounds = k.batch_fields(ts, kind)
        cls, counts = k.local_minima(ts, D, bounds)
        cls, counts = cls.cpu().numpy(), counts.cpu().numpy()
        Pt, thr = dv.truncate(P.astype(np.float64), tau)
        for i, t in enumerate(ts):
            ref = dv.tv_trunc_field(Pt, int(t)) if kind == "tv" else dv.kl_trunc_field(Pt, int(t), thr)
            _, n_cert, n_und = check_against_oracle(cls[i], ref, g.adj_ptr, g.adj_idx, int(t))
            assert counts[i, 0] == n_cert and counts[i, 1] == n_und
    finally:
        k.free()


def test_planted_minima_exact(gpu_ctx):
    import torch
    from paper_1708_02845_amd import Kernel
    g = grid_domain(41, 1, (0.1, 0.2), seed_id=72)
    P = g.poisson_kernel().astype(np.float32)
    k = Kernel.load_dense(gpu_ctx, P, adjacency=(g.adj_ptr, g.adj_idx))
    try:
        t = g.N // 3
        f = np.abs(np.arange(g.N, dtype=np.float32) - t)   # decreasing towards t along ids
        pits = [5, g.N // 2, g.N - 7]
        for v in pits:
            f[v] = -1.0 - v                                   # strictly below every neighbour
        fields = torch.from_numpy(f).cuda().reshape(1, -1)
        cls, counts = k.local_minima([t], fields, [(0.0, 0.0)])
        cls = cls.cpu().numpy()[0]
        ref = op.spurious_minima(f.astype(np.float64), g.adj_ptr, g.adj_idx, t)
        # zero bounds: every decision is exact, ties count as minima (>=)
        assert sorted(np.nonzero(cls == 1)[0].tolist()) == ref
        assert not np.any(cls == 2)
        assert set(pits) <= set(ref)
        assert int(counts[0, 0].item()) == len(ref) and int(counts[0, 1].item()) == 0
    finally:
        k.free()


@pytest.mark.parametrize("kind", ["kl", "tv"])
@pytest.mark.parametrize("T", [4, 12])
def test_resolved_census_equals_oracle(gpu_ctx, kind, T):
    """After the FP64 re-decision the census is the oracle's set of spurious
    minima exactly (T = 12 takes the many-target pass)."""
    from paper_1708_02845_amd import Kernel
    g = grid_domain(97, 3, (0.1, 0.25), seed_id=71)
    P = g.poisson_kernel().astype(np.float32)
    tau = 1e-3
    k = Kernel.load_dense(gpu_ctx, P, tau=tau, adjacency=(g.adj_ptr, g.adj_idx))
    try:
        ts = targets_sources(73, g.N, T)[0]
        D, bounds = k.batch_fields(ts, kind)
        # bounds widened 1000-fold: many undecided entries for the re-decision
        wide = [(1000.0 * a, 1000.0 * r) for a, r in bounds]
        cls, counts = k.local_minima(ts, D, wide)
        und_before = counts.cpu().numpy()[:, 1].copy()
        k.resolve_minima(ts, kind, cls, counts)
        cls, counts = cls.cpu().numpy(), counts.cpu().numpy()
        Pt, thr = dv.truncate(P.astype(np.float64), tau)
        assert und_before.sum() > 0
        for i, t in enumerate(ts):
            ref = dv.tv_trunc_field(Pt, int(t)) if kind == "tv" else dv.kl_trunc_field(Pt, int(t), thr)
            want = sorted(op.spurious_minima(ref, g.adj_ptr, g.adj_idx, int(t)))
            got = np.nonzero(cls[i] == 1)[0].tolist()
            assert got == want, (i, t)
            assert counts[i, 0] == len(want) and counts[i, 1] == 0
    finally:
        k.free()


def test_resolved_census_on_contraction_fields(gpu_ctx):
    """Dense KL from the contraction: no spurious minima once resolved."""
    from paper_1708_02845_amd import Kernel
    g = grid_domain(97, 3, (0.1, 0.25), seed_id=71)
    P = g.poisson_kernel().astype(np.float32)
    k = Kernel.load_dense(gpu_ctx, P, adjacency=(g.adj_ptr, g.adj_idx), gemm_form="f16x3")
    try:
        ts = targets_sources(74, g.N, 6)[0]
        D, bounds = k.batch_fields(ts, "kl")
        cls, counts = k.local_minima(ts, D, bounds)
        k.resolve_minima(ts, "kl", cls, counts)
        cls, counts = cls.cpu().numpy(), counts.cpu().numpy()
        for i, t in enumerate(ts):
            want = op.spurious_minima(dv.kl_field(P.astype(np.float64), int(t)), g.adj_ptr,
                                      g.adj_idx, int(t))
            assert np.nonzero(cls[i] == 1)[0].tolist() == sorted(want)
            assert counts[i, 1] == 0
    finally:
        k.free()
