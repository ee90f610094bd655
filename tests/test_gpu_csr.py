"""GPU parity of the truncated (CSR) fields and their paths against the oracle."""

import numpy as np
import pytest

from conftest import normwise, within_bound
from oracle import divergence as dv
from oracle import path as op
from workloads import build_config, grid_domain
from workloads.seeds import targets_sources

pytestmark = pytest.mark.gpu

TOL = 1e-5


def oracle_trunc(P32, tau, relative, t, kind):
    Pt, thr = dv.truncate(np.asarray(P32, dtype=np.float64), tau, relative)
    if kind == "tv":
        return dv.tv_trunc_field(Pt, t)
    return dv.kl_trunc_field(Pt, t, thr)


@pytest.fixture(scope="module")
def grid(gpu_ctx):
    g = grid_domain(81, 3, (0.1, 0.25), seed_id=41)
    return g, g.poisson_kernel().astype(np.float32)


@pytest.mark.parametrize("tau,relative", [(1e-3, True), (1e-6, True), (1e-4, False)])
@pytest.mark.parametrize("kind", ["tv", "kl"])
def test_truncated_fields(gpu_ctx, grid, tau, relative, kind):
    from paper_1708_02845_amd import Kernel
    g, P = grid
    k = Kernel.load_dense(gpu_ctx, P, tau=tau, tau_relative=relative)
    try:
        assert k.is_csr and 0 < k.nnz <= k.N * k.B
        for t in (0, 400, g.N - 1):
            d, b = k.field(t, kind)
            d = d.cpu().numpy()
            ref = oracle_trunc(P, tau, relative, t, kind)
            assert d[t] == 0.0
            assert normwise(d, ref) <= TOL
            assert within_bound(d, ref, b)
    finally:
        k.free()


def test_host_csr_load_equals_truncating_load(gpu_ctx, grid):
    from paper_1708_02845_amd import Kernel
    g, P = grid
    tau = 1e-3
    keep = P.max(axis=0) > 0
    Pk = P[:, keep]
    Pt, thr = dv.truncate(Pk.astype(np.float64), tau)
    ptr, col, val = dv.csr_from_truncated(Pt)
    kc = Kernel.load_csr(gpu_ctx, Pk.shape[0], Pk.shape[1], ptr, col, val.astype(np.float32),
                         Pk.astype(np.float64).max(axis=1), tau)
    kd = Kernel.load_dense(gpu_ctx, P, tau=tau)
    try:
        assert kc.nnz == kd.nnz == len(val)
        for kind in ("tv", "kl"):
            a = kc.field(55, kind)[0].cpu().numpy()
            b = kd.field(55, kind)[0].cpu().numpy()
            assert np.array_equal(a, b)
    finally:
        kc.free()
        kd.free()


def test_csr_load_rejects_bad_rows(gpu_ctx):
    from paper_1708_02845_amd import DDError, Kernel
    ptr = np.array([0, 2, 3])
    with pytest.raises(DDError, match="DD_EINVAL"):   # descending columns
        Kernel.load_csr(gpu_ctx, 2, 4, ptr, [2, 1, 0], [0.5, 0.5, 1.0], [0.5, 1.0], 1e-3)
    with pytest.raises(DDError, match="DD_EINVAL"):   # empty row
        Kernel.load_csr(gpu_ctx, 2, 4, [0, 2, 2], [0, 1], [0.5, 0.5], [0.5, 1.0], 1e-3)
    with pytest.raises(DDError, match="DD_EINVAL"):   # zero value stored
        Kernel.load_csr(gpu_ctx, 2, 4, ptr, [0, 1, 0], [0.5, 0.0, 1.0], [0.5, 1.0], 1e-3)


@pytest.mark.parametrize("kind", ["kl", "tv"])
def test_truncated_paths_identical(gpu_ctx, grid, kind):
    from paper_1708_02845_amd import Kernel
    g, P = grid
    tau = 1e-3
    k = Kernel.load_dense(gpu_ctx, P, tau=tau, adjacency=(g.adj_ptr, g.adj_idx))
    try:
        ts, ss = targets_sources(41, g.N, 5)
        for s, t in zip(ss, ts):
            got, status, _ = k.plan_path(int(s), int(t), kind, 4000)
            ref_field = oracle_trunc(P, tau, True, int(t), kind)
            ref, ref_status = op.steepest_descent_path(ref_field, g.adj_ptr, g.adj_idx, int(s),
                                                       int(t), 4000)
            assert status == {0: "reached", 1: "stuck", 2: "max_steps"}[ref_status]
            assert got == ref
    finally:
        k.free()


@pytest.mark.parametrize("kind", ["tv", "kl"])
def test_grid257_truncated_full_size(gpu_ctx, kind):
    from paper_1708_02845_amd import Kernel
    g = build_config("grid257")
    P = g.poisson_kernel(dtype=np.float32)
    k = Kernel.load_dense(gpu_ctx, P, tau=1e-6)
    try:
        t = int(targets_sources(1, g.N, 1)[0][0])
        d, b = k.field(t, kind)
        d = d.cpu().numpy()
        ref = oracle_trunc(P, 1e-6, True, t, kind)
        assert normwise(d, ref) <= TOL and within_bound(d, ref, b)
    finally:
        k.free()


def test_truncated_handle_rejects_other_f_divergences(gpu_ctx, grid):
    from paper_1708_02845_amd import DDError, Kernel
    g, P = grid
    k = Kernel.load_dense(gpu_ctx, P, tau=1e-3, adjacency=(g.adj_ptr, g.adj_idx))
    try:
        for kind in ("chi2", "hellinger"):
            with pytest.raises(DDError, match="dense handle"):
                k.field(0, kind)
            with pytest.raises(DDError, match="dense handle"):
                k.batch_fields([0, 1], kind)
            with pytest.raises(DDError, match="dense handle"):
                k.plan_path(3, 0, kind, 10)
    finally:
        k.free()
