"""GPU parity of the many-target pass over truncated (CSR) rows.

From 8 targets up, dd_batch_distance_fields on a truncated handle runs one
pass over the stored rows for up to 256 targets (1, 2 or 4 targets per lane),
in place of one streaming pass per target.  Its fields are checked against the
oracle's truncated fields, against the single-target pass, across batch
compositions, and through the paths traced on them.
"""

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


def batch_targets(N, T, seed):
    return np.random.default_rng(seed).integers(0, N, size=T).astype(np.int32)


# T = 8 and 70 and 130 and 300 take 1, 2, 4 targets per lane and two launches
@pytest.mark.parametrize("T", [8, 70, 130, 300])
@pytest.mark.parametrize("tau,relative", [(1e-3, True), (1e-6, True), (1e-4, False)])
@pytest.mark.parametrize("kind", ["tv", "kl"])
def test_batch_matches_oracle(gpu_ctx, grid, T, tau, relative, kind):
    from paper_1708_02845_amd import Kernel
    g, P = grid
    k = Kernel.load_dense(gpu_ctx, P, tau=tau, tau_relative=relative)
    try:
        ts = batch_targets(g.N, T, 1000 + T)
        ts[0] = 0
        ts[-1] = g.N - 1
        d, bounds = k.batch_fields(ts, kind)
        d = d.cpu().numpy()
        # the oracle on a sample of slots: both ends, lane and launch boundaries
        for i in sorted({0, 1, 7, 63, 64, 127, 128, 255, 256, T - 1} & set(range(T))):
            t = int(ts[i])
            ref = oracle_trunc(P, tau, relative, t, kind)
            assert d[i, t] == 0.0
            assert normwise(d[i], ref) <= TOL, (i, t)
            assert within_bound(d[i], ref, bounds[i]), (i, t)
    finally:
        k.free()


@pytest.mark.parametrize("kind", ["tv", "kl"])
def test_batch_agrees_with_single_target_pass(gpu_ctx, grid, kind):
    from paper_1708_02845_amd import Kernel
    g, P = grid
    k = Kernel.load_dense(gpu_ctx, P, tau=1e-5)
    try:
        ts = batch_targets(g.N, 40, 7)
        d, bounds = k.batch_fields(ts, kind)
        d = d.cpu().numpy()
        for i, t in enumerate(ts):
            s, bs = k.field(int(t), kind)
            s = s.cpu().numpy().astype(np.float64)
            err = np.abs(d[i] - s)
            assert np.all(err <= bounds[i][0] + bs[0] + (bounds[i][1] + bs[1]) * np.abs(s) +
                          2.0 ** -23 * np.abs(s))
    finally:
        k.free()


@pytest.mark.parametrize("kind", ["tv", "kl"])
def test_batch_composition_invariance(gpu_ctx, grid, kind):
    """A target's field is bit-identical whatever else is in the batch and at
    whichever slot, for every batch that takes the many-target pass."""
    from paper_1708_02845_amd import Kernel
    g, P = grid
    k = Kernel.load_dense(gpu_ctx, P, tau=1e-4)
    try:
        t = 1234
        small = batch_targets(g.N, 8, 3)
        small[5] = t
        big = batch_targets(g.N, 256, 4)
        big[200] = t
        mid = batch_targets(g.N, 100, 5)
        mid[99] = t
        a = k.batch_fields(small, kind)[0][5].cpu().numpy()
        b = k.batch_fields(big, kind)[0][200].cpu().numpy()
        c = k.batch_fields(mid, kind)[0][99].cpu().numpy()
        assert np.array_equal(a, b) and np.array_equal(a, c)
        # duplicates in one batch give identical rows
        dup = np.array([t] * 9, dtype=np.int32)
        e = k.batch_fields(dup, kind)[0].cpu().numpy()
        assert all(np.array_equal(e[i], a) for i in range(9))
    finally:
        k.free()


@pytest.mark.parametrize("kind", ["kl", "tv"])
def test_paths_on_batched_truncated_fields(gpu_ctx, grid, kind):
    from paper_1708_02845_amd import Kernel
    g, P = grid
    tau = 1e-3
    k = Kernel.load_dense(gpu_ctx, P, tau=tau, adjacency=(g.adj_ptr, g.adj_idx))
    try:
        ts, ss = targets_sources(43, g.N, 12)
        fields, bounds = k.batch_fields(ts, kind)
        paths, lens, status, _ = k.trace_paths(ss, ts, kind, fields, bounds, 4000)
        paths = paths.cpu().numpy()
        lens = lens.cpu().numpy()
        status = status.cpu().numpy()
        for i, (s, t) in enumerate(zip(ss, ts)):
            ref_field = oracle_trunc(P, tau, True, int(t), kind)
            ref, ref_status = op.steepest_descent_path(ref_field, g.adj_ptr, g.adj_idx, int(s),
                                                       int(t), 4000)
            assert int(status[i]) == ref_status
            assert paths[i, :lens[i]].tolist() == ref
    finally:
        k.free()


@pytest.mark.parametrize("kind", ["tv", "kl"])
def test_grid257_batch_full_size(gpu_ctx, kind):
    """The 257^2 domain truncated at 1e-6 relative, 64 targets in one pass;
    the oracle on two of them."""
    from paper_1708_02845_amd import Kernel
    g = build_config("grid257")
    P = g.poisson_kernel(dtype=np.float32)
    k = Kernel.load_dense(gpu_ctx, P, tau=1e-6)
    try:
        ts = batch_targets(g.N, 64, 11)
        d, bounds = k.batch_fields(ts, kind)
        for i in (0, 63):
            t = int(ts[i])
            got = d[i].cpu().numpy()
            ref = oracle_trunc(P, 1e-6, True, t, kind)
            assert normwise(got, ref) <= TOL and within_bound(got, ref, bounds[i])
    finally:
        k.free()
