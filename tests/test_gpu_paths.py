"""GPU steepest-descent paths: identical vertex sequences to the oracle's."""

import numpy as np
import pytest

from oracle import divergence as dv
from oracle import path as op
from workloads import build_config, grid_domain
from workloads.seeds import targets_sources

pytestmark = pytest.mark.gpu

STATUS = {op.REACHED: "reached", op.STUCK: "stuck", op.MAX_STEPS: "max_steps"}


def oracle_path(P, adj_ptr, adj_idx, s, t, kind, max_steps):
    P64 = np.asarray(P, dtype=np.float64)
    d = dv.field(P64, t, kind)
    path, status = op.steepest_descent_path(d, adj_ptr, adj_idx, s, t, max_steps)
    return path, STATUS[status]


@pytest.fixture(scope="module")
def disk(gpu_ctx):
    from paper_1708_02845_amd import Kernel
    inst = build_config("disk4096")
    k = Kernel.load_dense(gpu_ctx, inst.P, adjacency=(inst.adj_ptr, inst.adj_idx))
    yield inst, k
    k.free()


@pytest.mark.parametrize("kind", ["kl", "tv", "chi2", "hellinger", ("power", 3), ("alpha", 0.5)])
def test_disk_paths_identical(disk, kind):
    inst, k = disk
    ts, ss = targets_sources(0, inst.N, 8)
    for s, t in zip(ss, ts):
        got, status, _ = k.plan_path(int(s), int(t), kind, 4000)
        ref, ref_status = oracle_path(inst.P, inst.adj_ptr, inst.adj_idx, int(s), int(t), kind, 4000)
        assert status == ref_status == "reached"
        assert got == ref


@pytest.fixture(scope="module")
def grid(gpu_ctx):
    from paper_1708_02845_amd import Kernel
    g = grid_domain(97, 3, (0.1, 0.25), seed_id=31)
    P = g.poisson_kernel().astype(np.float32)
    k = Kernel.load_dense(gpu_ctx, P, adjacency=(g.adj_ptr, g.adj_idx))
    yield g, P, k
    k.free()


@pytest.mark.parametrize("kind", ["kl", "tv", "chi2", "hellinger"])
def test_grid_paths_identical(grid, kind):
    g, P, k = grid
    ts, ss = targets_sources(31, g.N, 6)
    for s, t in zip(ss, ts):
        got, status, _ = k.plan_path(int(s), int(t), kind, 4000)
        ref, ref_status = oracle_path(P, g.adj_ptr, g.adj_idx, int(s), int(t), kind, 4000)
        assert status == ref_status
        assert got == ref


def test_step_cap_and_source_equals_target(grid):
    g, P, k = grid
    t, s = 10, g.N - 10
    got, status, _ = k.plan_path(s, t, "kl", 3)
    ref, ref_status = oracle_path(P, g.adj_ptr, g.adj_idx, s, t, "kl", 3)
    assert status == ref_status == "max_steps" and got == ref and len(got) == 4
    got, status, _ = k.plan_path(t, t, "kl", 10)
    assert got == [t] and status == "reached"


def test_batched_trace_equals_single_queries(grid):
    import torch
    g, P, k = grid
    ts, ss = targets_sources(32, g.N, 5)
    fields, bounds = k.batch_fields(ts, "kl")
    paths, lens, status, rechecks = k.trace_paths(ss, ts, "kl", fields, bounds, 500)
    torch.cuda.synchronize()
    paths, lens, status = paths.cpu().numpy(), lens.cpu().numpy(), status.cpu().numpy()
    for i in range(len(ts)):
        single, st, _ = k.plan_path(int(ss[i]), int(ts[i]), "kl", 500)
        assert list(paths[i, :lens[i]]) == single
        assert np.all(paths[i, lens[i]:] == -1)
        assert {0: "reached", 1: "stuck", 2: "max_steps"}[int(status[i])] == st


def test_planted_minimum_is_stuck(grid):
    import torch
    g, P, k = grid
    # a crafted field: distance to vertex t along the grid index, with a pit
    t = g.N - 1
    f = np.arange(g.N, dtype=np.float32)[::-1].copy() + 1.0
    f[t] = 0.0
    pit = g.N // 2
    f[pit] = 0.5
    nb = g.adj_idx[g.adj_ptr[pit]:g.adj_ptr[pit + 1]]
    s = int(nb[0])
    fields = torch.from_numpy(f).cuda().reshape(1, -1)
    paths, lens, status, _ = k.trace_paths([s], [t], "kl", fields, [(0.0, 0.0)], 100)
    torch.cuda.synchronize()
    assert int(status[0]) == 1
    assert paths[0, :int(lens[0])].cpu().tolist() == [s, pit]


def test_path_without_adjacency_is_rejected(gpu_ctx):
    from paper_1708_02845_amd import DDError, Kernel
    P = np.full((4, 4), 0.25, dtype=np.float32)
    k = Kernel.load_dense(gpu_ctx, P)
    try:
        with pytest.raises(DDError, match="without adjacency"):
            k.plan_path(0, 1, "kl", 10)
    finally:
        k.free()


def test_grid257_paths(gpu_ctx):
    from paper_1708_02845_amd import Kernel
    g = build_config("grid257")
    P = g.poisson_kernel(dtype=np.float32)
    k = Kernel.load_dense(gpu_ctx, P, adjacency=(g.adj_ptr, g.adj_idx))
    try:
        ts, ss = targets_sources(1, g.N, 2)
        for kind in ("kl", "tv", "chi2", "hellinger"):
            for s, t in zip(ss, ts):
                got, status, _ = k.plan_path(int(s), int(t), kind, 4000)
                ref, ref_status = oracle_path(P, g.adj_ptr, g.adj_idx, int(s), int(t), kind, 4000)
                assert status == ref_status
                assert got == ref
    finally:
        k.free()


ALL_KINDS = ["kl", "tv", "chi2", "hellinger"]


def test_exact_tie_goes_to_lowest_id(gpu_ctx):
    # vertices 2 and 3 have identical rows, so their distances tie exactly in
    # FP32 and in FP64: the walk takes the lower id, after an FP64 re-decision
    from paper_1708_02845_amd import Kernel
    P = np.array([[0.7, 0.1, 0.1, 0.1],
                  [0.1, 0.3, 0.3, 0.3],
                  [0.4, 0.2, 0.2, 0.2],
                  [0.4, 0.2, 0.2, 0.2]], dtype=np.float32)
    adj_ptr = np.array([0, 2, 4, 6, 8], dtype=np.int64)
    adj_idx = np.array([2, 3, 2, 3, 0, 1, 0, 1], dtype=np.int32)
    k = Kernel.load_dense(gpu_ctx, P, adjacency=(adj_ptr, adj_idx))
    try:
        for kind in ALL_KINDS:
            got, status, rechecks = k.plan_path(1, 0, kind, 10)
            ref, ref_status = oracle_path(P, adj_ptr, adj_idx, 1, 0, kind, 10)
            assert ref == [1, 2, 0] and got == ref and status == ref_status == "reached"
            assert rechecks >= 1
    finally:
        k.free()


def test_high_degree_vertices(gpu_ctx):
    # a hub adjacent to 63 vertices (padded width 64: every lane of the wave
    # holds a neighbour) and a ring through the rest
    from paper_1708_02845_amd import Kernel
    g = np.random.default_rng(11)
    N, B = 90, 40
    P = (g.random((N, B)) ** 3 + 1e-4).astype(np.float64)
    P /= P.sum(axis=1, keepdims=True)
    P = P.astype(np.float32)
    nbrs = [set() for _ in range(N)]
    for u in range(1, 64):
        nbrs[0].add(u)
        nbrs[u].add(0)
    for u in range(1, N):
        w = u + 1 if u + 1 < N else 1
        nbrs[u].add(w)
        nbrs[w].add(u)
    order = [sorted(s) for s in nbrs]
    adj_ptr = np.cumsum([0] + [len(o) for o in order]).astype(np.int64)
    adj_idx = np.concatenate([np.array(o, dtype=np.int32) for o in order])
    k = Kernel.load_dense(gpu_ctx, P, adjacency=(adj_ptr, adj_idx))
    try:
        pairs = [(70, 5), (0, 40), (85, 63), (12, 77), (33, 0)]
        for kind in ALL_KINDS:
            for s, t in pairs:
                got, status, _ = k.plan_path(s, t, kind, 200)
                ref, ref_status = oracle_path(P, adj_ptr, adj_idx, s, t, kind, 200)
                assert got == ref and status == ref_status
    finally:
        k.free()
