"""Level-1 re-decisions of KL walks (the steepest-descent rule of Section IV,
decided first on FP32 hardware logarithms summed in FP64 with a stated bound,
then in FP64 where that bound does not settle the step): the device passes
the exhaustive log2 check the bound rests on, and paths, statuses and
re-decision counts are the same with level 1 on and off, on FP32 and FP64
matrices, on streamed and on contraction fields; sampled paths equal the
oracle's."""

import numpy as np
import pytest

from oracle import divergence as dv
from oracle import path as op
from workloads import build_config
from workloads.seeds import targets_sources

pytestmark = pytest.mark.gpu


def test_hardware_log2_meets_the_assumed_bound(gpu_ctx):
    on, (ratio, rel) = gpu_ctx.path_level1()
    # every FP32 value in [2^-126, 1]: |L(x) - log2 x| <= 2^-22 |log2 x| + 2^-40
    assert 0.0 <= ratio <= 1.0, (ratio, rel)
    assert on


def _trace(k, ss, ts, fields, bounds):
    import torch
    paths, lens, status, rechecks = k.trace_paths(ss, ts, "kl", fields, bounds, 4000)
    torch.cuda.synchronize()
    lens = lens.cpu().numpy()
    paths = paths.cpu().numpy()
    return ([paths[i, :lens[i]].tolist() for i in range(len(ts))], status.cpu().numpy(),
            rechecks.cpu().numpy())


def _both(ctx, k, ss, ts, fields, bounds):
    assert ctx.path_level1()[0]
    on = _trace(k, ss, ts, fields, bounds)
    try:
        assert not ctx.path_level1(False)[0]
        off = _trace(k, ss, ts, fields, bounds)
    finally:
        assert ctx.path_level1(True)[0]
    return on, off


def _oracle(P, adj_ptr, adj_idx, s, t):
    d = dv.field(np.asarray(P, dtype=np.float64), t, "kl")
    path, status = op.steepest_descent_path(d, adj_ptr, adj_idx, s, t, 4000)
    return path, status


@pytest.fixture(scope="module")
def grid257():
    g = build_config("grid257")
    return g, g.poisson_kernel(dtype=np.float32)


@pytest.mark.parametrize("form", [None, "f16x3"])
def test_level1_leaves_grid_paths_unchanged(gpu_ctx, grid257, form):
    from paper_1708_02845_amd import Kernel
    g, P = grid257
    k = Kernel.load_dense(gpu_ctx, P, adjacency=(g.adj_ptr, g.adj_idx), gemm_form=form)
    try:
        ts, ss = targets_sources(4, g.N, 48)
        fields, bounds = k.batch_fields(ts, "kl")
        (p1, s1, r1), (p0, s0, r0) = _both(gpu_ctx, k, ss, ts, fields, bounds)
        assert p1 == p0 and np.array_equal(s1, s0) and np.array_equal(r1, r0)
        assert r1.sum() > 0
        for i in (int(np.argmax(r1)), 0):
            ref, st = _oracle(P, g.adj_ptr, g.adj_idx, int(ss[i]), int(ts[i]))
            assert p1[i] == ref and int(s1[i]) == st
    finally:
        k.free()


def test_level1_leaves_fp64_matrix_paths_unchanged(gpu_ctx):
    # FP64 rows: level-1 rounds q and p to FP32 and adds that to its bound
    from paper_1708_02845_amd import Kernel
    inst = build_config("disk4096")
    k = Kernel.load_dense(gpu_ctx, inst.P, adjacency=(inst.adj_ptr, inst.adj_idx),
                          gemm_form="f16x3")
    try:
        ts, ss = targets_sources(5, inst.N, 64)
        fields, bounds = k.batch_fields(ts, "kl")
        (p1, s1, r1), (p0, s0, r0) = _both(gpu_ctx, k, ss, ts, fields, bounds)
        assert p1 == p0 and np.array_equal(s1, s0) and np.array_equal(r1, r0)
        assert r1.sum() > 0
        for i in (int(np.argmax(r1)), 1):
            ref, st = _oracle(inst.P, inst.adj_ptr, inst.adj_idx, int(ss[i]), int(ts[i]))
            assert p1[i] == ref and int(s1[i]) == st
    finally:
        k.free()


def test_level1_switch_is_checked(gpu_ctx):
    from paper_1708_02845_amd import DDError
    from paper_1708_02845_amd import _lib as L
    import ctypes as C
    lib = L.load()
    assert lib.dd_path_level1(gpu_ctx.handle, 2, None, None) == L.DD_EINVAL
    with pytest.raises(DDError, match="DD_EINVAL"):
        L.check(lib.dd_path_level1(gpu_ctx.handle, -2, None, None))
    on = C.c_int()
    assert lib.dd_path_level1(gpu_ctx.handle, -1, C.byref(on), None) == L.DD_OK and on.value == 1


def _on_demand(k, ss, ts, **kw):
    import torch
    paths, lens, status, evals = k.trace_paths_on_demand(ss, ts, "kl", 4000, **kw)
    torch.cuda.synchronize()
    lens = lens.cpu().numpy()
    paths = paths.cpu().numpy()
    return ([paths[i, :lens[i]].tolist() for i in range(len(ts))], status.cpu().numpy(),
            evals.cpu().numpy())


@pytest.mark.parametrize("tau", [0.0, 1e-3])
def test_level1_leaves_on_demand_walks_unchanged(gpu_ctx, grid257, tau):
    # the on-demand walk (no field) decides every step on row values: level 1
    # first, FP64 where it does not settle the step
    from paper_1708_02845_amd import Kernel
    g, P = grid257
    k = Kernel.load_dense(gpu_ctx, P, adjacency=(g.adj_ptr, g.adj_idx))
    try:
        ts, ss = targets_sources(6, g.N, 24)
        on = _on_demand(k, ss, ts, target_tau=tau)
        try:
            assert not gpu_ctx.path_level1(False)[0]
            off = _on_demand(k, ss, ts, target_tau=tau)
        finally:
            assert gpu_ctx.path_level1(True)[0]
        assert on[0] == off[0] and np.array_equal(on[1], off[1]) and np.array_equal(on[2], off[2])
        if tau == 0.0:
            fields, bounds = k.batch_fields(ts[:4], "kl")
            walked = _trace(k, ss[:4], ts[:4], fields, bounds)
            assert on[0][:4] == walked[0] and np.array_equal(on[1][:4], walked[1])
            ref, st = _oracle(P, g.adj_ptr, g.adj_idx, int(ss[0]), int(ts[0]))
            assert on[0][0] == ref and int(on[1][0]) == st
    finally:
        k.free()


def test_level1_on_demand_fp64_matrix(gpu_ctx):
    from paper_1708_02845_amd import Kernel
    inst = build_config("disk4096")
    k = Kernel.load_dense(gpu_ctx, inst.P, adjacency=(inst.adj_ptr, inst.adj_idx))
    try:
        ts, ss = targets_sources(7, inst.N, 16)
        on = _on_demand(k, ss, ts)
        try:
            gpu_ctx.path_level1(False)
            off = _on_demand(k, ss, ts)
        finally:
            gpu_ctx.path_level1(True)
        assert on[0] == off[0] and np.array_equal(on[1], off[1])
        ref, st = _oracle(inst.P, inst.adj_ptr, inst.adj_idx, int(ss[3]), int(ts[3]))
        assert on[0][3] == ref and int(on[1][3]) == st
    finally:
        k.free()
