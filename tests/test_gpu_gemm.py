"""GPU parity of the batched KL contraction (eq. 35 expanded) against the oracle."""

import numpy as np
import pytest

from conftest import normwise, within_bound
from oracle import divergence as dv
from oracle import path as op
from workloads import build_config, grid_domain
from workloads.seeds import targets_sources

pytestmark = pytest.mark.gpu

FORMS = ["f32", "f16x3", "bf16x3", "f16"]
# normwise tolerance per form: BF16 carries 8 + 8 significant bits per operand
# (about 2^-17 relative per product), FP16 11 + 11 with a scaled B operand.
# The hi-only FP16 form rounds each operand once to 11 bits: every product is
# within 2^-10 + 2^-22 of itself, and the products' absolute sum is at most
# |d| + |H_t| (all log-kernel entries are <= 0), below 2 max|d| on these
# domains, hence 2^-9.
TOL = {"f32": 1e-5, "f16x3": 1e-5, "bf16x3": 1e-4, "f16": 2.0 ** -9}


@pytest.fixture(scope="module")
def grid(gpu_ctx):
    g = grid_domain(71, 2, (0.1, 0.3), seed_id=51)     # N, B not multiples of 128 / 64
    return g, g.poisson_kernel().astype(np.float32)


@pytest.fixture(scope="module", params=FORMS)
def gemm_kernel(request, gpu_ctx, grid):
    from paper_1708_02845_amd import Kernel
    g, P = grid
    k = Kernel.load_dense(gpu_ctx, P, adjacency=(g.adj_ptr, g.adj_idx), gemm_form=request.param)
    yield request.param, k
    k.free()


@pytest.mark.parametrize("T", [1, 5, 32, 33, 64, 70, 128, 200, 256, 300])
def test_batched_kl_matches_oracle(grid, gemm_kernel, T):
    g, P = grid
    form, k = gemm_kernel
    assert k.N % 128 != 0 and k.B % 64 != 0
    ts = targets_sources(51 + T, g.N, T)[0]
    D, bounds = k.batch_fields(ts, "kl")
    D = D.cpu().numpy()
    P64 = P.astype(np.float64)
    # first, middle and last target, and the first and last of each group of 64
    picks = {0, T // 2, T - 1} | {i for g0 in range(64, T, 64) for i in (g0 - 1, g0)}
    for i in sorted(picks):
        ref = dv.kl_field(P64, int(ts[i]))
        assert normwise(D[i], ref) <= TOL[form], (form, T, i)
        assert within_bound(D[i], ref, bounds[i]), (form, T, i)


def test_batch_invariance(grid, gemm_kernel):
    g, P = grid
    form, k = gemm_kernel
    ts = list(targets_sources(77, g.N, 64)[0])
    t = ts[37]
    alone = k.batch_fields([t], "kl")[0].cpu().numpy()[0]
    in_64 = k.batch_fields(ts, "kl")[0].cpu().numpy()[37]
    first = k.batch_fields([t] + ts[1:], "kl")[0].cpu().numpy()[0]
    wide = list(targets_sources(78, g.N, 256)[0])
    wide[200] = t
    in_256 = k.batch_fields(wide, "kl")[0].cpu().numpy()[200]
    assert np.array_equal(alone, in_64)
    assert np.array_equal(alone, first)
    assert np.array_equal(alone, in_256)


def test_paths_on_contraction_fields(grid, gemm_kernel):
    import torch
    g, P = grid
    form, k = gemm_kernel
    ts, ss = targets_sources(52, g.N, 8)
    D, bounds = k.batch_fields(ts, "kl")
    paths, lens, status, rechecks = k.trace_paths(ss, ts, "kl", D, bounds, 4000)
    torch.cuda.synchronize()
    paths, lens, status = paths.cpu().numpy(), lens.cpu().numpy(), status.cpu().numpy()
    P64 = P.astype(np.float64)
    for i in range(len(ts)):
        ref, ref_status = op.steepest_descent_path(dv.kl_field(P64, int(ts[i])), g.adj_ptr,
                                                   g.adj_idx, int(ss[i]), int(ts[i]), 4000)
        assert int(status[i]) == ref_status
        assert list(paths[i, :lens[i]]) == ref


@pytest.mark.parametrize("form", FORMS)
def test_unit_disk_fp64_input(gpu_ctx, form):
    from paper_1708_02845_amd import Kernel
    inst = build_config("disk4096")
    k = Kernel.load_dense(gpu_ctx, inst.P, gemm_form=form)
    try:
        ts = targets_sources(0, inst.N, 16)[0]
        D, bounds = k.batch_fields(ts, "kl")
        D = D.cpu().numpy()
        for i in (0, 7, 15):
            ref = dv.kl_field(inst.P, int(ts[i]))
            assert normwise(D[i], ref) <= TOL[form]
            assert within_bound(D[i], ref, bounds[i])
    finally:
        k.free()


def test_zero_entry_cannot_build_operand(gpu_ctx):
    from paper_1708_02845_amd import DDError, Kernel
    g = np.random.default_rng(3)
    P = g.random((40, 30)) + 0.1
    P[5, 7] = 0.0                    # column 7 is not all-zero, so it is kept
    P /= P.sum(axis=1, keepdims=True)
    with pytest.raises(DDError, match="batched-KL operand"):
        Kernel.load_dense(gpu_ctx, P.astype(np.float32), gemm_form="f16x3")
    k = Kernel.load_dense(gpu_ctx, P.astype(np.float32))     # the streaming form is fine
    k.free()


@pytest.mark.parametrize("form", FORMS)
def test_grid257_batch_of_256(gpu_ctx, form):
    from paper_1708_02845_amd import Kernel
    g = build_config("grid257")
    P = g.poisson_kernel(dtype=np.float32)
    k = Kernel.load_dense(gpu_ctx, P, gemm_form=form)
    try:
        ts = targets_sources(1, g.N, 256)[0]
        D, bounds = k.batch_fields(ts, "kl")
        D = D.cpu().numpy()
        P64 = P.astype(np.float64)
        for i in (0, 63, 64, 191, 255):
            ref = dv.kl_field(P64, int(ts[i]))
            assert normwise(D[i], ref) <= TOL[form]
            assert within_bound(D[i], ref, bounds[i])
    finally:
        k.free()


@pytest.mark.parametrize("form", ["f16x3", "bf16x3", "f16"])
def test_ragged_rows_every_target(gpu_ctx, form):
    """An odd number of 128-row operand tiles with a ragged last tile, batches
    of 65, 128 and 200 targets (ragged and whole target groups): every target
    against the oracle, and fields equal to those computed alone."""
    from paper_1708_02845_amd import Kernel
    g = grid_domain(61, 2, (0.1, 0.3), seed_id=51)
    P = g.poisson_kernel().astype(np.float32)
    k = Kernel.load_dense(gpu_ctx, P, gemm_form=form)
    try:
        assert (-(-k.N // 128)) % 2 == 1 and k.N % 128 != 0
        P64 = P.astype(np.float64)
        for T in (65, 128, 200):
            ts = targets_sources(60 + T, g.N, T)[0]
            ts[-1] = g.N - 1
            D, bounds = k.batch_fields(ts, "kl")
            D = D.cpu().numpy()
            for i in range(T):
                ref = dv.kl_field(P64, int(ts[i]))
                assert normwise(D[i], ref) <= TOL[form], (T, i)
                assert within_bound(D[i], ref, bounds[i]), (T, i)
            for i in (0, 64, T - 1):
                alone = k.batch_fields([int(ts[i])], "kl")[0].cpu().numpy()[0]
                assert np.array_equal(alone, D[i]), (T, i)
    finally:
        k.free()
