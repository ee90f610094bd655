"""GPU parity of the truncated KL through the contraction.

On a truncated handle loaded with a contraction form, KL_tau of many targets
is one MFMA contraction over the floored log-kernel l~_xb = log max(P_xb,
phi_x) - o_x: the stored value when kept, the row's floor otherwise, which
is the reading of the truncated KL (Section V, "Precision") the oracle's
kl_trunc_field evaluates.  Checked against the oracle within the stated bound
and the form's normwise tolerance, against the pass over the stored rows, for
batches past one launch, relative and absolute thresholds, FP64 input, and
through the paths; and the rejections.
"""

import numpy as np
import pytest

from conftest import normwise, within_bound
from oracle import divergence as dv
from oracle import path as op
from workloads import grid_domain
from workloads.seeds import targets_sources

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "f16x3": 1e-5, "bf16x3": 1e-4}


def oracle_trunc_kl(P, tau, relative, t):
    Pt, thr = dv.truncate(np.asarray(P, dtype=np.float64), tau, relative)
    return dv.kl_trunc_field(Pt, t, thr)


@pytest.fixture(scope="module")
def grid(gpu_ctx):
    g = grid_domain(81, 3, (0.1, 0.25), seed_id=41)
    return g, g.poisson_kernel().astype(np.float32)


@pytest.mark.parametrize("form", ["f16x3", "f32", "bf16x3"])
@pytest.mark.parametrize("tau,relative", [(1e-3, True), (1e-5, True), (1e-4, False)])
def test_matches_oracle(gpu_ctx, grid, form, tau, relative):
    from paper_1708_02845_amd import Kernel
    g, P = grid
    k = Kernel.load_dense(gpu_ctx, P, tau=tau, tau_relative=relative, gemm_form=form)
    try:
        assert k.is_csr and k.gemm_form != -1
        ts = targets_sources(91, g.N, 70)[0]
        ts[0], ts[-1] = 0, g.N - 1
        d, bounds = k.batch_fields(ts, "kl")
        d = d.cpu().numpy()
        for i in (0, 1, 31, 32, 63, 64, 69):
            ref = oracle_trunc_kl(P, tau, relative, int(ts[i]))
            assert normwise(d[i], ref) <= TOL[form], (form, i)
            assert within_bound(d[i], ref, bounds[i]), (form, i)
    finally:
        k.free()


def test_agrees_with_pass_over_stored_rows(gpu_ctx, grid):
    from paper_1708_02845_amd import Kernel
    g, P = grid
    kc = Kernel.load_dense(gpu_ctx, P, tau=1e-5, gemm_form="f16x3")
    ks = Kernel.load_dense(gpu_ctx, P, tau=1e-5)
    try:
        ts = targets_sources(92, g.N, 300)[0]        # two launches: 256 + 44
        a, ba = kc.batch_fields(ts, "kl")
        b, bb = ks.batch_fields(ts, "kl")
        a, b = a.cpu().numpy().astype(np.float64), b.cpu().numpy().astype(np.float64)
        for i in range(0, 300, 13):
            err = np.abs(a[i] - b[i])
            assert np.all(err <= ba[i][0] + bb[i][0] + (ba[i][1] + bb[i][1]) * np.abs(b[i])
                          + 2.0 ** -23 * np.abs(b[i])), i
        # TV on the same handle still takes the pass over the stored rows
        t1, _ = kc.batch_fields(ts[:20], "tv")
        t2, _ = ks.batch_fields(ts[:20], "tv")
        assert np.array_equal(t1.cpu().numpy(), t2.cpu().numpy())
    finally:
        kc.free()
        ks.free()


def test_fp64_input(gpu_ctx, grid):
    from paper_1708_02845_amd import Kernel
    g, _ = grid
    P64 = g.poisson_kernel()
    k = Kernel.load_dense(gpu_ctx, P64, tau=1e-4, gemm_form="f16x3")
    try:
        ts = targets_sources(93, g.N, 16)[0]
        d, bounds = k.batch_fields(ts, "kl")
        d = d.cpu().numpy()
        for i in (0, 7, 15):
            ref = oracle_trunc_kl(P64, 1e-4, True, int(ts[i]))
            assert normwise(d[i], ref) <= 1e-5
            assert within_bound(d[i], ref, bounds[i])
    finally:
        k.free()


def test_paths_on_floored_contraction_fields(gpu_ctx, grid):
    from paper_1708_02845_amd import Kernel
    g, P = grid
    tau = 1e-3
    k = Kernel.load_dense(gpu_ctx, P, tau=tau, adjacency=(g.adj_ptr, g.adj_idx), gemm_form="f16x3")
    try:
        ts, ss = targets_sources(94, g.N, 10)
        fields, bounds = k.batch_fields(ts, "kl")
        paths, lens, status, _ = k.trace_paths(ss, ts, "kl", fields, bounds, 4000)
        paths, lens, status = paths.cpu().numpy(), lens.cpu().numpy(), status.cpu().numpy()
        for i, (s, t) in enumerate(zip(ss, ts)):
            ref_field = oracle_trunc_kl(P, tau, True, int(t))
            ref, ref_status = op.steepest_descent_path(ref_field, g.adj_ptr, g.adj_idx, int(s),
                                                       int(t), 4000)
            assert int(status[i]) == ref_status
            assert paths[i, :lens[i]].tolist() == ref
    finally:
        k.free()


def test_rejections(gpu_ctx, grid):
    from paper_1708_02845_amd import DDError, Kernel
    g, P = grid
    with pytest.raises(DDError, match="FP32 stored values"):
        Kernel.load_dense(gpu_ctx, P, tau=1e-3, gemm_form="f16x3", csr_values="f16")


@pytest.mark.parametrize("T", [1, 33])
def test_small_and_ragged_batches(gpu_ctx, grid, T):
    """One target (32 padded target slots) and 33 targets (a ragged group of 64)
    through the floored contraction, every target against the oracle."""
    from paper_1708_02845_amd import Kernel
    g, P = grid
    k = Kernel.load_dense(gpu_ctx, P, tau=1e-4, gemm_form="f16x3")
    try:
        ts = targets_sources(95 + T, g.N, T)[0]
        d, bounds = k.batch_fields(ts, "kl")
        d = d.cpu().numpy()
        for i in range(T):
            ref = oracle_trunc_kl(P, 1e-4, True, int(ts[i]))
            assert normwise(d[i], ref) <= 1e-5, i
            assert within_bound(d[i], ref, bounds[i]), i
    finally:
        k.free()
