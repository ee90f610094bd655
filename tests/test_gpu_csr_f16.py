"""GPU checks of the FP16 value form of a truncated handle (csr_values="f16").

The field entry points then read each stored value as FP16 scaled per row by a
power of two.  Checked: the fields against the oracle's truncated fields of the
FP32 input within the stated bound (which includes the FP16 rounding); that
they are exactly the fields of an FP32 handle holding the FP16-rounded values
(the form changes the stored values and nothing else); paths identical to the
oracle's (near-ties are re-decided on the FP32 values); rejections.
"""

import numpy as np
import pytest

from conftest import normwise, within_bound
from oracle import divergence as dv
from oracle import path as op
from workloads import grid_domain
from workloads.seeds import targets_sources

pytestmark = pytest.mark.gpu


def oracle_trunc(P32, tau, relative, t, kind):
    Pt, thr = dv.truncate(np.asarray(P32, dtype=np.float64), tau, relative)
    if kind == "tv":
        return dv.tv_trunc_field(Pt, t)
    return dv.kl_trunc_field(Pt, t, thr)


@pytest.fixture(scope="module")
def grid(gpu_ctx):
    g = grid_domain(81, 3, (0.1, 0.25), seed_id=41)
    return g, g.poisson_kernel().astype(np.float32)


def f16_rounded(val, ptr):
    """The values as the FP16 form stores them: per row, scaled so that the row
    max lies in [2^14, 2^15), rounded to FP16 (nearest even), scaled back."""
    out = np.empty_like(val, dtype=np.float32)
    for x in range(len(ptr) - 1):
        v = val[ptr[x]:ptr[x + 1]].astype(np.float32)
        _, E = np.frexp(np.float64(v.max()))
        e = 15 - int(E)
        h = (v * np.float32(2.0 ** e)).astype(np.float16)
        out[ptr[x]:ptr[x + 1]] = h.astype(np.float32) * np.float32(2.0 ** -e)
    return out


@pytest.mark.parametrize("tau,relative", [(1e-3, True), (1e-5, True), (1e-4, False)])
@pytest.mark.parametrize("kind", ["tv", "kl"])
def test_f16_fields_within_bound(gpu_ctx, grid, tau, relative, kind):
    from paper_1708_02845_amd import Kernel
    g, P = grid
    k = Kernel.load_dense(gpu_ctx, P, tau=tau, tau_relative=relative, csr_values="f16")
    k32 = Kernel.load_dense(gpu_ctx, P, tau=tau, tau_relative=relative)
    try:
        assert k.csr_values == "f16" and k32.csr_values == "f32"
        assert k.hbm_bytes > k32.hbm_bytes
        ts = np.array([0, 400, 2000, g.N - 1] + list(range(5, 5 + 8 * 13, 13)), dtype=np.int32)
        batch, bbounds = k.batch_fields(ts, kind)      # 12 targets: the many-target pass
        batch = batch.cpu().numpy()
        for i, t in enumerate(ts[:4]):
            t = int(t)
            ref = oracle_trunc(P, tau, relative, t, kind)
            d, b = k.field(t, kind)
            d = d.cpu().numpy()
            assert d[t] == 0.0 and batch[i, t] == 0.0
            assert within_bound(d, ref, b), t
            assert within_bound(batch[i], ref, bbounds[i]), t
            # the FP16 rounding dominates: well above the FP32 handle's error,
            # within 2^-10 of the field's scale
            assert normwise(d, ref) <= 2.0 ** -10
    finally:
        k.free()
        k32.free()


@pytest.mark.parametrize("kind", ["tv", "kl"])
def test_f16_form_equals_f32_handle_of_rounded_values(gpu_ctx, grid, kind):
    from paper_1708_02845_amd import Kernel
    g, P = grid
    tau = 1e-4
    keep = P.max(axis=0) > 0
    Pk = P[:, keep]
    Pt, _ = dv.truncate(Pk.astype(np.float64), tau)
    ptr, col, val = dv.csr_from_truncated(Pt)
    val32 = val.astype(np.float32)
    rmax = Pk.astype(np.float64).max(axis=1)
    kh = Kernel.load_csr(gpu_ctx, Pk.shape[0], Pk.shape[1], ptr, col, val32, rmax, tau,
                         csr_values="f16")
    kr = Kernel.load_csr(gpu_ctx, Pk.shape[0], Pk.shape[1], ptr, col, f16_rounded(val32, ptr),
                         rmax, tau)
    try:
        for t in (3, 777, g.N - 2):
            a = kh.field(t, kind)[0].cpu().numpy()
            b = kr.field(t, kind)[0].cpu().numpy()
            assert np.array_equal(a, b), t
        ts = np.arange(10, 10 + 40 * 7, 7, dtype=np.int32)
        a = kh.batch_fields(ts, kind)[0].cpu().numpy()
        b = kr.batch_fields(ts, kind)[0].cpu().numpy()
        assert np.array_equal(a, b)
    finally:
        kh.free()
        kr.free()


@pytest.mark.parametrize("kind", ["kl", "tv"])
def test_f16_paths_identical(gpu_ctx, grid, kind):
    from paper_1708_02845_amd import Kernel
    g, P = grid
    tau = 1e-3
    k = Kernel.load_dense(gpu_ctx, P, tau=tau, adjacency=(g.adj_ptr, g.adj_idx),
                          csr_values="f16")
    try:
        ts, ss = targets_sources(47, g.N, 10)
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
            got, st, _ = k.plan_path(int(s), int(t), kind, 4000)
            assert got == ref
    finally:
        k.free()


def test_f16_rejections(gpu_ctx, grid):
    from paper_1708_02845_amd import DDError, Kernel
    g, P = grid
    # a relative threshold below 2^-28 keeps values FP16 cannot hold at the row's scale
    with pytest.raises(DDError, match="DD_EINVAL"):
        Kernel.load_dense(gpu_ctx, P, tau=1e-9, csr_values="f16")
    with pytest.raises(KeyError):
        Kernel.load_dense(gpu_ctx, P, tau=1e-3, csr_values="bf16")


@pytest.mark.parametrize("T", [200, 257])
@pytest.mark.parametrize("kind", ["tv", "kl"])
def test_f16_many_target_pass_every_target(gpu_ctx, grid, T, kind):
    """FP16 values with more than 128 targets: the four-lists-per-lane instance
    of the many-target pass (257 = one full group of 256 and a ragged one of 1).
    Every target of the batch is checked against the oracle's truncated field
    of the FP32 input within its stated bound."""
    from paper_1708_02845_amd import Kernel
    g, P = grid
    tau = 1e-5
    k = Kernel.load_dense(gpu_ctx, P, tau=tau, csr_values="f16")
    try:
        ts = targets_sources(53, g.N, T)[0].astype(np.int32)
        batch, bounds = k.batch_fields(ts, kind)
        batch = batch.cpu().numpy()
        Pt, thr = dv.truncate(np.asarray(P, dtype=np.float64), tau, True)
        for i, t in enumerate(ts):
            t = int(t)
            ref = dv.tv_trunc_field(Pt, t) if kind == "tv" else dv.kl_trunc_field(Pt, t, thr)
            assert batch[i, t] == 0.0, (i, t)
            assert within_bound(batch[i], ref, bounds[i]), (i, t)
            assert normwise(batch[i], ref) <= 2.0 ** -10, (i, t)
        # a target's field does not depend on the batch it is computed in
        single = k.batch_fields(ts[:8], kind)[0].cpu().numpy()
        assert np.array_equal(single, batch[:8])
    finally:
        k.free()
