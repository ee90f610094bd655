"""GPU parity of the streaming fields against the FP64 oracle: TV and KL
(eqs. 34, 35) and the chi-squared and Hellinger f-divergences (Section VI).

Gate: normwise error max|d_hat - d| / max|d| <= 1e-5 and every entry inside
the bound the library states for that field.
"""

import numpy as np
import pytest

from conftest import normwise, within_bound
from oracle import divergence as dv
from workloads import build_config, grid_domain
from workloads.seeds import targets_sources

pytestmark = pytest.mark.gpu

TOL = 1e-5


def random_kernel(N, B, seed):
    g = np.random.default_rng(seed)
    P = g.random((N, B)) ** 2 + 1e-3
    P /= P.sum(axis=1, keepdims=True)
    return P.astype(np.float32)


ORACLE = {"tv": dv.tv_field, "kl": dv.kl_field, "chi2": dv.chi2_field,
          "hellinger": dv.hellinger_field}
KINDS = list(ORACLE)


def oracle_field(P, t, kind):
    return ORACLE[kind](np.asarray(P, dtype=np.float64), t)


def run_field(kern, t, kind):
    d, b = kern.field(t, kind)
    return d.cpu().numpy(), b


@pytest.mark.parametrize("B", [1, 3, 5, 63, 64, 65, 255, 256, 257, 511, 1023, 1024, 1025, 4099])
@pytest.mark.parametrize("kind", KINDS)
def test_ragged_widths(gpu_ctx, B, kind):
    from paper_1708_02845_amd import Kernel
    N = 37
    P = random_kernel(N, B, seed=B)
    k = Kernel.load_dense(gpu_ctx, P)
    try:
        for t in (0, 5, N - 1):
            d, b = run_field(k, t, kind)
            ref = oracle_field(P, t, kind)
            assert d[t] == 0.0
            assert normwise(d, ref) <= TOL
            assert within_bound(d, ref, b)
    finally:
        k.free()


@pytest.mark.parametrize("N", [1, 2, 3, 17, 1000, 4097])
def test_ragged_row_counts(gpu_ctx, N):
    from paper_1708_02845_amd import Kernel
    P = random_kernel(N, 300, seed=N)
    k = Kernel.load_dense(gpu_ctx, P)
    try:
        for kind in KINDS:
            d, b = run_field(k, N // 2, kind)
            ref = oracle_field(P, N // 2, kind)
            assert normwise(d, ref) <= TOL and within_bound(d, ref, b)
    finally:
        k.free()


@pytest.fixture(scope="module")
def disk_kernel(gpu_ctx):
    from paper_1708_02845_amd import Kernel
    inst = build_config("disk4096")
    k = Kernel.load_dense(gpu_ctx, inst.P, adjacency=(inst.adj_ptr, inst.adj_idx))
    yield inst, k
    k.free()


@pytest.mark.parametrize("kind", KINDS)
def test_unit_disk_fp64_input(disk_kernel, kind):
    inst, k = disk_kernel
    assert (k.N, k.B) == (4096, 256)
    targets, _ = targets_sources(0, inst.N, 4)
    for t in targets:
        d, b = run_field(k, int(t), kind)
        ref = oracle_field(inst.P, int(t), kind)
        assert d[t] == 0.0
        assert normwise(d, ref) <= TOL
        assert within_bound(d, ref, b)


@pytest.fixture(scope="module")
def grid65(gpu_ctx):
    from paper_1708_02845_amd import Kernel
    g = grid_domain(65, 2, (0.1, 0.3), seed_id=21)
    P = g.poisson_kernel().astype(np.float32)
    k = Kernel.load_dense(gpu_ctx, P, adjacency=(g.adj_ptr, g.adj_idx))
    yield g, P, k
    k.free()


def test_zero_columns_are_dropped(grid65):
    g, P, k = grid65
    assert k.B_in == g.K and k.B == g.K - 4


@pytest.mark.parametrize("kind", KINDS)
def test_small_grid_fields(grid65, kind):
    g, P, k = grid65
    for t in (0, 123, g.N - 1):
        d, b = run_field(k, t, kind)
        ref = oracle_field(P, t, kind)
        assert normwise(d, ref) <= TOL and within_bound(d, ref, b)


def test_runs_are_bitwise_deterministic(grid65):
    g, P, k = grid65
    a, _ = run_field(k, 77, "kl")
    b, _ = run_field(k, 77, "kl")
    assert np.array_equal(a, b)


def test_streaming_batch_equals_single_fields(grid65):
    g, P, k = grid65
    ts = [3, 77, 900, 3]
    for kind in KINDS:
        D, bounds = k.batch_fields(ts, kind)
        D = D.cpu().numpy()
        for i, t in enumerate(ts):
            d, b = run_field(k, t, kind)
            assert np.array_equal(D[i], d)
            assert bounds[i] == b


def test_device_resident_input_matches_host_input(gpu_ctx, grid65):
    import torch
    from paper_1708_02845_amd import Kernel
    g, P, k = grid65
    kd = Kernel.load_dense(gpu_ctx, torch.from_numpy(P).cuda())
    try:
        for kind in KINDS:
            assert np.array_equal(run_field(kd, 200, kind)[0], run_field(k, 200, kind)[0])
    finally:
        kd.free()


def test_invalid_inputs_are_rejected(gpu_ctx, grid65):
    from paper_1708_02845_amd import DDError, Kernel
    g, P, k = grid65
    bad = random_kernel(10, 20, 1)
    for mutate in (lambda a: a.__setitem__((3, 4), -1e-3),
                   lambda a: a.__setitem__((3, 4), np.nan),
                   lambda a: a.__setitem__((3, 4), a[3, 4] + 0.01),
                   lambda a: a.__setitem__((2, 2), 1e-40)):
        a = bad.copy()
        mutate(a)
        with pytest.raises(DDError, match="DD_EINVAL"):
            Kernel.load_dense(gpu_ctx, a)
    with pytest.raises(DDError, match="DD_EINVAL"):
        k.field(g.N, "kl")
    with pytest.raises(DDError, match="DD_EINVAL"):
        k.field(-1, "tv")
    with pytest.raises(ValueError):
        k.field(0, "jensen-shannon")
    with pytest.raises(DDError, match="DD_EINVAL"):
        k.field(0, 4)
    with pytest.raises(DDError, match="DD_EINVAL"):
        Kernel.load_dense(gpu_ctx, np.zeros((4, 8), dtype=np.float32), validate=False)


@pytest.fixture(scope="module")
def grid257(gpu_ctx):
    """The 257x257, 3-obstacle workload at its full size (FP32 dense)."""
    from paper_1708_02845_amd import Kernel
    g = build_config("grid257")
    P = g.poisson_kernel(dtype=np.float32)
    k = Kernel.load_dense(gpu_ctx, P, adjacency=(g.adj_ptr, g.adj_idx))
    yield g, P, k
    k.free()


@pytest.mark.parametrize("kind", KINDS)
def test_grid257_full_size(grid257, kind):
    g, P, k = grid257
    t = int(targets_sources(1, g.N, 1)[0][0])
    d, b = run_field(k, t, kind)
    ref = oracle_field(P, t, kind)
    assert d[t] == 0.0
    assert normwise(d, ref) <= TOL
    assert within_bound(d, ref, b)


def test_chi2_off_support_rows_are_infinite(gpu_ctx):
    # a target row with zeros: rows with mass there have chi2 = +inf, the
    # rest are finite and inside the bound; Hellinger stays finite.
    from paper_1708_02845_amd import Kernel
    P = random_kernel(50, 200, seed=7)
    P[4, 10:30] = 0.0
    P[9, :] = P[4, :]
    P[9, 0] += 1e-3
    P[4] /= P[4].sum(dtype=np.float64)
    P[9] /= P[9].sum(dtype=np.float64)
    k = Kernel.load_dense(gpu_ctx, P)
    try:
        d, b = run_field(k, 4, "chi2")
        ref = oracle_field(P, 4, "chi2")
        inf = np.isinf(ref)
        assert inf.sum() == 48 and np.array_equal(np.isinf(d), inf)
        assert np.isfinite(d[9]) and within_bound(d[~inf], ref[~inf], b)
        h, bh = run_field(k, 4, "hellinger")
        href = oracle_field(P, 4, "hellinger")
        assert np.isfinite(h).all() and within_bound(h, href, bh) and h.max() <= 2.0
    finally:
        k.free()


def test_hellinger_bound_is_relative_near_the_target(grid65):
    # the cancellation-free form: no absolute floor on FP32 input, so even the
    # smallest nonzero values (neighbours of the target) carry a relative bound
    g, P, k = grid65
    t = 500
    d, b = run_field(k, t, "hellinger")
    assert b[0] < 1e-250
    ref = oracle_field(P, t, "hellinger")
    nz = ref > 0
    assert np.max(np.abs(d[nz] - ref[nz]) / ref[nz]) <= 2 * b[1]


FAMILY = [("power", 1), ("power", 3), ("power", 4), ("power", 16),
          ("alpha", -0.875), ("alpha", -0.25), ("alpha", 0.0), ("alpha", 0.5), ("alpha", 0.875)]


def check_member(d, ref, b, what):
    # values beyond the FP32 range can only come back as +inf (|1-u|^16 on the
    # grid reaches 1e110); the rest meet the tolerance and the bound
    big = ref > np.finfo(np.float32).max
    assert np.all(np.isinf(d[big])), what
    fin = ~big
    assert np.all(np.isfinite(d[fin])), what
    assert normwise(d[fin], ref[fin]) <= TOL and within_bound(d[fin], ref[fin], b), what


@pytest.mark.parametrize("member", FAMILY)
def test_family_members_match_oracle(grid65, disk_kernel, member):
    g, P, k = grid65
    for t in (0, 321, g.N - 1):
        d, b = k.field(t, member)
        d = d.cpu().numpy()
        ref = dv.field(P.astype(np.float64), t, member)
        assert d[t] == 0.0
        check_member(d, ref, b, (member, t))
    inst, kd = disk_kernel
    t = int(targets_sources(0, inst.N, 1)[0][0])
    d, b = kd.field(t, member)
    check_member(d.cpu().numpy(), dv.field(inst.P, t, member), b, member)


def test_family_special_members_equal_named_kinds(grid65):
    # k = 1 is TV and k = 2 chi-squared term for term, so bit for bit
    g, P, k = grid65
    for t in (5, 900):
        assert np.array_equal(k.field(t, ("power", 1))[0].cpu().numpy(),
                              k.field(t, "tv")[0].cpu().numpy())
        assert np.array_equal(k.field(t, ("power", 2))[0].cpu().numpy(),
                              k.field(t, "chi2")[0].cpu().numpy())


def test_family_members_rejected_on_truncated_handles(gpu_ctx, grid65):
    from paper_1708_02845_amd import DDError, Kernel
    g, P, _ = grid65
    kc = Kernel.load_dense(gpu_ctx, P, tau=1e-3)
    try:
        for m in (("power", 3), ("alpha", 0.5)):
            with pytest.raises(DDError, match="dense handle"):
                kc.field(0, m)
    finally:
        kc.free()
    with pytest.raises(ValueError):
        grid65[2].field(0, ("power", 17))
    with pytest.raises(ValueError):
        grid65[2].field(0, ("alpha", 1.0))
