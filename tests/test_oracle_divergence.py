"""Pins for the oracle's TV (eq. 34) and KL (eq. 35) fields and the truncated fields."""

import numpy as np
import pytest
from scipy.spatial.distance import cityblock
from scipy.stats import entropy

from conftest import frac, read_golden
from oracle import disk as odisk
from oracle import divergence as dv
from workloads import build_config, grid_domain
from workloads.seeds import rng


@pytest.fixture(scope="module")
def c1():
    return build_config("disk4096")


@pytest.fixture(scope="module")
def grid_P():
    g = grid_domain(49, 2, (0.1, 0.3), seed_id=11)
    P = g.poisson_kernel()
    keep = P.max(axis=0) > 0
    return P[:, keep]


def test_kl_is_library_relative_entropy_with_target_as_reference(grid_P):
    # scipy.stats.entropy(pk, qk) = sum pk log(pk/qk): KL with pk the reference.
    P = grid_P
    t = 123
    d = dv.kl_field(P, t)
    for x in (0, 7, 400, P.shape[0] - 1):
        assert d[x] == pytest.approx(entropy(P[t], P[x]), rel=1e-12, abs=1e-15)
    # the reversed argument order is a different number on this domain
    x = 400
    assert abs(entropy(P[x], P[t]) - d[x]) > 1e-3 * d[x]


def test_chi2_is_library_chisquare_with_target_as_expected(grid_P):
    from scipy.stats import chisquare
    P = grid_P
    t = 77
    d = dv.chi2_field(P, t)
    for x in (0, 9, 333, P.shape[0] - 1):
        assert d[x] == pytest.approx(chisquare(P[x], P[t]).statistic, rel=1e-10)
    x = 333
    assert abs(chisquare(P[t], P[x]).statistic - d[x]) > 1e-3 * d[x]   # the order matters


def test_hellinger_is_squared_euclidean_of_square_roots(grid_P):
    from scipy.spatial.distance import sqeuclidean
    P = grid_P
    t = 12
    d = dv.hellinger_field(P, t)
    for x in (0, 5, 500, P.shape[0] - 1):
        assert d[x] == pytest.approx(sqeuclidean(np.sqrt(P[t]), np.sqrt(P[x])), rel=1e-12)
    assert d.max() <= 2.0 and d[t] == 0.0


def test_chi2_infinite_when_reference_is_zero():
    P = np.array([[0.5, 0.5, 0.0], [0.4, 0.4, 0.2]])
    assert np.isinf(dv.chi2_field(P, 0)[1])
    assert dv.chi2_field(P, 1)[0] == pytest.approx(0.01 / 0.4 * 2 + 0.2)


@pytest.mark.parametrize("k", range(3))
def test_disk_chi2_and_hellinger_closed_forms(c1, k):
    # Theorem A5 with f(x) = (x - 1)^2 and f(x) = (sqrt x - 1)^2, carried to
    # any target by the Moebius map (A10) and conformal invariance (A2).
    t = int(rng(0, "targets").integers(0, c1.N, size=3)[k])
    chi = dv.chi2_field(c1.P, t)
    ref = odisk.chi2_closed(c1.z, c1.z[t])
    assert np.max(np.abs(chi - ref) / np.maximum(ref, 1e-3)) < 1e-4
    hel = dv.hellinger_field(c1.P, t)
    assert np.abs(hel - odisk.hellinger_closed(c1.z, c1.z[t])).max() < 5e-6


def test_tv_is_library_l1_distance(grid_P):
    P = grid_P
    t = 55
    d = dv.tv_field(P, t)
    for x in (0, 9, 333, P.shape[0] - 1):
        assert d[x] == pytest.approx(cityblock(P[t], P[x]), rel=1e-13)


def test_hand_solved_two_vertex_grid_divergences():
    rows = {r[0]: r[1:] for r in read_golden("grid4x3_two_vertex.txt")}
    P = np.array([[frac(v) for v in rows["a"]], [frac(v) for v in rows["b"]]])
    assert dv.tv_field(P, 0)[1] == pytest.approx(frac(rows["TV_a_to_b"][0]), rel=1e-15)
    assert dv.kl_field(P, 0)[1] == pytest.approx(frac(rows["KL_a_to_b_over_log4"][0]) * np.log(4),
                                                 rel=1e-15)


@pytest.mark.parametrize("k", range(3))
def test_disk_fields_match_closed_forms(c1, k):
    # Appendix eqs. A6 and A8 carried to any target by the Moebius map (A10)
    # and conformal invariance (Theorem A2).  The sampled kernel is a B-point
    # trapezoid rule, exact up to O(r^B) for KL; TV has a kink, so its
    # quadrature converges algebraically.
    t = int(rng(0, "targets").integers(0, c1.N, size=3)[k])
    kl = dv.kl_field(c1.P, t)
    tv = dv.tv_field(c1.P, t)
    assert np.abs(kl - odisk.kl_closed(c1.z, c1.z[t])).max() < 5e-6
    assert np.abs(tv - odisk.tv_closed(c1.z, c1.z[t])).max() < 2.5e-3


def test_fields_vanish_at_target_and_respect_ranges(grid_P):
    P = grid_P
    for t in (0, 100, 700):
        kl = dv.kl_field(P, t)
        tv = dv.tv_field(P, t)
        assert kl[t] == 0.0 and tv[t] == 0.0
        assert kl.min() >= 0.0                      # Gibbs' inequality
        assert tv.min() >= 0.0 and tv.max() <= 2.0
        others = np.arange(P.shape[0]) != t
        assert kl[others].min() > 0.0 and tv[others].min() > 0.0


def test_brute_force_loops_on_tiny_stochastic_matrix():
    g = np.random.default_rng(5)
    P = g.random((9, 6)) ** 3
    P[2, 4] = 0.0                    # a zero in the reference row
    P /= P.sum(axis=1, keepdims=True)
    t = 2
    kl, tv = dv.kl_field(P, t), dv.tv_field(P, t)
    hel = dv.hellinger_field(P, t)
    for x in range(9):
        s_kl = 0.0
        s_tv = 0.0
        s_h = 0.0
        for b in range(6):
            s_tv += abs(P[t, b] - P[x, b])
            s_h += (P[t, b] ** 0.5 - P[x, b] ** 0.5) ** 2
            if P[t, b] > 0:
                s_kl += P[t, b] * np.log(P[t, b] / P[x, b])
        assert kl[x] == pytest.approx(s_kl, rel=1e-13, abs=1e-16)
        assert tv[x] == pytest.approx(s_tv, rel=1e-13, abs=1e-16)
        assert hel[x] == pytest.approx(s_h, rel=1e-13, abs=1e-16)


def test_kl_infinite_when_reference_mass_meets_zero():
    P = np.array([[0.5, 0.5], [1.0, 0.0]])
    assert np.isinf(dv.kl_field(P, 0)[1])
    assert dv.kl_field(P, 1)[0] == pytest.approx(np.log(2.0))


def test_truncation_threshold_zero_is_dense(grid_P):
    P = grid_P
    Pt, thr = dv.truncate(P, 0.0)
    assert np.array_equal(Pt, P)
    t = 321
    assert np.array_equal(dv.tv_trunc_field(Pt, t), dv.tv_field(P, t))
    assert np.allclose(dv.kl_trunc_field(Pt, t, thr), dv.kl_field(P, t), rtol=1e-12, atol=1e-15)


def test_truncated_fields_brute_force(grid_P):
    P = grid_P[:40]
    tau = 1e-3
    Pt, thr = dv.truncate(P, tau)
    assert 0 < (Pt == 0).sum() < Pt.size
    t = 11
    kl = dv.kl_trunc_field(Pt, t, thr)
    tv = dv.tv_trunc_field(Pt, t)
    for x in range(P.shape[0]):
        rowmax = max(P[x])
        s_kl = 0.0
        s_tv = 0.0
        for b in range(P.shape[1]):
            pt = P[t, b] if P[t, b] >= tau * max(P[t]) else 0.0
            qx = P[x, b] if P[x, b] >= tau * rowmax else 0.0
            s_tv += abs(pt - qx)
            if pt > 0:
                s_kl += pt * (np.log(pt) - np.log(qx if qx > 0 else tau * rowmax))
        assert kl[x] == pytest.approx(s_kl, rel=1e-12, abs=1e-14)
        assert tv[x] == pytest.approx(s_tv, rel=1e-12, abs=1e-15)
    assert kl[t] == 0.0 and tv[t] == 0.0


def test_csr_round_trip(grid_P):
    Pt, _ = dv.truncate(grid_P, 1e-4)
    ptr, col, val = dv.csr_from_truncated(Pt)
    back = np.zeros_like(Pt)
    for x in range(Pt.shape[0]):
        back[x, col[ptr[x]:ptr[x + 1]]] = val[ptr[x]:ptr[x + 1]]
    assert np.array_equal(back, Pt)


def test_support_kl_threshold_zero_is_dense_kl(grid_P):
    t = 210
    assert np.array_equal(dv.kl_support_field(grid_P, t, 0.0), dv.kl_field(grid_P, t))


def test_support_kl_brute_force():
    g = np.random.default_rng(9)
    P = g.random((12, 30)) ** 4
    P /= P.sum(axis=1, keepdims=True)
    t, tau = 3, 0.05
    d = dv.kl_support_field(P, t, tau)
    da = dv.kl_support_field(P, t, 0.01, relative=False)
    for x in range(12):
        s_rel = 0.0
        s_abs = 0.0
        for b in range(30):
            p, q = P[t, b], P[x, b]
            if p >= tau * max(P[t]):
                s_rel += p * np.log(p / q)
            if p >= 0.01:
                s_abs += p * np.log(p / q)
        assert d[x] == pytest.approx(s_rel, rel=1e-13, abs=1e-16)
        assert da[x] == pytest.approx(s_abs, rel=1e-13, abs=1e-16)


def test_support_kl_log_sum_lower_bound(grid_P):
    # log-sum inequality on S_t: d(x) >= W_S log(W_S / Q_S(x)), equality at x = t
    t, tau = 400, 1e-2
    d = dv.kl_support_field(grid_P, t, tau)
    sup = dv.support(grid_P[t], tau)
    assert 0 < sup.sum() < sup.size
    W = grid_P[t, sup].sum()
    Q = grid_P[:, sup].sum(axis=1)
    lb = W * np.log(W / Q)
    assert np.all(d >= lb - 1e-12 * np.abs(d)) and d[t] == 0.0
    # it is not the dense KL: the dropped mass changes the value
    assert np.abs(d - dv.kl_field(grid_P, t)).max() > 1e-4


def test_row_distances_equal_field_entries(grid_P):
    t = 50
    xs = [0, 7, 50, 900, 901]
    # equal up to the order numpy sums a row in (the stacked matrix is small)
    for kind, f in dv.FIELDS.items():
        assert np.allclose(dv.distances(grid_P, t, xs, kind), f(grid_P, t)[xs],
                           rtol=1e-14, atol=0)
    assert np.allclose(dv.distances(grid_P, t, xs, "kl_s", 1e-3),
                       dv.kl_support_field(grid_P, t, 1e-3)[xs], rtol=1e-14, atol=0)


def test_power_family_special_cases(grid_P):
    t = 99
    assert np.allclose(dv.power_field(grid_P, t, 1), dv.tv_field(grid_P, t), rtol=1e-13, atol=0)
    assert np.allclose(dv.power_field(grid_P, t, 2), dv.chi2_field(grid_P, t), rtol=1e-13, atol=0)


def test_alpha_family_special_cases(grid_P):
    # alpha = 0 is twice the squared Hellinger distance (rows sum to 1)
    t = 99
    W = grid_P.sum(axis=1)
    assert np.allclose(W, 1.0, atol=1e-12)
    assert np.allclose(dv.alpha_field(grid_P, t, 0.0), 2 * dv.hellinger_field(grid_P, t),
                       rtol=1e-10, atol=1e-13)
    # alpha = 3 is half the chi-squared distance
    assert np.allclose(dv.alpha_field(grid_P, t, 3.0), 0.5 * dv.chi2_field(grid_P, t),
                       rtol=1e-10, atol=1e-13)


def test_power_and_alpha_brute_force():
    g = np.random.default_rng(17)
    P = g.random((7, 9)) ** 2
    P[1, 3] = 0.0
    P /= P.sum(axis=1, keepdims=True)
    t = 2
    for k in (1, 3, 4):
        d = dv.power_field(P, t, k)
        for x in range(7):
            s = sum(P[t, b] * abs(1 - P[x, b] / P[t, b]) ** k for b in range(9))
            assert d[x] == pytest.approx(s, rel=1e-12, abs=1e-15)
    for a in (-0.75, 0.25, 0.875):
        d = dv.alpha_field(P, t, a)
        for x in range(7):
            s = sum(P[t, b] * 4 / (1 - a * a) * (1 - (P[x, b] / P[t, b]) ** ((1 + a) / 2))
                    for b in range(9))
            assert d[x] == pytest.approx(s, rel=1e-12, abs=1e-14)


@pytest.mark.parametrize("k", range(2))
def test_disk_power_and_alpha_closed_forms(c1, k):
    # Theorem A5 with f(x) = |1-x|^4 and the alpha-divergences, through the
    # Moebius map (A10) and conformal invariance (A2); moments by 2F1
    # (the B-point rule converges more slowly for |1-x|^4, whose integrand
    # carries fourth powers of the kernel: 1.1e-3 relative at worst here)
    t = int(rng(0, "targets").integers(0, c1.N, size=2)[k])
    ref = odisk.power_closed(c1.z, c1.z[t], 4)
    got = dv.power_field(c1.P, t, 4)
    assert np.max(np.abs(got - ref) / np.maximum(ref, 1e-3)) < 5e-3
    for a in (-0.5, 0.25, 0.75):
        ref = odisk.alpha_closed(c1.z, c1.z[t], a)
        assert np.abs(dv.alpha_field(c1.P, t, a) - ref).max() < 2e-5


@pytest.mark.parametrize("tau,relative", [(1e-3, True), (1e-6, True), (2e-4, False)])
def test_truncated_kl_is_a_floored_contraction(grid_P, tau, relative):
    # An entry is stored when P_xb >= phi_x, and a dropped one stands at phi_x, so
    # the value KL_tau takes for row x is max(P_xb, phi_x) and
    #   KL_tau(x, t) = sum_b p~_b log p~_b - sum_b p~_b log max(P_xb, phi_x):
    # one matrix product over the floored log-kernel (the form the library's
    # contraction takes on truncated handles).
    P = np.asarray(grid_P, dtype=np.float64)
    Pt, thr = dv.truncate(P, tau, relative)
    L = np.log(np.maximum(P, thr[:, None]))
    for t in (0, 17, P.shape[0] - 1):
        p = Pt[t]
        H = float((p[p > 0] * np.log(p[p > 0])).sum())
        alt = H - L @ p
        ref = dv.kl_trunc_field(Pt, t, thr)
        assert np.abs(alt - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max()), t
