"""Divergence distance fields between discrete Poisson-kernel rows (Section IV).

For a target interior vertex t with kernel row p = P[t, :], and every interior
vertex x with row q = P[x, :]:

* TV (eq. 34):  d(x) = sum_b |p_b - q_b|          (the L1 distance, range [0, 2])
* KL (eq. 35):  d(x) = sum_b p_b log(p_b / q_b)   (target row as the reference
                 distribution; terms with p_b = 0 contribute 0; a term with
                 p_b > 0 and q_b = 0 is +inf)

Two more members of the f-divergence family named in the paper's conclusion
(Section VI), in the same target-as-reference form d(x) = sum_b p_b f(q_b / p_b):

* chi-squared, f(x) = (x - 1)^2:    d(x) = sum_b (q_b - p_b)^2 / p_b   (+inf if some
                                    p_b = 0 < q_b)
* Hellinger,   f(x) = (sqrt x - 1)^2: d(x) = sum_b (sqrt q_b - sqrt p_b)^2
* power k,     f(x) = |1 - x|^k, integer k >= 1 (k = 1 is TV, k = 2 chi-squared):
               d(x) = sum_b |q_b - p_b|^k / p_b^(k-1)   (+inf if some p_b = 0 < q_b, k > 1)
* alpha,       f(x) = 4/(1 - a^2) (1 - x^((1+a)/2)), a != +-1:
               d(x) = 4/(1 - a^2) sum_b (p_b - p_b^((1-a)/2) q_b^((1+a)/2))

Truncated (sparsified) kernels follow the sparsification remark of Section V
("Precision"): entries of a row below a threshold are dropped, with no
renormalisation.  The row-relative threshold keeps q_b >= tau * max_b q_b;
the absolute threshold keeps q_b >= tau.  The sum the paper uses for the
sparse KL is not in the text; this oracle evaluates the reading where every
dropped entry of row x stands at the threshold of row x (the floor phi_x):

* TV_tau:  d(x) = sum_b |p~_b - q~_b|
* KL_tau:  d(x) = sum_{b: p~_b > 0} p~_b (log p~_b - log q^_b),
           q^_b = q~_b if q~_b > 0 else phi_x.

The paper's own sparse KL keeps log P of every row exact and sums only over
the support of the truncated *target* row (the remedy of Section V,
"Precision": log P combined in the sparse sum after small values of P are
eliminated).  This oracle evaluates it as

* KL_S:    d(x) = sum_{b in S_t} p_b log(p_b / q_b),   S_t = {b : p_b >= thr_t, p_b > 0},
           thr_t = tau * max_b p_b (row-relative) or tau (absolute).

All arithmetic is FP64, rows processed in chunks to bound memory.
"""

import numpy as np

_CHUNK = 1 << 22   # entries per chunk


def _row_chunks(n, width):
    step = max(1, _CHUNK // max(1, width))
    for lo in range(0, n, step):
        yield lo, min(n, lo + step)


def tv_field(P, t):
    """TV distance from every row of P to row t (eq. 34)."""
    P = np.asarray(P, dtype=np.float64)
    p = P[t]
    d = np.empty(P.shape[0])
    for lo, hi in _row_chunks(P.shape[0], P.shape[1]):
        d[lo:hi] = np.abs(p[None, :] - P[lo:hi]).sum(axis=1)
    return d


def kl_field(P, t):
    """KL distance from every row of P, with row t as the reference (eq. 35)."""
    P = np.asarray(P, dtype=np.float64)
    p = P[t]
    sup = p > 0
    ps = p[sup]
    d = np.empty(P.shape[0])
    with np.errstate(divide="ignore"):
        for lo, hi in _row_chunks(P.shape[0], int(sup.sum())):
            q = P[lo:hi][:, sup]
            d[lo:hi] = (ps[None, :] * np.log(ps[None, :] / q)).sum(axis=1)
    return d


def chi2_field(P, t):
    """Chi-squared divergence from every row of P, row t as the reference."""
    P = np.asarray(P, dtype=np.float64)
    p = P[t]
    sup = p > 0
    ps = p[sup]
    d = np.empty(P.shape[0])
    for lo, hi in _row_chunks(P.shape[0], P.shape[1]):
        q = P[lo:hi]
        d[lo:hi] = ((q[:, sup] - ps[None, :]) ** 2 / ps[None, :]).sum(axis=1)
        off = (q[:, ~sup] > 0).any(axis=1)
        d[lo:hi][off] = np.inf
    return d


def hellinger_field(P, t):
    """Squared Hellinger divergence from every row of P to row t."""
    P = np.asarray(P, dtype=np.float64)
    sp = np.sqrt(P[t])
    d = np.empty(P.shape[0])
    for lo, hi in _row_chunks(P.shape[0], P.shape[1]):
        d[lo:hi] = ((np.sqrt(P[lo:hi]) - sp[None, :]) ** 2).sum(axis=1)
    return d


def support(p, tau, relative=True):
    """Mask of the truncated support of row p: p_b > 0 and p_b >= the threshold."""
    p = np.asarray(p, dtype=np.float64)
    thr = tau * p.max() if relative else float(tau)
    return (p > 0) & (p >= thr)


def kl_support_field(P, t, tau, relative=True):
    """KL_S: eq. (35) summed over the truncated support of the target row only."""
    P = np.asarray(P, dtype=np.float64)
    sup = support(P[t], tau, relative)
    ps = P[t][sup]
    d = np.empty(P.shape[0])
    with np.errstate(divide="ignore"):
        for lo, hi in _row_chunks(P.shape[0], int(sup.sum())):
            q = P[lo:hi][:, sup]
            d[lo:hi] = (ps[None, :] * np.log(ps[None, :] / q)).sum(axis=1)
    return d


FIELDS = {"tv": tv_field, "kl": kl_field, "chi2": chi2_field, "hellinger": hellinger_field}


def field(P, t, kind):
    """Field of a kind name: "tv", "kl", "chi2", "hellinger", ("power", k),
    ("alpha", a)."""
    if isinstance(kind, tuple):
        return power_field(P, t, kind[1]) if kind[0] == "power" else alpha_field(P, t, kind[1])
    return FIELDS[kind](P, t)


def distances(P, t, xs, kind, tau=0.0, relative=True):
    """Distances of the rows xs to the target row t: the field functions
    applied to the stacked rows [P[t]; P[xs]] (equal to the field entries up
    to summation order).  kind "kl_s" is KL_S with threshold tau."""
    P = np.asarray(P, dtype=np.float64)
    sub = np.vstack([P[t][None, :], P[np.asarray(xs, dtype=np.int64)]])
    if kind == "kl_s":
        return kl_support_field(sub, 0, tau, relative)[1:]
    return field(sub, 0, kind)[1:]


def power_field(P, t, k):
    """f(x) = |1 - x|^k (Section VI): sum_b |q_b - p_b|^k / p_b^(k-1)."""
    P = np.asarray(P, dtype=np.float64)
    k = int(k)
    p = P[t]
    sup = p > 0
    ps = p[sup]
    d = np.empty(P.shape[0])
    for lo, hi in _row_chunks(P.shape[0], P.shape[1]):
        q = P[lo:hi]
        d[lo:hi] = (np.abs(q[:, sup] - ps[None, :]) ** k / ps[None, :] ** (k - 1)).sum(axis=1)
        off = q[:, ~sup].sum(axis=1)     # p_b = 0: |q_b| for k = 1, +inf for k > 1 if q_b > 0
        d[lo:hi] += off if k == 1 else np.where(off > 0, np.inf, 0.0)
    return d


def alpha_field(P, t, alpha):
    """alpha-divergence (Section VI): 4/(1-a^2) sum_b (p_b - p_b^((1-a)/2) q_b^((1+a)/2))."""
    P = np.asarray(P, dtype=np.float64)
    a = float(alpha)
    p = P[t]
    d = np.empty(P.shape[0])
    for lo, hi in _row_chunks(P.shape[0], P.shape[1]):
        q = P[lo:hi]
        d[lo:hi] = (p[None, :] - p[None, :] ** ((1 - a) / 2) * q ** ((1 + a) / 2)).sum(axis=1)
    return 4.0 / (1.0 - a * a) * d


def truncate(P, tau, relative=True):
    """P~ with entries below the threshold set to 0, and the per-row threshold."""
    P = np.asarray(P, dtype=np.float64)
    if relative:
        thr = tau * P.max(axis=1)
    else:
        thr = np.full(P.shape[0], float(tau))
    keep = P >= thr[:, None]
    return np.where(keep, P, 0.0), thr


def tv_trunc_field(Pt, t):
    """TV_tau: eq. (34) on the truncated rows."""
    return tv_field(Pt, t)


def kl_trunc_field(Pt, t, floor):
    """KL_tau with dropped entries of row x floored at ``floor[x]``."""
    Pt = np.asarray(Pt, dtype=np.float64)
    floor = np.asarray(floor, dtype=np.float64)
    p = Pt[t]
    sup = p > 0
    ps = p[sup]
    lp = np.log(ps)
    d = np.empty(Pt.shape[0])
    for lo, hi in _row_chunks(Pt.shape[0], int(sup.sum())):
        q = Pt[lo:hi][:, sup]
        qh = np.where(q > 0, q, floor[lo:hi, None])
        d[lo:hi] = (ps[None, :] * (lp[None, :] - np.log(qh))).sum(axis=1)
    return d


def csr_from_truncated(Pt):
    """CSR (row_ptr int64, col int32, val float64) of a truncated dense kernel."""
    Pt = np.asarray(Pt)
    r, c = np.nonzero(Pt)
    ptr = np.zeros(Pt.shape[0] + 1, dtype=np.int64)
    np.add.at(ptr, r + 1, 1)
    return np.cumsum(ptr), c.astype(np.int32), Pt[r, c].astype(np.float64)
