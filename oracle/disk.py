"""Unit-disk closed forms (Appendix, Sections 1-2).

* rho(x, t) = |x - t| / |1 - conj(t) x|: modulus of the Moebius map that sends
  t to 0 (eq. A10).
* Hyperbolic distance HB = 2 atanh(rho) (eq. A1).
* By conformal invariance of the divergence distances (Theorem A2) and their
  values on the disk with target 0 (eqs. A6, A8):
      KL(x; t) = -log(1 - rho^2),     TV(x; t) = (4/pi) asin(rho).
* For any f-divergence the value on the disk with target 0 is
  g(r) = (1/2pi) int f(h(r, phi)) dphi with h the Poisson kernel ratio
  (Theorem A5).  For f(x) = (x - 1)^2 this is 2 r^2 / (1 - r^2) (the
  Appendix table lists (1 + r^2)/(1 - r^2), which is off by the constant 1:
  g(0) must be 0); for f(x) = (sqrt x - 1)^2 it is
  2 - (4/pi) sqrt(1 - r^2) K(r), K the complete elliptic integral of the first
  kind with modulus r (scipy's ellipk takes the parameter r^2).  For
  f(x) = |1 - x|^k with even k and for the alpha-divergences, g follows from
  the moments (1/2pi) int h^s dphi = (1 - r^2)^s 2F1(s, s; 1; r^2).
* Gradient-descent paths on the disk are hyperbolic geodesics: arcs of the
  circle through source and target orthogonal to the unit circle (Appendix
  Section 2.2), which also passes through 1/conj(source).
"""

import numpy as np


def rho(x, t):
    x = np.asarray(x, dtype=np.complex128)
    return np.abs(x - t) / np.abs(1.0 - np.conj(t) * x)


def hyperbolic(x, t):
    return 2.0 * np.arctanh(rho(x, t))


def kl_closed(x, t):
    r = rho(x, t)
    return -np.log1p(-r * r)


def tv_closed(x, t):
    return (4.0 / np.pi) * np.arcsin(rho(x, t))


def chi2_closed(x, t):
    r = rho(x, t)
    return 2.0 * r * r / (1.0 - r * r)


def hellinger_closed(x, t):
    from scipy.special import ellipk
    r = rho(x, t)
    return 2.0 - (4.0 / np.pi) * np.sqrt(1.0 - r * r) * ellipk(r * r)


def _poisson_moment(i, r):
    """(1/2pi) int h(r, phi)^i dphi = (1 - r^2)^i 2F1(i, i; 1; r^2), h the disk
    Poisson kernel ratio (1 - r^2) / (1 - 2 r cos phi + r^2)."""
    from scipy.special import hyp2f1
    return (1.0 - r * r) ** i * hyp2f1(i, i, 1.0, r * r)


def power_closed(x, t, k):
    """f(x) = |1 - x|^k for even k: binomial expansion of (1 - h)^k (Theorem A5)."""
    from scipy.special import comb
    assert k % 2 == 0
    r = rho(x, t)
    return sum(comb(k, i, exact=True) * (-1) ** i * _poisson_moment(i, r) for i in range(k + 1))


def alpha_closed(x, t, alpha):
    """alpha-divergence: 4/(1-a^2) (1 - (1/2pi) int h^s), s = (1+a)/2 (Theorem A5)."""
    s = (1.0 + alpha) / 2.0
    return 4.0 / (1.0 - alpha * alpha) * (1.0 - _poisson_moment(s, rho(x, t)))


def geodesic_distance(points, s, t):
    """Euclidean distance of each point from the hyperbolic geodesic through s, t.

    The geodesic is the arc of the circle through s, t and 1/conj(s); when s, t
    and 0 are collinear it degenerates to the line through s and t.
    """
    points = np.asarray(points, dtype=np.complex128)
    cross = (np.conj(s) * t).imag
    if abs(cross) < 1e-12 * max(1.0, abs(s) * abs(t)):
        direction = (t - s) / abs(t - s)
        rel = points - s
        return np.abs((np.conj(direction) * rel).imag)
    a, b, c = s, t, 1.0 / np.conj(s)
    # circumcentre of a, b, c
    d = 2.0 * (a.real * (b.imag - c.imag) + b.real * (c.imag - a.imag) + c.real * (a.imag - b.imag))
    ux = ((abs(a) ** 2) * (b.imag - c.imag) + (abs(b) ** 2) * (c.imag - a.imag)
          + (abs(c) ** 2) * (a.imag - b.imag)) / d
    uy = ((abs(a) ** 2) * (c.real - b.real) + (abs(b) ** 2) * (a.real - c.real)
          + (abs(c) ** 2) * (b.real - a.real)) / d
    centre = complex(ux, uy)
    radius = abs(a - centre)
    return np.abs(np.abs(points - centre) - radius)
