"""Continuum values of F_eps on tanh-profile fields, by one-dimensional quadrature.

TEST INFRASTRUCTURE ONLY (see the oracle package header).

For u = tanh(d / (sqrt(2) eps)) with d the signed distance to a surface
(eq. (tanh_profile)), the diffuse curvatures equal the curvatures of the level
sets (Sec. 3.1) and the co-area argument of Sec. 3.2 gives

    F_eps(u) = int_{-1}^{1} sqrt(2 W(t)) F({u = t}) dt,   sqrt(2 W(t)) = (1 - t^2)/sqrt(2),

where the level set {u = t} sits at signed distance d_t = sqrt(2) eps artanh(t).
For spheres, cylinders and planes every level set is again a sphere, cylinder or
plane, so F({u = t}) is elementary and the whole value is a 1-D integral.

sigma = int_{-1}^{1} sqrt(2W) = 4/(3 sqrt 2) is the constant of Sec. 2.3.
"""

import math

import numpy as np
from scipy import integrate

SIGMA = 4.0 / (3.0 * math.sqrt(2.0))   # Sec. 2.3 (Notations), closed form


def sqrt_2w(t):
    """sqrt(2 W(t)) = (1 - t^2)/sqrt(2) for |t| <= 1."""
    return (1.0 - t * t) / math.sqrt(2.0)


def sigma_by_quadrature():
    """sigma = int_{-1}^{1} sqrt(2 W(s)) ds computed numerically."""
    val, _ = integrate.quad(lambda s: math.sqrt(2.0 * 0.25 * (1.0 - s * s) ** 2), -1.0, 1.0,
                            epsabs=1e-13, epsrel=1e-12)
    return val


def poly(a, k1, k2):
    """p(k1, k2) = sum_|alpha|<=2 a_alpha (k1, k2)^alpha, order (a20, a11, a02, a10, a01, a00)."""
    a20, a11, a02, a10, a01, a00 = a
    return a20 * k1 * k1 + a11 * k1 * k2 + a02 * k2 * k2 + a10 * k1 + a01 * k2 + a00


def _coarea(level_value, eps, t_max):
    """int sqrt(2W(t)) F(level set t) dt over t in (-1, t_max), substituted t = tanh(s).

    In the variable s = artanh(t) the integrand is smooth and decays like
    sech^4(s), so the infinite range is cut at |s| = 40 without loss.
    """
    s_max = math.atanh(t_max) if t_max < 1.0 else 40.0
    # the centre line / centre point (radius -> 0) carries weight ~ sech^4(s_max);
    # stop just short of it so that no level set of radius 0 is evaluated
    s_max = min(s_max * (1.0 - 1e-9), 40.0)

    def integrand(s):
        t = math.tanh(s)
        return sqrt_2w(t) * (1.0 - t * t) * level_value(math.sqrt(2.0) * eps * s)

    val, _ = integrate.quad(integrand, -40.0, s_max, epsabs=1e-13, epsrel=1e-13, limit=400)
    return val


def sphere_feps(a, R, eps):
    """F_eps of a tanh-profile ball of radius R, u = +1 inside.

    The level set at distance d_t inside is a sphere of radius R_t = R - d_t with
    kappa1 = kappa2 = 1/R_t (positive on a convex set, Sec. 2.1), area 4 pi R_t^2.
    Level sets exist only while R_t > 0.
    """
    t_max = math.tanh(R / (math.sqrt(2.0) * eps))

    def level(d):
        Rt = R - d
        return 4.0 * math.pi * Rt * Rt * poly(a, 1.0 / Rt, 1.0 / Rt)

    return _coarea(level, eps, t_max)


def cylinder_feps(a, r, eps, length=1.0):
    """F_eps of a tanh-profile solid cylinder of radius r and length `length`.

    Level set: cylinder of radius r_t = r - d_t, kappa1 = 1/r_t, kappa2 = 0,
    area 2 pi r_t length.
    """
    t_max = math.tanh(r / (math.sqrt(2.0) * eps))

    def level(d):
        rt = r - d
        return 2.0 * math.pi * rt * length * poly(a, 1.0 / rt, 0.0)

    return _coarea(level, eps, t_max)


def planes_feps(a, area):
    """F_eps of flat tanh interfaces of total area `area`: kappa1 = kappa2 = 0, so
    every level set contributes a00 * area, and the integral is a00 * sigma * area."""
    return poly(a, 0.0, 0.0) * SIGMA * area
