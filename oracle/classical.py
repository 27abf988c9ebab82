"""Classical phase fields and diffuse curvatures, written from their own formulas.

TEST INFRASTRUCTURE ONLY (see the oracle package header). These functionals are
the ones F_eps must reduce to for particular coefficient vectors, so each is
coded directly from its defining equation rather than through the F_eps
density:

* A_eps, the Cahn-Hilliard (diffuse area) energy, eq. (CH_eps), Sec. 2.3;
* W_eps, the Bellettini-Paolini Willmore phase field, eq. (Willmore_eps);
* H_eps, the Bellettini-Mugnai Helfrich phase field, eq. (Helfrich_eps);
* the diffuse curvatures of eqs. (Beps)-(kepsb), Sec. 3.1;
* the normalised discrepancy used as a viability test in Sec. 4.5 (Experiment 4);
* a co-area weighted histogram of (kappa1, kappa2), standing in for the
  curvature diagram of Sec. 4.1, and the per-field viability summary.

The same discretisation readings as the F_eps oracle apply: periodic central
differences, the 7-point Laplacian, and |grad u| regularised by xi wherever it
divides or multiplies a curvature term; Tr(n (x) n) then equals q / (q + xi^2).
"""

import numpy as np

from .fe_oracle import XI, double_well, double_well_prime, fd_gradient, fd_hessian, fd_laplacian


def _grad_sq(u, h):
    g = fd_gradient(u, h)
    return g[0] ** 2 + g[1] ** 2 + g[2] ** 2


def cahn_hilliard(u, h, eps):
    """A_eps(u) = sum h^3 (eps/2 |grad u|^2 + W(u)/eps), eq. (CH_eps)."""
    u = np.asarray(u, dtype=np.float64)
    return float(h ** 3 * np.sum(0.5 * eps * _grad_sq(u, h) + double_well(u) / eps))


def willmore_eps(u, h, eps, xi=XI):
    """W_eps(u) = (1/eps) sum h^3 (eps Lap u - W'(u)/eps Tr(n (x) n))^2, eq. (Willmore_eps).

    With the regularised normal, Tr(n (x) n) = q/(q + xi^2) instead of 1.
    """
    u = np.asarray(u, dtype=np.float64)
    q = _grad_sq(u, h)
    tr_nn = q / (q + xi * xi)
    inner = eps * fd_laplacian(u, h) - double_well_prime(u) / eps * tr_nn
    return float(h ** 3 * np.sum(inner ** 2) / eps)


def _matrix_field(u, h, eps, xi):
    """M = -eps Hess u + W'(u)/eps n (x) n as a (..., 3, 3) array, eq. (Meps)."""
    g = np.stack(fd_gradient(u, h), axis=-1)
    H6 = fd_hessian(u, h)
    Hm = np.empty(u.shape + (3, 3))
    Hm[..., 0, 0], Hm[..., 1, 1], Hm[..., 2, 2] = H6[0], H6[1], H6[2]
    Hm[..., 0, 1] = Hm[..., 1, 0] = H6[3]
    Hm[..., 0, 2] = Hm[..., 2, 0] = H6[4]
    Hm[..., 1, 2] = Hm[..., 2, 1] = H6[5]
    q = np.sum(g * g, axis=-1)
    nn = g[..., :, None] * g[..., None, :] / (q + xi * xi)[..., None, None]
    return -eps * Hm + (double_well_prime(u) / eps)[..., None, None] * nn, q


def helfrich_eps(u, h, eps, chi_b, chi_G, H0, xi=XI):
    """H_eps(u) of eq. (Helfrich_eps): chi_b/(2eps)(Tr M - eps|grad u| H0)^2
    + chi_G/(2eps)((Tr M)^2 - ||M||^2), summed with weight h^3.

    |grad u| multiplying H0 is regularised as sqrt(q + xi^2) (Sec. 4.1).
    """
    u = np.asarray(u, dtype=np.float64)
    M, q = _matrix_field(u, h, eps, xi)
    tr = np.trace(M, axis1=-2, axis2=-1)
    fro2 = np.sum(M * M, axis=(-2, -1))
    rho = np.sqrt(q + xi * xi)
    dens = chi_b / (2 * eps) * (tr - eps * rho * H0) ** 2 + chi_G / (2 * eps) * (tr ** 2 - fro2)
    return float(h ** 3 * np.sum(dens))


def diffuse_curvatures(u, h, eps, xi=XI):
    """(H, K, kappa1, kappa2) per voxel from eqs. (Heps), (Keps), (kepsa), (kepsb).

    |grad u| in the denominators is regularised as sqrt(q + xi^2); the values are
    the curvatures of the level sets of u (exactly so for a tanh profile).
    """
    u = np.asarray(u, dtype=np.float64)
    M, q = _matrix_field(u, h, eps, xi)
    rho = np.sqrt(q + xi * xi)
    tr = np.trace(M, axis1=-2, axis2=-1)
    fro2 = np.sum(M * M, axis=(-2, -1))
    Hc = tr / (eps * rho)
    Kc = (tr ** 2 - fro2) / (2 * eps ** 2 * rho ** 2)
    disc = np.sqrt(np.maximum(2 * fro2 - tr ** 2, 0.0))
    k1 = (tr + disc) / (2 * eps * rho)
    k2 = (tr - disc) / (2 * eps * rho)
    return Hc, Kc, k1, k2


def discrepancy(u, h, eps):
    """Normalised discrepancy of Sec. 4.5: sum|eps/2|grad u|^2 - W/eps| / A_eps-sum."""
    u = np.asarray(u, dtype=np.float64)
    a = 0.5 * eps * _grad_sq(u, h)
    b = double_well(u) / eps
    return float(np.sum(np.abs(a - b)) / np.sum(a + b))


def curvature_histogram(u, h, eps, nbins, kmax, xi=XI):
    """Co-area weighted histogram of the diffuse principal curvatures: a mesh-free
    stand-in for the curvature diagram of Sec. 4.1 (the area-weighted law of
    (kappa1, kappa2) on the surface).

    Each voxel contributes the weight h^3 eps |grad u|^2, the density that
    concentrates on the diffuse interface (for a tanh profile it equals
    sqrt(2 W(u)) |grad u|, so by co-area the weights add up to the
    sigma-weighted areas of the level sets). Its (kappa1, kappa2) from
    eqs. (kepsa), (kepsb) are clamped to [-kmax, kmax] (values are truncated
    there, as in the paper's diagrams) and binned uniformly:
    index = floor((kappa + kmax) * nbins / (2 kmax)), at most nbins - 1.
    Returns hist[nbins, nbins], indexed [bin of kappa1, bin of kappa2].
    """
    u = np.asarray(u, dtype=np.float64)
    _, _, k1, k2 = diffuse_curvatures(u, h, eps, xi)
    w = h ** 3 * eps * _grad_sq(u, h)
    scale = nbins / (2.0 * kmax)

    def index(k):
        kc = np.clip(k, -kmax, kmax)
        return np.minimum(np.floor((kc + kmax) * scale).astype(np.int64), nbins - 1)

    hist = np.zeros((nbins, nbins))
    np.add.at(hist, (index(k1).ravel(), index(k2).ravel()), w.ravel())
    return hist


def diagnostic_stats(u, h, eps, a, xi=XI):
    """Per-field summary used to assess a generated texture (Sec. 4.5, Experiment 4):
    (F_h, A_eps, normalised discrepancy, min u, max u). The paper deems a shape
    viable when the discrepancy is under 0.75, max u > 0.1 and min u < -0.1."""
    from .fe_oracle import energy
    u = np.asarray(u, dtype=np.float64)
    return (energy(u, h, eps, a, xi), cahn_hilliard(u, h, eps), discrepancy(u, h, eps),
            float(u.min()), float(u.max()))
