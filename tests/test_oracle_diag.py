"""Pins of the oracle's texture diagnostics: the Cahn-Hilliard area A_eps (Sec. 2.3),
the normalised discrepancy (Sec. 4.5), the diffuse principal curvatures (Sec. 3.1)
and their co-area weighted histogram, the mesh-free stand-in for the curvature
diagram of Sec. 4.1. Closed forms come from the tanh profile, for which
eps |grad u|^2 = sqrt(2 W(u)) |grad u|, so co-area integrals over level sets apply."""

import math

import numpy as np

from oracle import classical, closed_forms, fe_oracle as fo
from paper_2103_04856_amd import inputs

SIGMA = closed_forms.SIGMA
I_TAIL = (math.pi ** 2 - 6.0) / 9.0      # int s^2 sech^4 s ds over R


def test_constant_field():
    """u = c: no gradient, so A_eps = W(c)/eps (unit volume), the discrepancy is 1,
    and every histogram weight is 0."""
    n, eps, c = 12, 0.1, 0.3
    u = np.full((n, n, n), c)
    F, A, disc, umin, umax = classical.diagnostic_stats(u, 1.0 / n, eps, (1, 0, 1, 0, 0, 0))
    assert abs(A - 0.25 * (1 - c * c) ** 2 / eps) < 1e-14
    assert disc == 1.0 and umin == c and umax == c
    assert not classical.curvature_histogram(u, 1.0 / n, eps, 9, 5.0).any()


def test_slab_area_and_discrepancy_converge_at_second_order():
    """Two parallel planes (area 2) with the tanh profile: A_eps -> 2 sigma, and the
    equipartition eps/2 |u'|^2 = W(u)/eps of the profile drives the discrepancy to 0;
    both errors shrink about 4x per halving of h at fixed eps."""
    eps = 0.03
    errs = []
    for n in (64, 128):
        u = inputs.tanh_slab(n, 0.25, eps)
        A = classical.cahn_hilliard(u, 1.0 / n, eps)
        errs.append((abs(A - 2 * SIGMA), classical.discrepancy(u, 1.0 / n, eps)))
    assert errs[1][0] < 0.005 * 2 * SIGMA and errs[1][1] < 0.01, errs
    assert errs[0][0] / errs[1][0] > 3.0 and errs[0][1] / errs[1][1] > 3.0, errs


def _centres(nbins, kmax):
    return (np.arange(nbins) + 0.5) * (2.0 * kmax / nbins) - kmax


def test_sphere_histogram_weight_and_first_moment():
    """Ball of radius R: by co-area the weights add up to int sqrt(2W(t)) Area({u=t}) dt
    = 4 pi (sigma R^2 + sqrt(2) I eps^2), and the weighted sum of kappa1 + kappa2 to
    int sqrt(2W(t)) 8 pi r(t) dt = 8 pi sigma R; both converge at second order. All
    the weight sits at positive curvatures (u > 0 inside: convex means H > 0)."""
    R, eps, nb, kmax = 0.25, 0.04, 400, 20.0
    c = _centres(nb, kmax)
    tot_ref = 4 * math.pi * (SIGMA * R * R + math.sqrt(2.0) * I_TAIL * eps * eps)
    mom_ref = 8 * math.pi * SIGMA * R
    errs = []
    for n in (64, 128):
        u = inputs.tanh_sphere(n, R, eps)
        H = classical.curvature_histogram(u, 1.0 / n, eps, nb, kmax)
        tot = H.sum()
        assert abs(tot - 1.0 / n ** 3 * eps * sum(g * g for g in fo.fd_gradient(u, 1.0 / n)).sum()) < 1e-12
        mom = (H * (c[:, None] + c[None, :])).sum()
        errs.append((abs(tot / tot_ref - 1), abs(mom / mom_ref - 1)))
        assert H[c > 0][:, c > 0].sum() > 0.999 * tot
    assert errs[1][0] < 0.005 and errs[1][1] < 0.005, errs
    assert errs[0][0] / errs[1][0] > 3.0 and errs[0][1] / errs[1][1] > 3.0, errs


def test_cylinder_histogram_orientation():
    """Cylinder of radius r: kappa1 = 1/r' > 0 on the level set of radius r', kappa2 = 0.
    With an odd bin count, 0 is a bin centre: the weight lies in the kappa2 columns
    around 0 (the stencil's anisotropy spreads kappa2 by about +-0.3 at eps/h = 3.8)
    and in the kappa1 rows of the interface band, never the other way round."""
    r, eps, n = 0.25, 0.04, 96
    nb, kmax = 41, 10.25                  # bin width 0.5, bin 20 = [-0.25, 0.25)
    u = inputs.tanh_cylinder(n, r, eps)
    H = classical.curvature_histogram(u, 1.0 / n, eps, nb, kmax)
    c = _centres(nb, kmax)
    tot = H.sum()
    assert H[:, 20].sum() > 0.6 * tot
    assert H[:, 19:22].sum() > 0.999 * tot
    band = (c > 1 / (r + 3 * eps)) & (c < 1 / (r - 3 * eps))
    assert H[band, 19:22].sum() > 0.97 * tot
    assert H[19:22, :].sum() < 0.01 * tot


def test_inside_out_mirrors_the_histogram():
    """u -> -u maps (kappa1, kappa2) to (-kappa2, -kappa1) (M changes sign, W' is odd),
    so with bins symmetric about 0 the histogram is mirrored through the anti-diagonal."""
    n, eps, nb, kmax = 32, 0.06, 31, 12.0
    u = inputs.noisy_sphere(n, 0.3, eps, 0.05, 3)
    H = classical.curvature_histogram(u, 1.0 / n, eps, nb, kmax)
    Hm = classical.curvature_histogram(-u, 1.0 / n, eps, nb, kmax)
    np.testing.assert_allclose(Hm, H[::-1, ::-1].T, rtol=1e-12, atol=1e-15 * H.sum())


def test_values_beyond_kmax_are_truncated_into_the_edge_bins():
    """A ball of radius 0.25 has kappa ~ 4; with kmax = 1 every weight lands in the last bin."""
    n, eps = 48, 0.05
    u = inputs.tanh_sphere(n, 0.25, eps)
    H = classical.curvature_histogram(u, 1.0 / n, eps, 8, 1.0)
    assert H[7, 7] > 0.999 * H.sum()
