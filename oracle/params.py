"""Coefficient vectors of the paper's polynomials.

TEST INFRASTRUCTURE ONLY (see the oracle package header).

a = (a20, a11, a02, a10, a01, a00) is the order of Sec. 3.2; p(k1, k2) =
a20 k1^2 + a11 k1 k2 + a02 k2^2 + a10 k1 + a01 k2 + a00.
"""


def a_from_redundant(b):
    """Expand eq. (redundant), Sec. 4.3:
    h2 (H - H0)^2 + k1 K + alpha (kappa1 - kappa1_0)^2 + beta (kappa2 - kappa2_0)^2
    with H = kappa1 + kappa2, K = kappa1 kappa2 and b = (h2, H0, k1, alpha, kappa1_0,
    beta, kappa2_0), into the reduced coefficients a.
    """
    h2, H0, k1, alpha, k10, beta, k20 = (float(v) for v in b)
    return (h2 + alpha,
            2.0 * h2 + k1,
            h2 + beta,
            -2.0 * h2 * H0 - 2.0 * alpha * k10,
            -2.0 * h2 * H0 - 2.0 * beta * k20,
            h2 * H0 * H0 + alpha * k10 * k10 + beta * k20 * k20)


def a_helfrich(chi_b, chi_G, H0):
    """Coefficients that turn F_eps into the Helfrich phase field (end of Sec. 3.2)."""
    return (chi_b / 2.0, chi_b + chi_G, chi_b / 2.0, -chi_b * H0, -chi_b * H0, chi_b * H0 * H0 / 2.0)


A_WILLMORE = (1.0, 2.0, 1.0, 0.0, 0.0, 0.0)      # p = H^2, end of Sec. 3.2


def a_inside_out(a):
    """Coefficients a' with F(-u; a) = F(u; a').

    W' is odd, so M(-u) = -M(u): Tr M changes sign while ||M|| and the
    anisotropy S do not, which swaps the roles of kappa1 and -kappa2.
    """
    a20, a11, a02, a10, a01, a00 = a
    return (a02, a11, a20, -a01, -a10, a00)
