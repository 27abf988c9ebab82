"""Pins of the oracle's Algorithm 2 (Sec. 4.2): replicate boundaries, the blur with
replicate padding, and the L-BFGS flow."""

import math

import numpy as np

from oracle import closed_forms, fe_oracle as fo, l2flow
from paper_2103_04856_amd import inputs

SIGMA = closed_forms.SIGMA
ALL_TERMS = (1.0, 0.3, 2.0, -3.0, 5.0, 0.7)
WILLMORE = (1.0, 2.0, 1.0, 0.0, 0.0, 0.0)          # p = H^2 = (k1 + k2)^2


def _even_extension(u):
    """Mirror u across its far face on every axis: a 2N-periodic field whose
    nearest neighbours across every face repeat the face value."""
    for axis in range(3):
        u = np.concatenate([u, np.flip(u, axis=axis)], axis=axis)
    return u


def test_pad_adjoint_is_the_transpose():
    rng = np.random.default_rng(1)
    u = rng.standard_normal((4, 5, 6))
    v = rng.standard_normal((4 + 6, 5 + 6, 6 + 6))
    lhs = np.sum(l2flow.pad_replicate(u, 3) * v)
    rhs = np.sum(u * l2flow.pad_replicate_adjoint(v, 3))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_blur_adjoint_is_the_transpose():
    rng = np.random.default_rng(2)
    u = rng.standard_normal((9, 8, 10))
    v = rng.standard_normal((9, 8, 10))
    lhs = np.sum(l2flow.blur_replicate(u, 1.5) * v)
    rhs = np.sum(u * l2flow.blur_replicate_adjoint(v, 1.5))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # replicate padding keeps constants
    np.testing.assert_allclose(l2flow.blur_replicate(np.full((6, 6, 6), 0.3), 1.5), 0.3, rtol=1e-14)


def test_replicate_energy_equals_the_even_extension():
    """The compact stencils reach one sample, so replicate padding sees exactly the
    mirrored field: F_rep(u) = F_per(E u) / 8 and dF_rep/du = dF_per/d(E u) on the
    original octant (the density is invariant under axis flips)."""
    n = (6, 7, 5)
    h, eps = 1 / 7, 0.3
    u = np.random.default_rng(3).uniform(-1, 1, size=n)
    E, g = l2flow.energy_grad_replicate(u, h, eps, ALL_TERMS)
    Ep, gp = fo.energy_grad(_even_extension(u), h, eps, ALL_TERMS)
    assert abs(E - Ep / 8) <= 1e-12 * fo.energy_abs(_even_extension(u), h, eps, ALL_TERMS) / 8
    np.testing.assert_allclose(g, gp[:n[0], :n[1], :n[2]], rtol=1e-10, atol=1e-12 * np.abs(gp).max())
    assert abs(l2flow.energy_replicate(u, h, eps, ALL_TERMS) - E) <= 1e-14 * abs(E)


def _fd(energy, g, u, d):
    flat = u.reshape(-1)
    fd = np.empty_like(flat)

    def central(i, step):
        old = flat[i]
        flat[i] = old + step
        ep = energy(u)
        flat[i] = old - step
        em = energy(u)
        flat[i] = old
        return (ep - em) / (2 * step)

    for i in range(flat.size):
        fd[i] = (4 * central(i, d / 2) - central(i, d)) / 3
    return np.linalg.norm(g.reshape(-1) - fd) / np.linalg.norm(fd)


def test_gradient_with_blur_matches_finite_differences():
    n = (5, 6, 7)
    h, eps = 1 / 7, 0.3
    u = np.random.default_rng(4).uniform(-1, 1, size=n)
    orient = (3.0, (0.0, 0.6, 0.8))
    for sk in (0.0, 1.0):
        _, g = l2flow.energy_grad_replicate(u, h, eps, ALL_TERMS, sk, orient=orient)
        err = _fd(lambda v: l2flow.energy_replicate(v, h, eps, ALL_TERMS, sk, orient=orient), g, u, 1e-6)
        assert err < 1e-6, (sk, err)


def test_sphere_is_stationary_under_the_flow():
    """Sec. 4.2: the Willmore flow is stationary on spheres. From a tanh ball far from
    the boundary, L-BFGS only relaxes the discrete profile: the energy settles within
    a few steps at F/sigma within 1.5% of 16 pi, and the ball keeps its radius."""
    n, eps, R = 40, 0.06, 0.25
    h = 1.0 / n
    u0 = inputs.tanh_sphere(n, R, eps)
    E0 = l2flow.energy_replicate(u0, h, eps, WILLMORE, 1.0)
    assert abs(E0 / SIGMA / (16 * math.pi) - 1) < 0.05
    u, Es = l2flow.lbfgs_flow(u0, h, eps, WILLMORE, 1.0, 10, max_iter=5)
    E1 = l2flow.energy_replicate(u, h, eps, WILLMORE, 1.0)
    assert E1 <= E0 and abs(E1 / SIGMA / (16 * math.pi) - 1) < 0.015
    assert abs(Es[-1] - Es[3]) < 1e-4 * Es[3]
    radius = (3 * np.count_nonzero(u > 0) / (4 * math.pi)) ** (1 / 3) * h
    assert abs(radius / R - 1) < 0.02
    assert np.abs(u - u0).max() < 0.1
