"""Pins of the oracle's Sec. 5.2 extensions: the orientation term
eps mu (theta . grad u)^2 and the space-dependent parameters a(x), m(x)."""

import math

import numpy as np

from oracle import closed_forms, fe_oracle as fo
from paper_2103_04856_amd import inputs

SIGMA = closed_forms.SIGMA
ALL_TERMS = (1.0, 0.3, 2.0, -3.0, 5.0, 0.7)
ZERO = (0.0, 0.0, 0.0, 0.0, 0.0, 0.0)


def _orientation_energy(u, h, eps, mu, theta):
    """The orientation term alone: F with it minus F without it, p = 0."""
    return fo.energy(u, h, eps, ZERO, orient=(mu, theta))


def test_orientation_term_on_a_slab():
    """Planes x = const: the term vanishes for theta in the planes, and for theta along
    the normal it tends to mu * sigma * area = 2 mu sigma (tanh equipartition),
    at second order in h."""
    eps, mu = 0.03, 2.5
    errs = []
    for n in (64, 128):
        h = 1.0 / n
        u = inputs.tanh_slab(n, 0.25, eps, axis="x")
        assert _orientation_energy(u, h, eps, mu, (0.0, 1.0, 0.0)) == 0.0
        assert _orientation_energy(u, h, eps, mu, (0.0, 0.0, 1.0)) == 0.0
        errs.append(abs(_orientation_energy(u, h, eps, mu, (1.0, 0.0, 0.0)) / (2 * mu * SIGMA) - 1))
    assert errs[1] < 0.01 and errs[0] / errs[1] > 3.0, errs


def test_orientation_term_on_a_cylinder():
    """Cylinder of radius r along z: zero for theta = e_z; for theta = e_x the level set
    of radius r' contributes int (e_x . n)^2 dA = pi r', so by co-area the term tends to
    mu pi sigma r (the odd part of r(t) integrates to 0), at second order in h."""
    r, eps, mu = 0.25, 0.04, 1.5
    errs = []
    for n in (48, 96):
        h = 1.0 / n
        u = inputs.tanh_cylinder(n, r, eps, axis="z")
        assert _orientation_energy(u, h, eps, mu, (0.0, 0.0, 1.0)) == 0.0
        errs.append(abs(_orientation_energy(u, h, eps, mu, (1.0, 0.0, 0.0)) / (mu * math.pi * SIGMA * r) - 1))
    assert errs[1] < 0.01 and errs[0] / errs[1] > 3.0, errs


def test_orientation_is_additive_and_rotates_with_the_field():
    """F(u; a, mu, theta) = F(u; a) + the term alone, and swapping the x and y axes of u
    swaps theta_x and theta_y."""
    n, eps = 10, 0.2
    h = 1.0 / n
    u = inputs.uniform_noise(n, 41)
    th = (0.6, -0.48, 0.64)
    F = fo.energy(u, h, eps, ALL_TERMS, orient=(3.0, th))
    parts = fo.energy(u, h, eps, ALL_TERMS) + _orientation_energy(u, h, eps, 3.0, th)
    assert abs(F - parts) <= 1e-12 * fo.energy_abs(u, h, eps, ALL_TERMS, orient=(3.0, th))
    ut = np.ascontiguousarray(np.swapaxes(u, 1, 2))              # [z, y, x] -> x and y exchanged
    Ft = fo.energy(ut, h, eps, ALL_TERMS, orient=(3.0, (th[1], th[0], th[2])))
    assert abs(F - Ft) <= 1e-12 * abs(F)


def _fd_check(energy, grad, x, d):
    """Central differences with one Richardson step at every entry of x."""
    flat = x.reshape(-1)
    fd = np.empty_like(flat)

    def central(i, step):
        old = flat[i]
        flat[i] = old + step
        ep = energy(x)
        flat[i] = old - step
        em = energy(x)
        flat[i] = old
        return (ep - em) / (2 * step)

    for i in range(flat.size):
        fd[i] = (4 * central(i, d / 2) - central(i, d)) / 3
    return np.linalg.norm(grad.reshape(-1) - fd) / np.linalg.norm(fd)


def test_orientation_gradient_matches_finite_differences():
    u = inputs.uniform_noise(6, 5).repeat(2, axis=2)[:, :, :7].copy()   # 6 x 6 x 7
    h, eps = 1.0 / 6, 0.3
    orient = (4.0, (1 / 3, 2 / 3, -2 / 3))
    _, g = fo.energy_grad(u, h, eps, ALL_TERMS, orient=orient)
    err = _fd_check(lambda v: fo.energy(v, h, eps, ALL_TERMS, orient=orient), g, u, 1e-6)
    assert err < 1e-6, err


def _field_coeffs(shape, seed):
    """a(x): each coefficient a smooth-ish random field around ALL_TERMS."""
    rng = np.random.default_rng(seed)
    return [ak + 0.5 * rng.standard_normal(shape) for ak in ALL_TERMS]


def test_constant_coefficient_fields_equal_scalars():
    n, eps = 8, 0.25
    u = inputs.uniform_noise(n, 3)
    af = [np.full((n, n, n), ak) for ak in ALL_TERMS]
    assert abs(fo.energy(u, 1 / n, eps, af) - fo.energy(u, 1 / n, eps, ALL_TERMS)) == 0.0
    g1 = fo.energy_grad(u, 1 / n, eps, af)[1]
    g2 = fo.energy_grad(u, 1 / n, eps, ALL_TERMS)[1]
    assert np.array_equal(g1, g2)


def test_coefficients_act_at_their_own_voxel():
    """F is linear in the coefficient field voxel by voxel: splitting a(x) over a random
    voxel mask and its complement gives two energies that add up to F(a), and each part
    equals the sum of the uniform-coefficient densities over its voxels."""
    n, eps = 10, 0.2
    h = 1.0 / n
    u = inputs.uniform_noise(n, 9)
    mask = np.random.default_rng(4).random((n, n, n)) < 0.4
    a1 = [np.where(mask, ak, 0.0) for ak in ALL_TERMS]
    a2 = [np.where(mask, 0.0, ak) for ak in ALL_TERMS]
    F = fo.energy(u, h, eps, ALL_TERMS)
    scale = fo.energy_abs(u, h, eps, ALL_TERMS)
    assert abs(fo.energy(u, h, eps, a1) + fo.energy(u, h, eps, a2) - F) <= 1e-12 * scale
    f = fo.pointwise(u, h, eps, ALL_TERMS)["f"]
    assert abs(fo.energy(u, h, eps, a1) - h ** 3 * f[mask].sum()) <= 1e-12 * scale


def test_coefficient_field_gradient_matches_finite_differences():
    n, eps = 6, 0.3
    h = 1.0 / n
    u = inputs.uniform_noise(n, 12)
    af = _field_coeffs(u.shape, 13)
    _, g = fo.energy_grad(u, h, eps, af)
    err = _fd_check(lambda v: fo.energy(v, h, eps, af), g, u, 1e-6)
    assert err < 1e-6, err


def test_mass_field_sets_the_mean_and_the_blurred_offset():
    """u = k * (div A + m(x)): at A = 0 it is the blurred m, and for any A its mean is
    mean(m), since div A has zero mean and the blur sums to one."""
    n, h = 12, 1.0 / 12
    x = inputs.cell_centres(n)
    m = np.broadcast_to(-0.5 + 0.3 * np.cos(2 * np.pi * x), (n, n, n)).copy()   # varies along x
    A0 = np.zeros((3, n, n, n))
    _, _, u0 = fo.hminus_energy_grad(A0, h, 2 * h, ALL_TERMS, m, 1.0)
    np.testing.assert_allclose(u0, fo.gaussian_blur(m, 1.0), rtol=0, atol=1e-15)
    A = inputs.white_noise_vector_field(n, 2, 0.4 * h)
    _, _, u = fo.hminus_energy_grad(A, h, 2 * h, ALL_TERMS, m, 1.0)
    assert abs(u.mean() - m.mean()) < 1e-14


def test_hminus_chain_with_fields_matches_finite_differences():
    n = 6
    h = 1.0 / n
    eps = 2 * h
    af = _field_coeffs((n, n, n), 21)
    m = -0.2 + 0.1 * np.random.default_rng(22).standard_normal((n, n, n))
    orient = (2.0, (0.0, 0.6, 0.8))
    A = inputs.white_noise_vector_field(n, 23, 0.4 * h)
    _, gA, _ = fo.hminus_energy_grad(A, h, eps, af, m, 1.0, orient=orient)
    err = _fd_check(lambda v: fo.hminus_energy(v, h, eps, af, m, 1.0, orient=orient), gA, A, 1e-6 * h)
    assert err < 1e-6, err
