"""The oracle's hand-derived adjoint gradient against central finite differences.

dF_h/du_i must equal [F_h(u + d e_i) - F_h(u - d e_i)] / (2d) at every voxel of
small grids (no shared code: the finite differences only call the energy).
"""

import numpy as np
import pytest

from oracle import fe_oracle as fo
from paper_2103_04856_amd import inputs

CASES = [
    # (name, field maker, eps/h, coefficients)
    ("noise_willmore", lambda n: inputs.uniform_noise(n, 1001), 2.0, (0.25, 0.5, 0.25, 0, 0, 0)),
    ("noise_asym", lambda n: inputs.uniform_noise(n, 1003), 2.0, (1.0, 0.0, 0.2, -4.0, -4.0, 0.0)),
    ("noise_all_terms", lambda n: inputs.uniform_noise(n, 77), 1.5, (1.0, 0.3, 2.0, -3.0, 5.0, 0.7)),
    ("sphere_helfrich", lambda n: inputs.noisy_sphere(n, 0.3, 1.5 / n, 0.01, 1002), 1.5,
     (1.0, 2.5, 1.0, -4.0, -4.0, 4.0)),
]


def _fd_gradient(u, h, eps, a, d, mode):
    """Central differences with one Richardson step, (4 D(d/2) - D(d)) / 3.

    The sqrt of the positive part has large higher derivatives where
    2||M||^2 - (Tr M)^2 is small, so a plain O(d^2) difference is not enough there.
    """
    g = np.empty_like(u)
    flat = u.reshape(-1)
    gf = g.reshape(-1)

    def central(i, step):
        old = flat[i]
        flat[i] = old + step
        ep = fo.energy(u, h, eps, a, mode=mode)
        flat[i] = old - step
        em = fo.energy(u, h, eps, a, mode=mode)
        flat[i] = old
        return (ep - em) / (2 * step)

    for i in range(flat.size):
        gf[i] = (4.0 * central(i, d / 2) - central(i, d)) / 3.0
    return g


@pytest.mark.parametrize("name,make,eps_h,a", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("mode", ["smooth", "hard"])
def test_adjoint_matches_central_differences_8cubed(name, make, eps_h, a, mode):
    n = 8
    h = 1.0 / n
    u = make(n).astype(np.float64)
    E, g = fo.energy_grad(u, h, eps_h * h, a, mode=mode)
    assert E == pytest.approx(fo.energy(u, h, eps_h * h, a, mode=mode), rel=1e-14)
    fd = _fd_gradient(u.copy(), h, eps_h * h, a, 1e-6, mode)
    rel = np.linalg.norm(g - fd) / np.linalg.norm(fd)
    assert rel < 1e-6, rel


@pytest.mark.parametrize("k", range(6))
def test_each_monomial_gradient(k):
    """Unit coefficient vectors: every term of eq. (Feps) has its own correct gradient."""
    n = 8
    h = 1.0 / n
    a = [0.0] * 6
    a[k] = 1.0
    u = inputs.noisy_sphere(n, 0.3, 2 * h, 0.3, 50 + k)
    _, g = fo.energy_grad(u, h, 2 * h, a)
    fd = _fd_gradient(u.copy(), h, 2 * h, a, 1e-6, "smooth")
    assert np.linalg.norm(g - fd) <= 1e-6 * np.linalg.norm(fd)


def test_random_direction_derivative_non_cubic():
    """<g, v> against a central difference along a random direction on a 6x8x10 grid."""
    rng = np.random.default_rng(5)
    u = rng.uniform(-1, 1, size=(6, 8, 10))
    v = rng.normal(size=u.shape)
    h, eps, a = 0.1, 0.2, (0.7, -0.4, 1.9, 2.0, -1.0, 0.3)
    _, g = fo.energy_grad(u, h, eps, a)
    def central(d):
        return (fo.energy(u + d * v, h, eps, a) - fo.energy(u - d * v, h, eps, a)) / (2 * d)

    fd = (4.0 * central(5e-7) - central(1e-6)) / 3.0
    assert np.sum(g * v) == pytest.approx(fd, rel=1e-7)


def test_gradient_commutes_with_roll():
    u = inputs.uniform_noise(8, 12)
    h, a = 1 / 8, (1.0, 0.0, 0.2, -4.0, -4.0, 0.0)
    _, g = fo.energy_grad(u, h, 2 * h, a)
    _, gr = fo.energy_grad(np.roll(u, (2, -3, 1), (0, 1, 2)), h, 2 * h, a)
    np.testing.assert_allclose(gr, np.roll(g, (2, -3, 1), (0, 1, 2)), rtol=1e-11, atol=1e-13 * np.abs(g).max())


def test_gradient_sums_to_zero_only_via_projection():
    """The projected step moves along g - mean(g): its mass change is zero."""
    u = inputs.uniform_noise(8, 13)
    h = 1 / 8
    _, g = fo.energy_grad(u, h, 2 * h, (0.25, 0.5, 0.25, 0, 0, 0))
    un, _ = fo.mass_projected_step(u, h, 2 * h, (0.25, 0.5, 0.25, 0, 0, 0), np.mean(u), 1e-3)
    np.testing.assert_allclose(un - u, -1e-3 * (g - g.mean()), atol=1e-15)
