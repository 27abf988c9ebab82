"""Pins of the oracle's Algorithm 1 (H^-1 flow, Sec. 4.1): the divergence and its
adjoint, the Gaussian blur, exact mass, and the whole chain dG/dA against finite
differences."""

import numpy as np
import pytest

from oracle import fe_oracle as fo
from paper_2103_04856_amd import inputs


def test_divergence_is_minus_adjoint_of_gradient():
    """<div A, phi> = -<A, grad phi> on a periodic grid (summation by parts), which is
    what makes dG/dA = -grad dF/du (Sec. 4.1)."""
    rng = np.random.default_rng(3)
    A = rng.normal(size=(3, 6, 7, 8))
    phi = rng.normal(size=(6, 7, 8))
    lhs = np.sum(fo.fd_divergence(A, 0.1) * phi)
    g = fo.fd_gradient(phi, 0.1)
    rhs = -sum(np.sum(A[k] * g[k]) for k in range(3))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_divergence_has_zero_mean_so_mass_is_exact():
    A = inputs.white_noise_vector_field(10, 1, 0.3)
    u = fo.fd_divergence(A, 0.1) + (-0.4)
    assert abs(u.mean() + 0.4) < 1e-14


def test_blur_weights_and_fourier_symbol():
    """Taps sum to 1 and are even; on a Fourier mode the blur multiplies by the
    closed-form symbol prod_a sum_j w_j cos(2 pi k_a j / n)."""
    w = fo.gaussian_weights(2.0)
    assert len(w) == 17 and abs(w.sum() - 1) < 1e-15 and np.allclose(w, w[::-1])
    assert np.array_equal(fo.gaussian_weights(0.0), [1.0])
    n, k = 24, (1, 3, 2)
    x = np.arange(n)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    u = np.cos(2 * np.pi * (k[0] * X + k[1] * Y + k[2] * Z) / n)
    r = (len(w) - 1) // 2
    j = np.arange(-r, r + 1)
    sym = np.prod([np.sum(w * np.cos(2 * np.pi * kk * j / n)) for kk in k])
    np.testing.assert_allclose(fo.gaussian_blur(u, 2.0), sym * u, atol=1e-13)


def test_blur_is_self_adjoint_and_keeps_the_mean():
    rng = np.random.default_rng(4)
    f, g = rng.normal(size=(2, 9, 10, 11))
    assert np.sum(fo.gaussian_blur(f, 1.5) * g) == pytest.approx(np.sum(f * fo.gaussian_blur(g, 1.5)), rel=1e-12)
    assert fo.gaussian_blur(f, 1.5).mean() == pytest.approx(f.mean(), abs=1e-15)


def test_chain_gradient_matches_finite_differences():
    """dG/dA of the whole chain (div, blur, energy) against central differences with a
    Richardson step at every component of a 6^3 field."""
    n = 6
    h = 1.0 / n
    eps, a, m0, sk = 2 * h, (1.0, 0.3, 2.0, -3.0, 5.0, 0.7), -0.2, 1.0
    A = inputs.white_noise_vector_field(n, 5, 0.4 * h)
    E, gA, _ = fo.hminus_energy_grad(A, h, eps, a, m0, sk)
    flat = A.reshape(-1)
    fd = np.empty_like(flat)

    def central(i, d):
        old = flat[i]
        flat[i] = old + d
        ep = fo.hminus_energy(A, h, eps, a, m0, sk)
        flat[i] = old - d
        em = fo.hminus_energy(A, h, eps, a, m0, sk)
        flat[i] = old
        return (ep - em) / (2 * d)

    d = 1e-6 * h
    for i in range(flat.size):
        fd[i] = (4 * central(i, d / 2) - central(i, d)) / 3
    assert np.linalg.norm(gA.reshape(-1) - fd) <= 1e-6 * np.linalg.norm(fd)


def test_adam_on_A_matches_torch_and_keeps_mass():
    import torch
    n = 6
    h = 1.0 / n
    eps, a, m0, sk = 2 * h, (1.0, 0.0, 0.2, -4.0, -4.0, 0.0), -0.3, 1.0
    A0 = inputs.white_noise_vector_field(n, 7, 0.4 * h)
    Ao, Es, u = fo.hminus_descend(A0, h, eps, a, m0, sk, 5)
    x = torch.tensor(A0, requires_grad=True)
    opt = torch.optim.Adam([x], lr=1e-3, betas=(0.9, 0.999), eps=1e-8, weight_decay=0)
    for _ in range(5):
        _, gA, _ = fo.hminus_energy_grad(x.detach().numpy(), h, eps, a, m0, sk)
        opt.zero_grad()
        x.grad = torch.from_numpy(gA)
        opt.step()
    np.testing.assert_allclose(x.detach().numpy(), Ao, rtol=0, atol=1e-14)
    assert abs(u.mean() - m0) < 1e-14
