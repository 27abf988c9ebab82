"""Texture diagnostics on the GPU against the oracle: the diffuse curvatures
(Sec. 3.1), the co-area weighted curvature histogram, the Cahn-Hilliard area,
the normalised discrepancy (Sec. 4.5) and min/max u, for FP64 and FP32 fields,
ragged grids and batches."""

import numpy as np
import pytest
import torch

from oracle import classical, fe_oracle as fo
from paper_2103_04856_amd import fe, inputs

from gpu_helpers import ASYM_C3, ALL_TERMS, WILLMORE_QUARTER, log, oracle_input, to_dev

pytestmark = pytest.mark.gpu

# curvature tolerance (per voxel, in units of |kappa1| + |kappa2| + 1) deciding which
# voxels may fall on either side of a bin edge
KAPPA_TOL = {torch.float64: 1e-8, torch.float32: 2e-3}


def _weights(u, h, eps):
    return h ** 3 * eps * sum(g * g for g in fo.fd_gradient(u, h))


def _ambiguous(k, scale, nbins, kmax, tol):
    """Voxels whose kappa lies within tol * scale of a bin edge (in either precision
    the bin may then differ from the oracle's)."""
    t = (np.clip(k, -kmax, kmax) + kmax) * (nbins / (2 * kmax))
    return np.abs(t - np.round(t)) < tol * scale * (nbins / (2 * kmax))


def _check_instance(u, h, eps, a, stats, curv, hist, nbins, kmax, dtype):
    """Compare one instance's GPU outputs with the oracle."""
    F, A, disc, umin, umax = classical.diagnostic_stats(u, h, eps, a)
    scale = fo.energy_abs(u, h, eps, a)
    rtol = 1e-11 if dtype == torch.float64 else 2e-5
    assert abs(stats[0] - F) <= (1e-10 if dtype == torch.float64 else 1e-4) * scale, (stats[0], F)
    assert abs(stats[1] - A) <= rtol * A, (stats[1], A)
    assert abs(stats[2] - disc) <= rtol * max(disc, 1e-3), (stats[2], disc)
    assert stats[3] == umin and stats[4] == umax
    w = _weights(u, h, eps)
    ref = classical.diffuse_curvatures(u, h, eps)
    errs = []
    if curv is not None:
        for i in range(4):
            e = np.sqrt(np.sum(w * (curv[i] - ref[i]) ** 2) / np.sum(w * ref[i] ** 2))
            errs.append(e)
        assert max(errs) <= (1e-9 if dtype == torch.float64 else 1e-3), errs
    if hist is not None:
        ho = classical.curvature_histogram(u, h, eps, nbins, kmax)
        ks = np.abs(ref[2]) + np.abs(ref[3]) + 1.0
        amb = (_ambiguous(ref[2], ks, nbins, kmax, KAPPA_TOL[dtype])
               | _ambiguous(ref[3], ks, nbins, kmax, KAPPA_TOL[dtype]))
        slack = 2 * w[amb].sum() + (1e-12 if dtype == torch.float64 else 1e-5) * w.sum()
        l1 = np.abs(hist - ho).sum()
        assert l1 <= slack, (l1, slack, amb.mean())
        assert abs(hist.sum() - w.sum()) <= (1e-12 if dtype == torch.float64 else 1e-5) * w.sum()
    return errs


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_noisy_sphere_matches_oracle(dtype):
    """40^3 (ragged against the 64 x 8 tiles), noisy tanh ball, every output."""
    n = 40
    h = 1.0 / n
    eps = 2 * h
    u0 = inputs.noisy_sphere(n, 0.3, eps, 0.02, 11)
    ud = to_dev(u0, dtype)
    ctx = fe.FeContext((1, n, n, n), h, eps, ALL_TERMS, dtype=dtype)
    stats, curv, hist = ctx.diagnostics(ud, curvatures=True, nbins=41, kmax=20.5)
    u = oracle_input(ud)
    errs = _check_instance(u, h, eps, ALL_TERMS, stats[0].numpy(), curv[0].cpu().double().numpy(),
                           hist[0].cpu().numpy(), 41, 20.5, dtype)
    log(f"  {dtype}: curvature weighted rel L2 {max(errs):.1e}")


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_batched_noise_matches_oracle_and_single_instances(dtype):
    """Three instances with their own eps and p on a 24 x 20 x 18 grid: each matches the
    oracle, and equals a single-instance context (stats and curvatures bitwise)."""
    nz, ny, nx = 18, 20, 24
    h = 1.0 / 24
    eps = [2 * h, 1.5 * h, 3 * h]
    coeffs = [ASYM_C3, WILLMORE_QUARTER, ALL_TERMS]
    rng = np.random.default_rng(8)
    U = rng.uniform(-1, 1, size=(3, nz, ny, nx))
    Ud = to_dev(U, dtype)
    ctx = fe.FeContext((3, nz, ny, nx), h, eps, coeffs, dtype=dtype)
    stats, curv, hist = ctx.diagnostics(Ud, curvatures=True, nbins=64, kmax=400.0)
    Uo = oracle_input(Ud)
    for b in range(3):
        _check_instance(Uo[b], h, eps[b], coeffs[b], stats[b].numpy(), curv[b].cpu().double().numpy(),
                        hist[b].cpu().numpy(), 64, 400.0, dtype)
        c1 = fe.FeContext((1, nz, ny, nx), h, eps[b], coeffs[b], dtype=dtype)
        s1, k1, _ = c1.diagnostics(Ud[b:b + 1].contiguous(), curvatures=True)
        assert torch.equal(s1[0], stats[b]) and torch.equal(k1[0], curv[b])


@pytest.mark.parametrize("shape,dtype", [((1, 9, 70), torch.float64), ((5, 1, 3), torch.float64),
                                         ((2, 3, 130), torch.float32), ((202, 64, 64), torch.float32)])
def test_thin_ragged_and_chunked_grids_match_oracle(shape, dtype):
    """Single planes and rows, x tiles ragged against 64, and a tall grid split into
    short z chunks (4 planes on 256 compute units) with a shorter last one: the
    curvature fields written by every plane of every chunk (the first and last
    included) and the other outputs against the oracle."""
    nz, ny, nx = shape
    h = 1.0 / max(shape)
    eps = 2 * h
    U = np.random.default_rng(sum(shape)).uniform(-1, 1, size=shape)
    ud = to_dev(U, dtype)[None].contiguous()
    ctx = fe.FeContext((1, nz, ny, nx), h, eps, ASYM_C3, dtype=dtype)
    stats, curv, hist = ctx.diagnostics(ud, curvatures=True, nbins=16, kmax=50.0)
    u = oracle_input(ud)[0]
    errs = _check_instance(u, h, eps, ASYM_C3, stats[0].numpy(), curv[0].cpu().double().numpy(),
                           hist[0].cpu().numpy(), 16, 50.0, dtype)
    log(f"  {shape} {dtype}: curvature weighted rel L2 {max(errs):.1e}")


def test_deterministic_and_optional_outputs():
    n = 32
    h = 1.0 / n
    u = to_dev(inputs.uniform_noise(n, 3), torch.float32)
    ctx = fe.FeContext((1, n, n, n), h, 2 * h, ASYM_C3, dtype=torch.float32)
    s1, c1, h1 = ctx.diagnostics(u, curvatures=True, nbins=16, kmax=50.0)
    s2, c2, h2 = ctx.diagnostics(u)
    assert c2 is None and h2 is None
    assert torch.equal(s1, s2)
    s3, c3, h3 = ctx.diagnostics(u, curvatures=True, nbins=16, kmax=50.0)
    assert torch.equal(c1, c3)
    torch.testing.assert_close(h1, h3, rtol=1e-12, atol=0)
    # the stream-ordered form fills the same outputs
    c5 = torch.empty_like(c1)
    h5 = torch.empty_like(h1)
    ctx.diagnostics_async(u, c5, h5, kmax=50.0)
    assert torch.equal(c5, c1)
    torch.testing.assert_close(h5, h1, rtol=1e-12, atol=0)
    # one bin holds the total weight
    _, _, h4 = ctx.diagnostics(u, nbins=1, kmax=1.0)
    torch.testing.assert_close(h4.sum(), h1.sum(), rtol=1e-5, atol=0)
    # the energy equals the energy entry point's
    E = ctx.energy(u)
    assert abs(E[0].item() - s1[0, 0].item()) <= 1e-6 * abs(E[0].item())


def test_full_size_area_discrepancy_and_weights():
    """128^3 FP32 batch of 2 at the sizes the bench uses: A_eps, the discrepancy,
    min/max u and the histogram total against the oracle."""
    n, B = 128, 2
    h = 1.0 / n
    U = np.stack([inputs.uniform_noise(n, 4000 + b) for b in range(B)])
    Ud = to_dev(U, torch.float32)
    ctx = fe.FeContext((B, n, n, n), h, 2 * h, WILLMORE_QUARTER, dtype=torch.float32)
    stats, _, hist = ctx.diagnostics(Ud, nbins=64, kmax=200.0)
    Uo = oracle_input(Ud)
    for b in range(B):
        A = classical.cahn_hilliard(Uo[b], h, 2 * h)
        disc = classical.discrepancy(Uo[b], h, 2 * h)
        assert abs(stats[b, 1].item() - A) <= 2e-5 * A
        assert abs(stats[b, 2].item() - disc) <= 2e-5 * disc
        assert stats[b, 3].item() == Uo[b].min() and stats[b, 4].item() == Uo[b].max()
        w = _weights(Uo[b], h, 2 * h).sum()
        assert abs(hist[b].sum().item() - w) <= 1e-5 * w


def test_rejects_bad_arguments():
    n = 16
    ctx = fe.FeContext((1, n, n, n), 1.0 / n, 2.0 / n, WILLMORE_QUARTER, dtype=torch.float32)
    u = torch.zeros((1, n, n, n), dtype=torch.float32, device="cuda")
    with pytest.raises(fe.FeError, match="nbins"):
        ctx.diagnostics(u, nbins=65)
    with pytest.raises(fe.FeError, match="kmax"):
        ctx.diagnostics(u, nbins=8, kmax=0.0)
