"""Launch shapes: the gradient does not depend on the tile, the block size or the
z chunk beyond rounding (every voxel's arithmetic and the gather's order are the
same; the compiler may contract multiply-adds differently in each
instantiation), the energy differs only in its summation order; the autotuner
keeps what it picks and its results."""

import numpy as np
import pytest
import torch

from paper_2103_04856_amd import fe, inputs

from gpu_helpers import ALL_TERMS, ASYM_C3, HELFRICH_SC, log, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_gradient_is_independent_of_the_launch(dtype):
    shape = (28, 36, 40)
    u = to_dev(np.random.default_rng(3).uniform(-1, 1, size=shape), dtype)
    ctx = fe.FeContext((1,) + shape, 1 / 40, 2 / 40, ALL_TERMS, dtype=dtype)
    mask = 1 if dtype == torch.float32 else 2
    ref = None
    worst = 0.0
    gtol, etol = (2e-6, 1e-6) if dtype == torch.float32 else (1e-13, 1e-12)
    for vi, v in enumerate(fe.variants()):
        if not v[3] & mask:
            continue
        for zc in (0, 3, 7):
            ctx.set_launch(vi, zc)
            E, g = ctx.energy_grad(u)
            if ref is None:
                ref = (E[0].item(), g.clone())
                continue
            d = (torch.linalg.vector_norm((g - ref[1]).double()) / torch.linalg.vector_norm(ref[1].double())).item()
            worst = max(worst, d)
            assert d <= gtol, (v[:3], zc, d)
            assert abs(E[0].item() - ref[0]) <= etol * abs(ref[0]), (v[:3], zc)
    log(f"  {dtype}: largest gradient difference between launch shapes {worst:.1e}")


def test_autotune_keeps_its_choice_and_the_results():
    n = 48
    u = to_dev(inputs.uniform_noise(n, 9), torch.float32)
    ctx = fe.FeContext((1, n, n, n), 1 / n, 2 / n, ALL_TERMS, dtype=torch.float32)
    E0, g0 = ctx.energy_grad(u)
    fe.tune_cache_clear()
    v, z, us, cached = ctx.autotune(u, iters=2)
    log(f"  autotune 48^3: variant {fe.variants()[v][:3]} z chunk {z}: {us:.1f} us")
    assert us > 0 and not cached and ctx.get_launch() == (v, z)
    E1, g1 = ctx.energy_grad(u)
    d = (torch.linalg.vector_norm((g1 - g0).double()) / torch.linalg.vector_norm(g0.double())).item()
    assert d <= 2e-6
    assert abs(E1[0].item() - E0[0].item()) <= 1e-6 * abs(E0[0].item())
    # and it is reproducible at that launch
    E2, g2 = ctx.energy_grad(u)
    assert torch.equal(g2, g1) and E2[0].item() == E1[0].item()


def test_autotune_cache_is_used_and_persists(tmp_path):
    """A second context with the same grid, batch, dtype, body and kind takes the cached
    choice without timing; another kind is timed anew; a saved cache, loaded after the
    cache was emptied, serves the choice again; u is never modified."""
    n = 40
    u = to_dev(inputs.uniform_noise(n, 12), torch.float32)
    u_before = u.clone()
    fe.tune_cache_clear()
    c1 = fe.FeContext((1, n, n, n), 1 / n, 2 / n, ALL_TERMS, dtype=torch.float32)
    v1, z1, us1, cached1 = c1.autotune(u, kind="step", iters=2)
    assert not cached1 and torch.equal(u, u_before)
    c2 = fe.FeContext((1, n, n, n), 1 / n, 2 / n, ALL_TERMS, dtype=torch.float32)
    v2, z2, us2, cached2 = c2.autotune(u, kind="step", iters=2)
    assert cached2 and (v2, z2, us2) == (v1, z1, us1) and c2.get_launch() == (v1, z1)
    _, _, _, cached3 = c2.autotune(u, kind="grad", iters=2)
    assert not cached3
    path = str(tmp_path / "tune.txt")
    fe.tune_cache_save(path)
    fe.tune_cache_clear()
    c3 = fe.FeContext((1, n, n, n), 1 / n, 2 / n, ALL_TERMS, dtype=torch.float32)
    fe.tune_cache_load(path)
    v3, z3, _, cached4 = c3.autotune(u, kind="step", iters=2)
    assert cached4 and (v3, z3) == (v1, z1)
    # a p symmetric in k1, k2 runs another kernel: another key
    c4 = fe.FeContext((1, n, n, n), 1 / n, 2 / n, (1.0, 2.5, 1.0, -4.0, -4.0, 4.0), dtype=torch.float32)
    _, _, _, cached5 = c4.autotune(u, kind="step", iters=2)
    assert not cached5
    assert torch.equal(u, u_before)
    log(f"  cache file:\n{open(path).read()}")


def test_autotune_for_adam_keeps_the_optimiser_state():
    """Tuning the Adam sweep between steps does not disturb the context's moments or step
    number: 3 steps, tuning, 2 steps equal 5 steps in one call of a fresh context."""
    n = 24
    u0 = inputs.uniform_noise(n, 13)
    fe.tune_cache_clear()
    ca = fe.FeContext((1, n, n, n), 1 / n, 2 / n, ALL_TERMS, dtype=torch.float32)
    cb = fe.FeContext((1, n, n, n), 1 / n, 2 / n, ALL_TERMS, dtype=torch.float32)
    ua, ub = to_dev(u0, torch.float32), to_dev(u0, torch.float32)
    ca.step_adam(ua, [0.1], 3)
    keep = ca.get_launch()
    ca.autotune(ua, kind="adam", iters=2)
    ca.set_launch(*keep)
    ca.step_adam(ua, [0.1], 2)
    cb.set_launch(*keep)
    cb.step_adam(ub, [0.1], 5)
    assert torch.equal(ua, ub)


def test_automatic_z_chunks_follow_the_occupancy_of_the_kernel_that_runs():
    """The automatic z chunks come from the blocks per compute unit of the kernel the
    call launches: at 256^3 in 32 x 32 tiles the symmetric step (the body without the
    S terms, 75 VGPRs) fits three blocks per CU and takes 22-plane chunks (768 blocks,
    one round), a p with the S terms two blocks and 32-plane chunks (512 blocks). The
    two launch shapes give the same gradient to rounding."""
    n = 256
    h = 1.0 / n
    u = to_dev(inputs.uniform_noise(n, 1005), torch.float32)
    v32 = [i for i, v in enumerate(fe.variants()) if v[:3] == (32, 32, 512)][0]
    sym = fe.FeContext(u.shape, h, 1.5 * h, HELFRICH_SC, dtype=torch.float32)
    asym = fe.FeContext(u.shape, h, 1.5 * h, ASYM_C3, dtype=torch.float32)
    log("case 256^3 automatic z chunks")
    assert sym.get_launch() == (v32, 22)
    assert asym.get_launch() == (v32, 32)
    E22, g22 = sym.energy_grad(u)
    sym.set_launch(v32, 32)
    E32, g32 = sym.energy_grad(u)
    d = (torch.linalg.vector_norm((g22 - g32).double()) / torch.linalg.vector_norm(g32.double())).item()
    assert d <= 2e-6, d
    assert abs(E22[0].item() - E32[0].item()) <= 1e-6 * abs(E32[0].item())
