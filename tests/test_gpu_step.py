"""The mass-projected descent step on the GPU: trajectory parity with the oracle
for the first steps, exact mass, graph replay equal to eager, energy decrease."""

import numpy as np
import pytest
import torch

from oracle import fe_oracle as fo
from paper_2103_04856_amd import fe, inputs

from gpu_helpers import (ALL_TERMS, ASYM_C3, HELFRICH_SC, TOL, WILLMORE_QUARTER, assert_same_to_rounding, log,
                         oracle_input, rel_l2, to_dev, voxel_errors)

pytestmark = pytest.mark.gpu


def test_first_steps_match_oracle_fp64():
    """32^3 FP64, u0 ~ U(-1,1), eps = 2h, Willmore p, mean 0, tau = 1e-3: ten steps."""
    n = 32
    h = 1.0 / n
    u0 = inputs.uniform_noise(n, 1001)
    ud = to_dev(u0, torch.float64)
    ctx = fe.FeContext((1, n, n, n), h, 2 * h, WILLMORE_QUARTER, dtype=torch.float64)
    uo = oracle_input(ud)
    for k in range(10):
        Eg = ctx.step(ud, [0.0], 1e-3, 1)
        uo, Eo = fo.mass_projected_step(uo, h, 2 * h, WILLMORE_QUARTER, 0.0, 1e-3)
        assert abs(Eg[0].item() - Eo) <= 1e-10 * abs(Eo)
        err = rel_l2(ud.cpu().numpy(), uo)
        assert err <= 1e-11, (k, err)
    log(f"  10-step trajectory rel {err:.2e}")


def test_nsteps_call_equals_single_steps_and_oracle():
    """fe_step(n = 37) replays captured graphs; it must equal 37 calls of n = 1 (bitwise).
    Against the oracle: 37 steps with p = (k1+k2)^2/4, and 5 steps with an asymmetric p
    (with a20 != a02 the flow amplifies rounding differences ~1e13-fold over 37 steps,
    through dS/dX = 1/(2S) near umbilic voxels, so only a short prefix is unique)."""
    n = 16
    h = 1.0 / n
    u0 = inputs.uniform_noise(n, 21)
    for dtype in (torch.float64, torch.float32):
        for a, nref in ((ASYM_C3, 5), (WILLMORE_QUARTER, 37)):
            ctx = fe.FeContext((1, n, n, n), h, 2 * h, a, dtype=dtype)
            u1 = to_dev(u0, dtype)
            u2 = u1.clone()
            uo = oracle_input(u1)
            E1 = ctx.step(u1, [-0.3], 1e-3, 37)
            for _ in range(37):
                E2 = ctx.step(u2, [-0.3], 1e-3, 1)
            assert torch.equal(u1, u2) and E1[0].item() == E2[0].item()
            if dtype == torch.float64:
                u3 = to_dev(u0, dtype)
                Eg = ctx.step(u3, [-0.3], 1e-3, nref)
                uo, Es = fo.descend(uo, h, 2 * h, a, -0.3, 1e-3, nref)
                assert rel_l2(u3.cpu().numpy(), uo) <= 1e-10, a
                assert abs(Eg[0].item() - Es[-1]) <= 1e-9 * abs(Es[-1])


def test_mass_is_exact_every_step():
    n = 32
    h = 1.0 / n
    for dtype, tol in ((torch.float64, 1e-12), (torch.float32, 2e-6)):
        u = to_dev(inputs.uniform_noise(n, 5), dtype)
        ctx = fe.FeContext((1, n, n, n), h, 2 * h, ASYM_C3, dtype=dtype)
        for k in range(5):
            ctx.step(u, [-0.3], 1e-3, 1 + k)
            s = u.double().sum().item()
            assert abs(s - (-0.3) * n ** 3) <= tol * u.double().abs().sum().item(), (dtype, k, s)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_steps_on_an_odd_sized_batch(dtype):
    """Two instances of 13 x 11 x 7 (1001 voxels: the final shift takes its scalar path,
    no 16-byte groups) with their own masses: three steps against the oracle, each
    instance's mean exact."""
    shape = (7, 11, 13)
    h = 1.0 / 13
    U = np.stack([inputs.uniform_noise(16, s)[:7, :11, :13] for s in (41, 42)])
    ud = to_dev(U, dtype)
    masses = [-0.2, 0.15]
    ctx = fe.FeContext(ud.shape, h, [2 * h, 2 * h], [WILLMORE_QUARTER, HELFRICH_SC], dtype=dtype)
    Uo = oracle_input(ud)
    ctx.step(ud, masses, 1e-3, 3)
    for b in range(2):
        uo, _ = fo.descend(Uo[b], h, 2 * h, [WILLMORE_QUARTER, HELFRICH_SC][b], masses[b], 1e-3, 3)
        err = rel_l2(ud[b].cpu().double().numpy(), uo)
        assert err <= (1e-11 if dtype == torch.float64 else 1e-5), (b, err)
        mean = ud[b].double().mean().item()
        assert abs(mean - masses[b]) <= (1e-13 if dtype == torch.float64 else 1e-6), (b, mean)


def test_energy_decreases_after_first_step():
    """Config-1 flow (32^3 FP64, tau = 1e-3): monotone decrease after step 1 and the
    energy after 200 steps within 1% of the oracle run."""
    n = 32
    h = 1.0 / n
    u0 = inputs.uniform_noise(n, 1001)
    ud = to_dev(u0, torch.float64)
    ctx = fe.FeContext((1, n, n, n), h, 2 * h, WILLMORE_QUARTER, dtype=torch.float64)
    Es = []
    for k in range(20):
        Es.append(ctx.step(ud, [0.0], 1e-3, 10)[0].item())
    assert all(Es[i + 1] < Es[i] for i in range(len(Es) - 1)), Es
    Efinal = ctx.energy(ud)[0].item()
    uo, _ = fo.descend(u0, h, 2 * h, WILLMORE_QUARTER, 0.0, 1e-3, 200)
    Eo = fo.energy(uo, h, 2 * h, WILLMORE_QUARTER)
    log(f"  200 steps: gpu {Efinal:.6g} oracle {Eo:.6g}")
    assert abs(Efinal - Eo) <= 1e-2 * abs(Eo)


def test_batched_step_per_instance_mass():
    n, B = 24, 5
    h = 1.0 / n
    coeffs, means = inputs.random_instance_table(B, 4999)
    U = np.stack([inputs.uniform_noise(n, 4000 + b) for b in range(B)])
    ud = to_dev(U, torch.float64)
    ctx = fe.FeContext(ud.shape, h, 2 * h, coeffs, dtype=torch.float64)
    uo = [oracle_input(ud[b]) for b in range(B)]
    ctx.step(ud, list(means), 1e-3, 4)
    for b in range(B):
        ref, _ = fo.descend(uo[b], h, 2 * h, coeffs[b], means[b], 1e-3, 4)
        assert rel_l2(ud[b].cpu().numpy(), ref) <= 1e-10
        assert abs(ud[b].mean().item() - means[b]) <= 1e-12


def test_adam_first_steps_match_oracle():
    """Mass-projected Adam steps (lr 1e-3, betas (0.9, 0.999)): FP64 trajectory and
    energies against the oracle for five steps, across two calls (moments persist)."""
    n = 20
    h = 1.0 / n
    u0 = inputs.uniform_noise(n, 1003)
    for a in (ASYM_C3, WILLMORE_QUARTER):
        ud = to_dev(u0, torch.float64)
        ctx = fe.FeContext((1, n, n, n), h, 2 * h, a, dtype=torch.float64)
        ctx.step_adam(ud, [-0.3], 3)
        E = ctx.step_adam(ud, [-0.3], 2)
        uo, Es = fo.descend_adam(oracle_input(to_dev(u0, torch.float64)), h, 2 * h, a, -0.3, 5)
        assert rel_l2(ud.cpu().numpy(), uo) <= 1e-10, a
        assert abs(E[0].item() - Es[-1]) <= 1e-10 * abs(Es[-1])
        # reset: the same five steps again from u0
        ctx.adam_reset()
        ud2 = to_dev(u0, torch.float64)
        ctx.step_adam(ud2, [-0.3], 5)
        assert torch.equal(ud2, ud)


def test_adam_long_call_matches_oracle():
    """One call of 37 Adam steps (the first step, two directly launched pairs and a
    replay of the 16-step graph): the step numbers in the bias corrections advance
    across direct launches and graph replays exactly as the oracle's do."""
    n = 12
    h = 1.0 / n
    u0 = inputs.uniform_noise(n, 1009)
    ud = to_dev(u0, torch.float64)
    ctx = fe.FeContext((1, n, n, n), h, 2 * h, ASYM_C3, dtype=torch.float64)
    E = ctx.step_adam(ud, [-0.2], 37)
    uo, Es = fo.descend_adam(oracle_input(to_dev(u0, torch.float64)), h, 2 * h, ASYM_C3, -0.2, 37)
    assert rel_l2(ud.cpu().numpy(), uo) <= 1e-10
    assert abs(E[0].item() - Es[-1]) <= 1e-10 * abs(Es[-1])


def test_adam_graph_replay_equals_single_steps():
    n = 16
    h = 1.0 / n
    u0 = inputs.uniform_noise(n, 44)
    for dtype in (torch.float64, torch.float32):
        c1 = fe.FeContext((1, n, n, n), h, 2 * h, ASYM_C3, dtype=dtype)
        c2 = fe.FeContext((1, n, n, n), h, 2 * h, ASYM_C3, dtype=dtype)
        u1, u2 = to_dev(u0, dtype), to_dev(u0, dtype)
        c1.step_adam(u1, [0.1], 41)
        for _ in range(41):
            c2.step_adam(u2, [0.1], 1)
        assert torch.equal(u1, u2)
        assert abs(u1.double().mean().item() - 0.1) < (1e-13 if dtype == torch.float64 else 1e-6)


def test_batched_16x128_adam_flow_stays_finite():
    """The batched workload (16 x 128^3 FP32, per-instance coefficients and target
    means) with mass-projected Adam, lr 1e-3, for 300 graph-replayed steps: finite,
    mass kept, energy decreasing. (The plain gradient step diverges here within a
    few steps at any useful tau: dF_h/du spikes near umbilic voxels.)"""
    n, B = 128, 16
    h = 1.0 / n
    coeffs, means = inputs.random_instance_table(B, 4999)
    ud = torch.stack([to_dev(inputs.uniform_noise(n, 4000 + b), torch.float32) for b in range(B)])
    ctx = fe.FeContext(ud.shape, h, 2 * h, coeffs, dtype=torch.float32)
    E0 = ctx.energy(ud)
    E1 = ctx.step_adam(ud, list(means), 100)
    E2 = ctx.step_adam(ud, list(means), 200)
    assert torch.isfinite(E2).all()
    assert (E2 < E1).all() and (E1 < E0).all(), (E0, E1, E2)
    m = ud.double().mean(dim=(1, 2, 3)).cpu().numpy()
    assert np.abs(m - means).max() < 1e-6
    log(f"  batched Adam flow E0 {E0.sum().item():.4g} -> {E2.sum().item():.4g}")


def test_fp32_first_steps_close_to_oracle():
    n = 64
    h = 1.0 / n
    u0 = inputs.noisy_sphere(n, 0.3, 1.5 * h, 0.01, 1002)
    ud = to_dev(u0, torch.float32)
    m = float(ud.double().mean().item())
    uo = oracle_input(ud)
    ctx = fe.FeContext((1, n, n, n), h, 1.5 * h, WILLMORE_QUARTER, dtype=torch.float32)
    ctx.step(ud, [m], 1e-3, 3)
    uo, _ = fo.descend(uo, h, 1.5 * h, WILLMORE_QUARTER, m, 1e-3, 3)
    # the change of u over three steps is what is compared
    err = rel_l2(ud.cpu().double().numpy() - u0, uo - u0)
    log(f"  fp32 3-step update rel {err:.2e}")
    assert err <= 1e-3


def test_autograd_function_matches_kernel_gradient():
    n = 24
    h = 1.0 / n
    for dtype in (torch.float64, torch.float32):
        u = to_dev(inputs.uniform_noise(n, 9), dtype).requires_grad_(True)
        ctx = fe.FeContext((1, n, n, n), h, 2 * h, ASYM_C3, dtype=dtype)
        E = fe.feps(u, ctx)
        (3.0 * E.sum()).backward()
        _, g = ctx.energy_grad(u.detach())
        # the backward folds the incoming 3.0 into the coefficients: equal to rounding
        assert_same_to_rounding(u.grad, 3.0 * g, dtype, "backward")
        Eo, go = fo.energy_grad(oracle_input(u), h, 2 * h, ASYM_C3)
        assert rel_l2(u.grad.cpu().double().numpy() / 3.0, go) <= (1e-3 if dtype == torch.float32 else 1e-9)


def test_autograd_descent_loop_keeps_mass():
    """Descent driven by autograd: u <- u - tau dE/du, then the mean is projected back."""
    n = 32
    h = 1.0 / n
    u = to_dev(inputs.uniform_noise(n, 1003), torch.float32)
    ctx = fe.FeContext((1, n, n, n), h, 2 * h, ASYM_C3, dtype=torch.float32)
    m = -0.3
    Es = []
    for _ in range(30):
        x = u.clone().requires_grad_(True)
        E = fe.feps(x, ctx)
        E.sum().backward()
        with torch.no_grad():
            v = x - 1e-3 * x.grad
            u = v + (m - v.double().mean()).to(v.dtype)
        Es.append(E.item())
    assert abs(u.double().mean().item() - m) < 1e-6
    assert Es[-1] < Es[1]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_grad_scaled_equals_scaled_gradient(dtype):
    """fe_grad_scaled_async against s_b times fe_energy_grad's gradient, to rounding:
    three instances (asymmetric p with the orientation term, symmetric p, every term),
    scales (2.5, -0.75, 0); then the same with a coefficient field (scaled after the
    sweep); the context's own parameters stay unchanged."""
    n = 24
    h = 1.0 / n
    U = np.stack([inputs.uniform_noise(n, s) for s in (3, 4, 5)])
    ud = to_dev(U, dtype)
    ctx = fe.FeContext(ud.shape, h, [2 * h, 1.5 * h, 2 * h], [ASYM_C3, HELFRICH_SC, ALL_TERMS], dtype=dtype)
    ctx.set_orientation([30.0, 0.0, 5.0], [(0.0, 0.6, 0.8)] * 3)
    scale = torch.tensor([2.5, -0.75, 0.0], dtype=torch.float64, device="cuda")
    E0, g0 = ctx.energy_grad(ud)
    gs = ctx.grad_scaled_async(ud, scale)
    torch.cuda.synchronize()
    for b in range(3):
        ref = g0[b] * scale[b].item()
        if scale[b].item() == 0.0:
            assert torch.count_nonzero(gs[b]).item() == 0
        else:
            assert_same_to_rounding(gs[b], ref, dtype, f"instance {b}")
    E1, g1 = ctx.energy_grad(ud)
    assert torch.equal(E0, E1) and torch.equal(g0, g1)
    a_field = torch.empty((3, 6) + ud.shape[1:], dtype=dtype, device="cuda")
    for b, a in enumerate([ASYM_C3, HELFRICH_SC, ALL_TERMS]):
        for k in range(6):
            a_field[b, k] = a[k] * (1.0 + 0.1 * torch.rand(ud.shape[1:], device="cuda", dtype=dtype))
    ctx.set_coeff_field(a_field)
    _, gf = ctx.energy_grad(ud)
    gsf = ctx.grad_scaled_async(ud, scale)
    torch.cuda.synchronize()
    for b in range(2):
        assert_same_to_rounding(gsf[b], gf[b] * scale[b].item(), dtype, f"field instance {b}")
    assert torch.count_nonzero(gsf[2]).item() == 0


def _autograd_adam(ctx, x0, m, lr):
    """The paper's optimisation loop through autograd: y a leaf tensor, E = FeEnergy(y),
    backward by the adjoint kernel, torch.optim.Adam (fused and capturable: one kernel,
    its step count and bias corrections on the device), then y <- y + (m - mean y). Returns (y, one step)."""
    y = x0.clone().requires_grad_(True)
    opt = torch.optim.Adam([y], lr=lr, fused=True, capturable=True)

    def step():
        opt.zero_grad(set_to_none=True)
        fe.feps(y, ctx).sum().backward()
        opt.step()
        with torch.no_grad():
            y.add_(m - y.mean())
    return y, step


@pytest.mark.parametrize("n,dtype", [(20, torch.float64), (128, torch.float32)])
def test_graph_captured_autograd_step_equals_eager(n, dtype):
    """The autograd-driven Adam step (energy-only sweep forward, adjoint sweep backward,
    torch Adam, mass projection) captured in a CUDA graph after three eager steps: four
    replays, each followed by eager work on the same context and a synchronisation, each
    equal bit for bit to the same step run eagerly from the same state."""
    h = 1.0 / n
    ctx = fe.FeContext((1, n, n, n), h, 2 * h, ASYM_C3, dtype=dtype)
    x0 = to_dev(inputs.uniform_noise(n, 1003), dtype)
    yg, step_g = _autograd_adam(ctx, x0, -0.3, 1e-3)
    ye, step_e = _autograd_adam(ctx, x0, -0.3, 1e-3)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(3):
            step_g()
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step_g()
    for _ in range(3):
        step_e()
    assert torch.equal(yg, ye)
    other = to_dev(inputs.uniform_noise(n, 77), dtype)
    for r in range(4):
        graph.replay()
        step_e()
        torch.cuda.synchronize()
        assert torch.isfinite(yg).all() and torch.equal(yg, ye), f"replay {r}"
        ctx.energy_grad(other)                     # eager work on the same context between replays
        torch.cuda.synchronize()
    assert abs(yg.double().mean().item() + 0.3) < (1e-12 if dtype == torch.float64 else 1e-6)
    assert not torch.equal(yg, x0)


def test_config_128cubed_2000_autograd_adam_steps():
    """The 128^3 asymmetric-p workload driven through autograd for 2000 steps (the step
    captured in a CUDA graph and replayed): the field stays finite, keeps its mean -0.3
    and its energy falls."""
    n = 128
    h = 1.0 / n
    ctx = fe.FeContext((1, n, n, n), h, 2 * h, ASYM_C3, dtype=torch.float32)
    x0 = to_dev(inputs.uniform_noise(n, 1003), torch.float32)
    E0 = ctx.energy(x0)[0].item()
    y, step = _autograd_adam(ctx, x0, -0.3, 1e-3)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _ in range(3):
            step()
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    Es = []
    for k in range(1997):
        graph.replay()
        if (k + 1) % 499 == 0:
            torch.cuda.synchronize()
            Es.append(ctx.energy(y.detach())[0].item())
    torch.cuda.synchronize()
    E1 = ctx.energy(y.detach())[0].item()
    log(f"  2000 autograd Adam steps: F_h {E0:.6g} -> {E1:.6g} (every 499: {Es})")
    assert torch.isfinite(y).all()
    assert abs(y.double().mean().item() + 0.3) < 1e-5
    assert np.isfinite(Es).all() and E1 < 0.5 * E0


def test_config_256cubed_1000_steps():
    """The 256^3 benchmark workload for 1000 mass-projected steps (tau = 1e-3, graph
    replays): energies finite and falling from call to call, the mean kept to FP32
    rounding."""
    n = 256
    h = 1.0 / n
    u = to_dev(inputs.uniform_noise(n, 1005), torch.float32)
    m = float(u.double().mean().item())
    ctx = fe.FeContext((1, n, n, n), h, 1.5 * h, HELFRICH_SC, dtype=torch.float32)
    Es = [ctx.energy(u)[0].item()]
    for _ in range(4):
        Es.append(ctx.step(u, [m], 1e-3, 250)[0].item())
    Es.append(ctx.energy(u)[0].item())
    log(f"  1000 steps at 256^3: F_h {Es}")
    assert np.isfinite(Es).all() and all(b < a for a, b in zip(Es, Es[1:]))
    assert abs(u.double().mean().item() - m) < 1e-6


def _adam_reference(U0, h, eps, a, m, nsteps, vtol):
    """The oracle's mass-projected Adam trajectory from U0 and the voxels whose update the
    FP32 path cannot be expected to reproduce: those where the oracle's gradient at some
    step is within the FP32 gradient's per-voxel error bound of zero (|go| <= vtol (|go| +
    rms go)), so that its sign, which alone sets Adam's first move, is a rounding decision.
    A move there changes the gradient up to two voxels away at the next step, so the set
    grows by two voxels per later step (periodically)."""
    from scipy.ndimage import maximum_filter
    u, m1, m2 = U0.copy(), np.zeros_like(U0), np.zeros_like(U0)
    undecided = np.zeros(U0.shape, dtype=bool)
    for t in range(1, nsteps + 1):
        if t > 1:
            undecided = maximum_filter(undecided, size=5, mode="wrap")
        _, go = fo.energy_grad(u, h, eps, a)
        undecided |= np.abs(go) <= vtol * (np.abs(go) + np.sqrt(np.mean(go * go)))
        u, m1, m2, _ = fo.adam_projected_step(u, m1, m2, t, h, eps, a, m)
    return u, undecided


def _check_adam_update(d_got, d_ref, undecided, lr, what):
    """Update against the oracle's: relative L2 over the field; every voxel within the
    per-voxel bound except where a sign decision could reach (undecided), which must be
    rare; and every move a valid Adam move (at most about lr per step plus the shift)."""
    l2 = rel_l2(d_got, d_ref)
    ve = voxel_errors(d_got, d_ref)
    tol = TOL[torch.float32]["voxel"]
    bad = ve > tol
    worst = float(ve[~undecided].max()) if (~undecided).any() else 0.0
    log(f"  {what}: update rel L2 {l2:.2e}, worst voxel {float(ve.max()):.2e}, voxels beyond {tol:g}: "
        f"{int(bad.sum())}, worst outside the {int(undecided.sum())} undecided voxels {worst:.2e}")
    assert l2 <= 1e-3, (what, l2)
    assert not (bad & ~undecided).any(), (what, worst)
    assert bad.mean() <= 1e-3, (what, int(bad.sum()))
    assert np.abs(d_got).max() <= 1.01 * np.abs(d_ref).max() + 10 * lr


def test_fp32_adam_steps_match_oracle_128():
    """The asymmetric 128^3 workload (u0 ~ U(-1,1) seed 1003, eps = 2h, a = (1, 0, 0.2, -4,
    -4, 0), target mean -0.3): three FP32 mass-projected Adam steps (lr 1e-3) in the default
    launch against the oracle's FP64 steps, at every voxel."""
    n = 128
    h = 1.0 / n
    ud = to_dev(inputs.uniform_noise(n, 1003), torch.float32)
    U0 = oracle_input(ud)
    ctx = fe.FeContext((1, n, n, n), h, 2 * h, ASYM_C3, dtype=torch.float32)
    ctx.step_adam(ud, [-0.3], 3)
    uo, undecided = _adam_reference(U0, h, 2 * h, ASYM_C3, -0.3, 3, TOL[torch.float32]["voxel"])
    _check_adam_update(ud.cpu().double().numpy() - U0, uo - U0, undecided, 1e-3, "128^3 3 Adam steps")
    assert abs(ud.double().mean().item() + 0.3) <= 1e-6


def test_fp32_adam_step_matches_oracle_batched_16x128():
    """One FP32 Adam step of the batched workload (16 x 128^3, per-instance coefficients and
    means, the launch the batched benchmark times) against the oracle, every instance."""
    n, B = 128, 16
    h = 1.0 / n
    coeffs, means = inputs.random_instance_table(B, 4999)
    ud = torch.stack([to_dev(inputs.uniform_noise(n, 4000 + b), torch.float32) for b in range(B)])
    U0 = [oracle_input(ud[b]) for b in range(B)]
    ctx = fe.FeContext(ud.shape, h, 2 * h, coeffs, dtype=torch.float32)
    ctx.step_adam(ud, list(means), 1)
    for b in range(B):
        uo, undecided = _adam_reference(U0[b], h, 2 * h, coeffs[b], means[b], 1, TOL[torch.float32]["voxel"])
        _check_adam_update(ud[b].cpu().double().numpy() - U0[b], uo - U0[b], undecided, 1e-3, f"instance {b}")


@pytest.mark.parametrize("a", [ALL_TERMS, ASYM_C3], ids=["allterms", "asym"])
def test_autograd_function_against_finite_differences_8cubed(a):
    """FeEnergy in FP64 on an 8^3 grid (u ~ U(-1,1), eps = 2h): the gradient that backward
    returns (the adjoint sweep) against central differences of the energy that forward
    returns (the energy-only sweep), at every voxel with one Richardson step, and along a
    random direction; and against the oracle's gradient."""
    n = 8
    h = 1.0 / n
    u0 = inputs.uniform_noise(n, 808)
    ctx = fe.FeContext((1, n, n, n), h, 2 * h, a, dtype=torch.float64)
    u = to_dev(u0, torch.float64).requires_grad_(True)
    fe.feps(u, ctx).sum().backward()
    g = u.grad.detach().cpu().numpy()

    def energy(x):
        with torch.no_grad():
            return fe.feps(x, ctx).sum().item()

    base = to_dev(u0, torch.float64)
    flat = base.view(-1)

    def central(i, d):
        flat[i] += d
        ep = energy(base)
        flat[i] -= 2 * d
        em = energy(base)
        flat[i] += d
        return (ep - em) / (2 * d)

    fd = np.array([(4.0 * central(i, 5e-7) - central(i, 1e-6)) / 3.0 for i in range(n ** 3)]).reshape(g.shape)
    err = rel_l2(g, fd)
    v = torch.from_numpy(np.random.default_rng(3).normal(size=u0.shape)).cuda()

    def along(d):
        return (energy(base + d * v) - energy(base - d * v)) / (2 * d)

    dv = (4.0 * along(5e-7) - along(1e-6)) / 3.0
    gv = float(np.sum(g * v.cpu().numpy()))
    _, go = fo.energy_grad(u0, h, 2 * h, a)
    log(f"  FeEnergy 8^3: FD rel L2 {err:.2e}, direction rel {abs(gv - dv) / abs(dv):.2e}, "
        f"oracle rel L2 {rel_l2(g, go):.2e}")
    assert err <= 1e-6
    assert abs(gv - dv) <= 1e-7 * abs(dv)
    assert rel_l2(g, go) <= 1e-9


def test_adam_in_a_mixed_batch_equals_each_instance_alone():
    """A batch that mixes a p symmetric in k1, k2 (no S~ terms) with an asymmetric one runs
    the sweep that picks the body per instance; alone, each runs a single-body sweep. Both
    take the same body (the Adam sweep too), so three Adam steps agree to rounding (the two
    kernels may contract multiply-adds differently) in FP32 and FP64."""
    n = 20
    h = 1.0 / n
    coeffs = [HELFRICH_SC, ASYM_C3]
    U = np.stack([inputs.uniform_noise(n, 310 + b) for b in range(2)])
    for dtype in (torch.float32, torch.float64):
        ctx = fe.FeContext(U.shape, h, 2 * h, coeffs, dtype=dtype)
        ub = to_dev(U, dtype)
        ctx.step_adam(ub, [0.0, -0.2], 3)
        for b in range(2):
            c1 = fe.FeContext((1, n, n, n), h, 2 * h, coeffs[b], dtype=dtype)
            c1.set_launch(*ctx.get_launch())
            u1 = to_dev(U[b:b + 1], dtype)
            c1.step_adam(u1, [[0.0, -0.2][b]], 3)
            assert_same_to_rounding(u1[0] - to_dev(U[b], dtype), ub[b] - to_dev(U[b], dtype), dtype, (dtype, b))
