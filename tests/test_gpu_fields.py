"""Space-dependent coefficients a(x) and mass m(x) (Sec. 5.2) on the GPU against
the oracle: energy, gradient, steps, the flow and the diagnostics."""

import numpy as np
import pytest
import torch

from oracle import classical, fe_oracle as fo
from paper_2103_04856_amd import fe, inputs

from gpu_helpers import ALL_TERMS, ASYM_C3, TOL, WILLMORE_QUARTER, oracle_input, check_field, rel_l2, to_dev

pytestmark = pytest.mark.gpu

# the four parameter sets of the paper's spatialised example (Sec. 5.2 table), with their masses
SPATIAL_SETS = [(2, 2, 2, 0, 0, 0), (1, 2, 6, -40, -40, 400), (2, 2, 2, -75, -75, 937.5), (2, 2, 11, -180, -90, 4050)]
SPATIAL_MASSES = [-0.4, -0.6, -0.7, -0.7]


def _random_field(B, shape, seed):
    """a(x) around ALL_TERMS with +-50% voxel noise: [B, 6, nz, ny, nx]."""
    rng = np.random.default_rng(seed)
    base = np.asarray(ALL_TERMS)[None, :, None, None, None]
    return base * (1 + 0.5 * rng.uniform(-1, 1, size=(B, 6) + tuple(shape)))


def _oracle_a(a_dev, b):
    return list(oracle_input(a_dev)[b])


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_constant_field_equals_instance_coefficients(dtype):
    n = 24
    h = 1.0 / n
    u = to_dev(inputs.uniform_noise(n, 2)[None], dtype)
    ctx = fe.FeContext(u.shape, h, 2 * h, ASYM_C3, dtype=dtype)
    E0, g0 = ctx.energy_grad(u)
    af = torch.tensor(ASYM_C3, dtype=dtype, device="cuda").reshape(1, 6, 1, 1, 1).expand(1, 6, n, n, n).contiguous()
    ctx.set_coeff_field(af)
    E1, g1 = ctx.energy_grad(u)
    tol = 1e-13 if dtype == torch.float64 else 1e-5
    assert abs(E1[0].item() - E0[0].item()) <= tol * abs(E0[0].item())
    assert rel_l2(g1.cpu().double().numpy(), g0.cpu().double().numpy()) <= tol
    ctx.set_coeff_field(None)
    E2, g2 = ctx.energy_grad(u)
    assert E2[0].item() == E0[0].item() and torch.equal(g2, g0)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_random_field_matches_oracle_on_every_variant(dtype):
    """Batch of 2 on a ragged 36 x 28 x 20 grid; every launch variant (those without
    coefficient-field kernels hand over to one that has them)."""
    nz, ny, nx = 20, 28, 36
    h = 1.0 / 36
    U = np.stack([inputs.uniform_noise(36, 7)[:nz, :ny, :nx], inputs.uniform_noise(36, 8)[:nz, :ny, :nx]])
    Ud = to_dev(U, dtype)
    eps = [2 * h, 1.5 * h]
    ad = to_dev(_random_field(2, (nz, ny, nx), 9), dtype)
    ctx = fe.FeContext(Ud.shape, h, eps, [ALL_TERMS, ASYM_C3], dtype=dtype)
    ctx.set_orientation([0.0, 30.0], [(0, 0, 1), (0.6, 0.8, 0.0)])
    ctx.set_coeff_field(ad)
    Uo = oracle_input(Ud)
    ref = []
    for b in range(2):
        orient = (0.0, (0, 0, 1)) if b == 0 else (30.0, (0.6, 0.8, 0.0))
        a_b = _oracle_a(ad, b)
        Eo, go = fo.energy_grad(Uo[b], h, eps[b], a_b, orient=orient)
        ref.append((Eo, go, max(abs(Eo), fo.energy_abs(Uo[b], h, eps[b], a_b, orient=orient))))
    tol = TOL[dtype]
    mask = 1 if dtype == torch.float32 else 2
    for vi, (tx, ty, nt, m) in enumerate(fe.variants()):
        if not m & mask:
            continue
        ctx.set_launch(vi, 0)
        E, g = ctx.energy_grad(Ud)
        E_only = ctx.energy(Ud)
        for b in range(2):
            Eo, go, scale = ref[b]
            assert abs(E[b].item() - Eo) <= tol["energy"] * scale, (vi, b)
            assert abs(E_only[b].item() - Eo) <= tol["energy"] * scale, (vi, b)
            check_field(g[b].cpu().double().numpy(), go, tol, (vi, b))


def test_steps_and_graph_replay_with_a_field():
    """FP64: five mass-projected steps against the oracle; FP32: 19 Adam steps in one
    call (graph replays) equal 19 single calls bitwise."""
    n = 20
    h = 1.0 / n
    ad = to_dev(_random_field(1, (n, n, n), 3), torch.float64)
    ctx = fe.FeContext((1, n, n, n), h, 2 * h, WILLMORE_QUARTER, dtype=torch.float64)
    ctx.set_coeff_field(ad)
    ud = to_dev(inputs.uniform_noise(n, 4)[None], torch.float64)
    uo = oracle_input(ud)[0]
    Eg = ctx.step(ud, [0.0], 1e-4, 5)
    uo, Es = fo.descend(uo, h, 2 * h, _oracle_a(ad, 0), 0.0, 1e-4, 5)
    assert rel_l2(ud.cpu().numpy()[0], uo) <= 1e-10
    assert abs(Eg[0].item() - Es[-1]) <= 1e-10 * abs(Es[-1])
    c32 = fe.FeContext((1, n, n, n), h, 2 * h, WILLMORE_QUARTER, dtype=torch.float32)
    c32.set_coeff_field(ad.float())
    u1 = to_dev(inputs.uniform_noise(n, 4)[None], torch.float32)
    u2 = u1.clone()
    E1 = c32.step_adam(u1, [0.0], 19)
    c32.adam_reset()
    for _ in range(19):
        E2 = c32.step_adam(u2, [0.0], 1)
    assert torch.equal(u1, u2) and E1[0].item() == E2[0].item()


def test_flow_with_mass_and_coefficient_fields_matches_oracle_fp64():
    """Algorithm 1 with u = k * (div A + m(x)) and a(x) from the paper's interpolated
    parameter sets: three iterations against the oracle, and mean(u) = mean(m)."""
    nz, ny, nx = 16, 16, 24
    h = 1.0 / 24
    a_np, m_np = inputs.interpolated_parameters((nz, ny, nx), SPATIAL_SETS, SPATIAL_MASSES)
    ad = to_dev(a_np[None], torch.float64)
    md = to_dev(m_np[None], torch.float64)
    ctx = fe.FeContext((1, nz, ny, nx), h, 2 * h, WILLMORE_QUARTER, dtype=torch.float64)
    ctx.set_coeff_field(ad)
    ctx.set_mass_field(md)
    A = to_dev(inputs.white_noise_vector_field(24, 5, 0.4 * h)[:, :nz, :ny, :nx][None], torch.float64)
    Ao = oracle_input(A)[0]
    uo_dev = torch.empty((1, nz, ny, nx), dtype=torch.float64, device="cuda")
    Gg = ctx.hminus_step(A, None, 3, sigma_k=1.0, u_out=uo_dev)
    Ao, Gs, uo = fo.hminus_descend(Ao, h, 2 * h, list(a_np), m_np, 1.0, 3)
    assert rel_l2(A.cpu().numpy()[0], Ao) <= 1e-10
    assert abs(Gg[0].item() - Gs[-1]) <= 1e-10 * abs(Gs[-1])
    assert rel_l2(uo_dev.cpu().numpy()[0], uo) <= 1e-10
    assert abs(uo_dev.mean().item() - m_np.mean()) <= 1e-13
    # without the mass field the scalar m0 is back
    ctx.set_mass_field(None)
    with pytest.raises(fe.FeError, match="m0"):
        ctx.hminus_step(A, None, 1)


def test_diagnostics_energy_uses_the_field_and_set_params_drops_it():
    n = 24
    h = 1.0 / n
    u = to_dev(inputs.noisy_sphere(n, 0.3, 2 * h, 0.02, 6)[None], torch.float64)
    ad = to_dev(_random_field(1, (n, n, n), 10), torch.float64)
    ctx = fe.FeContext(u.shape, h, 2 * h, ALL_TERMS, dtype=torch.float64)
    ctx.set_coeff_field(ad)
    stats, _, _ = ctx.diagnostics(u)
    Eo = fo.energy(oracle_input(u)[0], h, 2 * h, _oracle_a(ad, 0))
    assert abs(stats[0, 0].item() - Eo) <= 1e-10 * fo.energy_abs(oracle_input(u)[0], h, 2 * h, _oracle_a(ad, 0))
    ctx.set_params([2 * h], [ALL_TERMS])
    E = ctx.energy(u)
    Eu = fo.energy(oracle_input(u)[0], h, 2 * h, ALL_TERMS)
    assert abs(E[0].item() - Eu) <= 1e-10 * fo.energy_abs(oracle_input(u)[0], h, 2 * h, ALL_TERMS)
