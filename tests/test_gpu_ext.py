"""The Sec. 5.2 extensions on the GPU against the oracle: the orientation term
eps mu (theta . grad u)^2 in the energy, its gradient, the steps and the flow."""

import numpy as np
import pytest
import torch

from oracle import fe_oracle as fo
from paper_2103_04856_amd import fe, inputs

from gpu_helpers import ALL_TERMS, ASYM_C3, TOL, WILLMORE_QUARTER, oracle_input, check_field, rel_l2, to_dev

pytestmark = pytest.mark.gpu

THETA = (1 / 3, 2 / 3, -2 / 3)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_orientation_energy_and_gradient(dtype):
    """Two instances on a ragged 40 x 36 x 28 grid, one with mu = 0, one with the term on."""
    nz, ny, nx = 28, 36, 40
    h = 1.0 / 40
    U = np.stack([inputs.uniform_noise(40, 5)[:nz, :ny, :nx], inputs.uniform_noise(40, 6)[:nz, :ny, :nx]])
    Ud = to_dev(U, dtype)
    eps = [2 * h, 1.5 * h]
    coeffs = [ALL_TERMS, ASYM_C3]
    mus = [0.0, 40.0]
    ctx = fe.FeContext(Ud.shape, h, eps, coeffs, dtype=dtype)
    ctx.set_orientation(mus, [THETA, THETA])
    E, g = ctx.energy_grad(Ud)
    E_only = ctx.energy(Ud)
    stats, _, _ = ctx.diagnostics(Ud)          # its F_h carries the term too
    Uo = oracle_input(Ud)
    tol = TOL[dtype]
    for b in range(2):
        orient = (mus[b], THETA)
        Eo, go = fo.energy_grad(Uo[b], h, eps[b], coeffs[b], orient=orient)
        scale = max(abs(Eo), fo.energy_abs(Uo[b], h, eps[b], coeffs[b], orient=orient))
        assert abs(E[b].item() - Eo) <= tol["energy"] * scale
        assert abs(E_only[b].item() - Eo) <= tol["energy"] * scale
        assert abs(stats[b, 0].item() - Eo) <= tol["energy"] * scale
        check_field(g[b].cpu().double().numpy(), go, tol, f"instance {b}")
    # the term changes the result of the second instance only
    ctx.set_orientation([0.0, 0.0], [THETA, THETA])
    E0, g0 = ctx.energy_grad(Ud)
    assert E0[0].item() == E[0].item() and torch.equal(g0[0], g[0])
    assert E0[1].item() != E[1].item()


def test_orientation_steps_and_flow_match_oracle_fp64():
    """Five mass-projected steps and three Algorithm 1 iterations with the term on."""
    n = 20
    h = 1.0 / n
    orient = (25.0, (0.0, 0.6, 0.8))
    u0 = inputs.uniform_noise(n, 31)
    ctx = fe.FeContext((1, n, n, n), h, 2 * h, WILLMORE_QUARTER, dtype=torch.float64)
    ctx.set_orientation([orient[0]], [orient[1]])
    ud = to_dev(u0, torch.float64)
    uo = oracle_input(ud)
    Eg = ctx.step(ud, [0.1], 1e-3, 5)
    uo, Es = fo.descend(uo, h, 2 * h, WILLMORE_QUARTER, 0.1, 1e-3, 5, orient=orient)
    assert rel_l2(ud.cpu().numpy(), uo) <= 1e-10
    assert abs(Eg[0].item() - Es[-1]) <= 1e-10 * abs(Es[-1])
    Ad = to_dev(inputs.white_noise_vector_field(n, 32, 0.4 * h)[None], torch.float64)
    Ao = oracle_input(Ad)[0]
    Gg = ctx.hminus_step(Ad, [-0.2], 3, sigma_k=1.0)
    Ao, Gs, _ = fo.hminus_descend(Ao, h, 2 * h, WILLMORE_QUARTER, -0.2, 1.0, 3, orient=orient)
    assert rel_l2(Ad.cpu().numpy()[0], Ao) <= 1e-10
    assert abs(Gg[0].item() - Gs[-1]) <= 1e-10 * abs(Gs[-1])


def test_orientation_rejects_non_finite():
    ctx = fe.FeContext((1, 8, 8, 8), 1 / 8, 0.25, WILLMORE_QUARTER, dtype=torch.float32)
    with pytest.raises(fe.FeError, match="mu"):
        ctx.set_orientation([float("nan")], [THETA])
    with pytest.raises(fe.FeError, match="theta"):
        ctx.set_orientation([1.0], [(0.0, float("inf"), 0.0)])
