"""Seeded random configurations against the oracle: grid shapes from 1 to 20 per
axis (no relation to the tiles), batches of 1-3 instances with their own eps,
coefficients (every term, either sign) and orientation terms, both precisions,
random launch variants and z chunks; smooth and rough fields."""

import math

import numpy as np
import pytest
import torch

from oracle import fe_oracle as fo
from paper_2103_04856_amd import fe

from gpu_helpers import TOL, log, oracle_input, check_field, rel_l2, to_dev

pytestmark = pytest.mark.gpu

N_CASES = 24


def _case(seed):
    rng = np.random.default_rng(seed)
    shape = tuple(int(v) for v in rng.integers(1, 21, size=3))        # (nz, ny, nx)
    B = int(rng.integers(1, 4))
    h = 1.0 / max(shape)
    eps = [float(rng.uniform(1.2, 3.0)) * h for _ in range(B)]
    coeffs = [tuple(float(v) for v in rng.uniform(-5, 5, size=6)) for _ in range(B)]
    mus = [0.0 if rng.random() < 0.5 else float(rng.uniform(0, 50)) for _ in range(B)]
    thetas = []
    for _ in range(B):
        t = rng.standard_normal(3)
        thetas.append(tuple(float(v) for v in t / np.linalg.norm(t)))
    if rng.random() < 0.5:
        U = rng.uniform(-1, 1, size=(B,) + shape)
    else:                                                              # smooth: a few Fourier modes
        z, y, x = np.meshgrid(*[np.arange(k) / k for k in shape], indexing="ij")
        U = np.stack([np.tanh(2 * np.sin(2 * math.pi * (x + rng.random())) * np.cos(2 * math.pi * (y + z))
                              + 0.1 * rng.standard_normal(shape)) for _ in range(B)])
    dtype = torch.float64 if rng.random() < 0.5 else torch.float32
    return shape, B, h, eps, coeffs, mus, thetas, U, dtype, rng


@pytest.mark.parametrize("seed", range(N_CASES))
def test_random_configuration_matches_oracle(seed):
    shape, B, h, eps, coeffs, mus, thetas, U, dtype, rng = _case(7000 + seed)
    ctx = fe.FeContext((B,) + shape, h, eps, coeffs, dtype=dtype)
    ctx.set_orientation(mus, thetas)
    mask = 1 if dtype == torch.float32 else 2
    choices = [vi for vi, v in enumerate(fe.variants()) if v[3] & mask]
    vi = int(rng.choice(choices))
    zc = int(rng.choice([0, 1, 2, 3, 5, 8]))
    ctx.set_launch(vi, zc)
    log(f"case seed={7000 + seed} shape={shape} B={B} {dtype} variant={fe.variants()[vi][:3]} zc={zc}")
    ud = to_dev(U, dtype)
    E, g = ctx.energy_grad(ud)
    E_only = ctx.energy(ud)
    Uo = oracle_input(ud)
    tol = TOL[dtype]
    for b in range(B):
        orient = (mus[b], thetas[b]) if mus[b] else None
        Eo, go = fo.energy_grad(Uo[b], h, eps[b], coeffs[b], orient=orient)
        scale = max(abs(Eo), fo.energy_abs(Uo[b], h, eps[b], coeffs[b], orient=orient))
        assert abs(E[b].item() - Eo) <= tol["energy"] * scale, (b, E[b].item(), Eo)
        assert abs(E_only[b].item() - Eo) <= tol["energy"] * scale, (b, E_only[b].item(), Eo)
        if np.linalg.norm(go) > 0:
            check_field(g[b].cpu().double().numpy(), go, tol, b)
