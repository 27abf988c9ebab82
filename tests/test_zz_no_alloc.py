"""The allocation-free entry point fe_energy_grad_noalloc against the context's
fe_energy_grad_async (the same kernels in the same launch shape): bit for bit, on two
calls in a row (the second on a smaller grid, so that it must not see the first
call's leftovers in the shared static workspace), and its argument checks."""

import ctypes

import numpy as np
import pytest
import torch

from paper_2103_04856_amd import fe, inputs

from gpu_helpers import ALL_TERMS, ASYM_C3, HELFRICH_SC, log, to_dev

pytestmark = pytest.mark.gpu


def _reference(U, h, eps, coeffs, dtype, with_grad):
    ctx = fe.FeContext(U.shape, h, eps, coeffs, dtype=dtype)
    E, g = ctx.energy_grad_async(U, with_grad=with_grad)
    torch.cuda.synchronize()
    ctx.close()
    return E, g


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noalloc_equals_the_context_entry_point(dtype):
    cases = [  # (shape [B, nz, ny, nx], eps/h, coefficients): larger first, then smaller
        ((3, 40, 36, 50), 2.0, [ALL_TERMS, ASYM_C3, HELFRICH_SC]),
        ((2, 9, 13, 20), 1.5, [HELFRICH_SC, ALL_TERMS]),
    ]
    for shape, eps_h, coeffs in cases:
        B, nz, ny, nx = shape
        h = 1.0 / nx
        rng = np.random.default_rng(90 + B)
        U = to_dev(rng.uniform(-1, 1, size=shape), dtype)
        for with_grad in (True, False):
            log(f"case noalloc {dtype} shape={shape} grad={with_grad}")
            Er, gr = _reference(U, h, [eps_h * h] * B, coeffs, dtype, with_grad)
            E, g = fe.energy_grad_noalloc(U, h, [eps_h * h] * B, coeffs, with_grad=with_grad)
            torch.cuda.synchronize()
            assert torch.equal(E, Er), (E, Er)
            if with_grad:
                assert torch.equal(g, gr)


def test_noalloc_full_size_bench_grid():
    """256^3 FP32 (the benchmark's field), then 16 x 128^3 (the batched one): the same bits
    as the context path."""
    for n, B in ((256, 1), (128, 16)):
        h = 1.0 / n
        log(f"case noalloc full {B} x {n}^3")
        U = torch.stack([to_dev(inputs.uniform_noise(n, 1005 + b), torch.float32) for b in range(B)])
        coeffs = [HELFRICH_SC if b % 2 == 0 else ASYM_C3 for b in range(B)]
        Er, gr = _reference(U, h, [1.5 * h] * B, coeffs, torch.float32, True)
        E, g = fe.energy_grad_noalloc(U, h, [1.5 * h] * B, coeffs)
        torch.cuda.synchronize()
        assert torch.equal(E, Er) and torch.equal(g, gr)


def test_noalloc_rejects_what_it_cannot_hold():
    """A batch above 16 and a grid whose sweep needs more block partials than the static
    array holds are rejected before anything is launched (the field passed with the
    oversized grid is a small real tensor that the call never reads)."""
    u = torch.zeros((17, 4, 4, 4), dtype=torch.float32, device="cuda")
    with pytest.raises(fe.FeError) as ei:
        fe.energy_grad_noalloc(u, 0.25, 0.5, ASYM_C3)
    assert ei.value.code == fe.FE_EINVAL and "16" in str(ei.value)
    grid = fe.FeGrid(8192, 8192, 1, 1, 1e-3, fe.FE_F32)    # 256 x 256 tile columns > 65280
    g = torch.zeros_like(u)
    rc = fe.lib().fe_energy_grad_noalloc(ctypes.byref(grid), fe._dbl([2e-3]), fe._dbl(list(ASYM_C3)),
                                         ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(g.data_ptr()),
                                         ctypes.c_void_p(0), None)
    assert rc == fe.FE_EINVAL and "partials" in fe.lib().fe_last_error().decode()
