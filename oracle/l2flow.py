"""Algorithm 2 (Sec. 4.2): the L2 flow of F_eps with replicate boundary conditions,
driven by L-BFGS, as used to validate the method on Willmore minimizers.

TEST INFRASTRUCTURE ONLY (see the oracle package header).

Readings:
* replicate padding: a sample outside the box takes the value of the nearest
  box voxel (each axis clamped); this is the padding of the finite differences
  and of the blur (Sec. 4.2 footnote: grad u . n = 0 on the boundary);
* the blur acts on u before the energy, as in Algorithm 1: the flow minimises
  F_h(k * u) over u, with k applied to the replicate-padded field;
* F_h sums the density over the box voxels only;
* the optimiser is L-BFGS as provided by torch.optim.LBFGS (lr, history size,
  iterations per step as in Sec. 4.2), driven by the oracle's FP64 energy and
  gradient.

The gradient is the exact one of that finite sum: the per-voxel adjoints of the
padded field (zero outside the box) go through the transposed stencils, and the
transpose of the padding adds every pad sample's derivative onto the box voxel it
copies (the same for the blur's padding).
"""

import numpy as np

from .fe_oracle import XI, adjoint_fields, gaussian_blur, gaussian_weights, pointwise, transpose_stencils


def pad_replicate(u, w):
    """Edge padding by w samples on every side of every axis."""
    return np.pad(np.asarray(u, dtype=np.float64), w, mode="edge") if w else np.asarray(u, dtype=np.float64)


def pad_replicate_adjoint(g, w):
    """Transpose of pad_replicate: pad samples added onto the box voxels they copy."""
    out = np.asarray(g, dtype=np.float64)
    if not w:
        return out.copy()
    for axis in range(3):
        a = np.moveaxis(out, axis, 0)
        inner = a[w:-w].copy()
        inner[0] += a[:w].sum(axis=0)
        inner[-1] += a[-w:].sum(axis=0)
        out = np.moveaxis(inner, 0, axis)
    return out


def blur_replicate(u, sigma_k):
    """k * u with replicate padding: the periodic blur of the padded field, cropped
    (the padding is as wide as the kernel, so no sample wraps)."""
    r = (len(gaussian_weights(sigma_k)) - 1) // 2
    if r == 0:
        return np.asarray(u, dtype=np.float64).copy()
    return gaussian_blur(pad_replicate(u, r), sigma_k)[r:-r, r:-r, r:-r]


def blur_replicate_adjoint(g, sigma_k):
    """Transpose of blur_replicate: zero-extend, blur (the kernel is even), fold the pads."""
    r = (len(gaussian_weights(sigma_k)) - 1) // 2
    if r == 0:
        return np.asarray(g, dtype=np.float64).copy()
    return pad_replicate_adjoint(gaussian_blur(np.pad(g, r), sigma_k), r)


def energy_replicate(u, h, eps, a, sigma_k=0.0, xi=XI, mode="smooth", orient=None):
    """F_h(k * u) = h^3 sum over the box of the density, with replicate padding."""
    ue = pad_replicate(blur_replicate(u, sigma_k), 1)
    f = pointwise(ue, h, eps, a, xi, mode, orient)["f"][1:-1, 1:-1, 1:-1]
    return float(h ** 3 * np.sum(f))


def energy_grad_replicate(u, h, eps, a, sigma_k=0.0, xi=XI, mode="smooth", orient=None):
    """(F_h(k * u), dF/du) with replicate boundaries."""
    ub = blur_replicate(u, sigma_k)
    ue = pad_replicate(ub, 1)
    ubar, gamma, theta, fw = adjoint_fields(ue, h, eps, a, xi, mode, orient)
    box = np.zeros(ue.shape, dtype=bool)
    box[1:-1, 1:-1, 1:-1] = True
    ubar = np.where(box, ubar, 0.0)
    gamma = [np.where(box, g, 0.0) for g in gamma]
    theta = [np.where(box, t, 0.0) for t in theta]
    E = float(h ** 3 * np.sum(fw["f"][box]))
    g_ext = h ** 3 * transpose_stencils(ubar, gamma, theta, h)
    return E, blur_replicate_adjoint(pad_replicate_adjoint(g_ext, 1), sigma_k)


def lbfgs_flow(u0, h, eps, a, sigma_k, nsteps, lr=1.0, history=10, max_iter=20, tolerance_grad=1e-7,
               tolerance_change=1e-9, xi=XI, orient=None):
    """nsteps calls of torch.optim.LBFGS.step (no line search, FP64 on the CPU) on
    F_h(k * u) with replicate boundaries. Returns (u, [F_h before each step])."""
    import torch
    x = torch.tensor(np.asarray(u0, dtype=np.float64), requires_grad=True)
    opt = torch.optim.LBFGS([x], lr=lr, history_size=history, max_iter=max_iter,
                            tolerance_grad=tolerance_grad, tolerance_change=tolerance_change)

    def closure():
        E, g = energy_grad_replicate(x.detach().numpy(), h, eps, a, sigma_k, xi, orient=orient)
        x.grad = torch.from_numpy(np.ascontiguousarray(g))
        return torch.tensor(E, dtype=torch.float64)

    energies = []
    for _ in range(nsteps):
        energies.append(float(opt.step(closure)))
    return x.detach().numpy(), energies
