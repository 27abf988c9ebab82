"""Seeded synthetic inputs for the energy, the gradient and the descent loop.

This module only makes initial fields and coefficient tables; it holds none of
the energy's arithmetic and imports nothing else from this package, so both the
HIP path's tests and the FP64 oracle's tests draw from it.

Fields are float64 numpy arrays indexed [z, y, x] on the periodic unit cube
[0, 1)^3 with N samples per axis at cell centres x_i = (i + 1/2) h, h = 1/N.
Shapes use the tanh profile u = tanh(d / (sqrt(2) eps)) of eq. (tanh_profile),
with d the minimum-image signed distance (positive inside, u ~ +1 inside).
"""

import math

import numpy as np


def cell_centres(n):
    h = 1.0 / n
    return (np.arange(n) + 0.5) * h


def _min_image(x, c):
    d = x - c
    return d - np.round(d)


def _mesh(n):
    x = cell_centres(n)
    return np.meshgrid(x, x, x, indexing="ij")    # [z, y, x] order: Z, Y, X


def uniform_noise(n, seed, lo=-1.0, hi=1.0, batch=None):
    """u0 ~ U(lo, hi) i.i.d. per voxel, from numpy's default_rng(seed)."""
    rng = np.random.default_rng(seed)
    shape = (n, n, n) if batch is None else (batch, n, n, n)
    return rng.uniform(lo, hi, size=shape)


def tanh_sphere(n, radius, eps, centre=(0.5, 0.5, 0.5)):
    """Ball of the given radius: d = radius - |x - centre| (minimum image)."""
    Z, Y, X = _mesh(n)
    r = np.sqrt(_min_image(X, centre[0]) ** 2 + _min_image(Y, centre[1]) ** 2
                + _min_image(Z, centre[2]) ** 2)
    return np.tanh((radius - r) / (math.sqrt(2.0) * eps))


def tanh_cylinder(n, radius, eps, axis="z", centre=(0.5, 0.5)):
    """Infinite (periodic) solid cylinder along `axis` with the given radius."""
    Z, Y, X = _mesh(n)
    coords = {"x": X, "y": Y, "z": Z}
    others = [k for k in "xyz" if k != axis]
    r = np.sqrt(_min_image(coords[others[0]], centre[0]) ** 2
                + _min_image(coords[others[1]], centre[1]) ** 2)
    return np.tanh((radius - r) / (math.sqrt(2.0) * eps))


def tanh_slab(n, half_width, eps, axis="x", centre=0.5):
    """Slab |x_axis - centre| < half_width (two parallel planes)."""
    Z, Y, X = _mesh(n)
    c = {"x": X, "y": Y, "z": Z}[axis]
    return np.tanh((half_width - np.abs(_min_image(c, centre))) / (math.sqrt(2.0) * eps))


def noisy_sphere(n, radius, eps, noise_std, seed):
    """tanh sphere plus i.i.d. N(0, noise_std^2) noise from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    return tanh_sphere(n, radius, eps) + rng.normal(0.0, noise_std, size=(n, n, n))


def random_instance_table(batch, seed):
    """Per-instance polynomial and mass draws for a batch of independent textures.

    p = a k1^2 + b k2^2 + c k1 k2 + d (k1 + k2), a, b ~ U(0, 2), c ~ U(-1, 1),
    d ~ U(-6, 0); returns (coeffs[batch, 6] in (a20, a11, a02, a10, a01, a00)
    order, target means[batch] ~ U(-0.5, 0.5)).
    """
    rng = np.random.default_rng(seed)
    A = rng.uniform(0.0, 2.0, batch)
    B = rng.uniform(0.0, 2.0, batch)
    C = rng.uniform(-1.0, 1.0, batch)
    D = rng.uniform(-6.0, 0.0, batch)
    coeffs = np.stack([A, C, B, D, D, np.zeros(batch)], axis=1)
    means = rng.uniform(-0.5, 0.5, batch)
    return coeffs, means


def white_noise_vector_field(n, seed, std, batch=None):
    """A0 ~ N(0, std^2) i.i.d. per voxel and component: the random initial vector field
    of Algorithm 1. Shape [3, n, n, n] (components x, y, z) or [batch, 3, n, n, n]; n may
    also be a grid shape (nz, ny, nx)."""
    rng = np.random.default_rng(seed)
    grid = (n, n, n) if np.isscalar(n) else tuple(n)
    shape = (3,) + grid if batch is None else (batch, 3) + grid
    return rng.normal(0.0, std, size=shape)


def interpolated_parameters(shape, params, masses, repeat_ends=True):
    """Space-dependent generation parameters varying along x only, for a grid of
    `shape` = (nz, ny, nx): the x-axis is cut into equal cells whose mid-planes
    carry the given parameter sets, and the values in between are linear
    interpolations between neighbouring mid-planes, periodic across the
    boundary. With repeat_ends the first and last sets are each used twice
    (p1, p1, p2, ..., pk, pk), the layout of the paper's spatialised example.

    params: k coefficient vectors (a20, a11, a02, a10, a01, a00); masses: k values.
    Returns (a_field [6, nz, ny, nx], m_field [nz, ny, nx]) in float64.
    """
    nz, ny, nx = shape
    P = np.asarray(params, dtype=np.float64)
    M = np.asarray(masses, dtype=np.float64)
    if repeat_ends:
        P = np.concatenate([P[:1], P, P[-1:]])
        M = np.concatenate([M[:1], M, M[-1:]])
    k = len(P)
    xc = (np.arange(nx) + 0.5) / nx * k - 0.5        # position in cell units from the first mid-plane
    i0 = np.floor(xc).astype(np.int64)
    t = xc - i0
    lo, hi = i0 % k, (i0 + 1) % k
    a_x = P[lo] * (1 - t)[:, None] + P[hi] * t[:, None]      # [nx, 6]
    m_x = M[lo] * (1 - t) + M[hi] * t
    a_field = np.broadcast_to(a_x.T[:, None, None, :], (6, nz, ny, nx)).copy()
    m_field = np.broadcast_to(m_x[None, None, :], (nz, ny, nx)).copy()
    return a_field, m_field


def tanh_torus(n, R, r, eps, centre=(0.5, 0.5, 0.5)):
    """Solid torus around the z axis through `centre`: major radius R, tube radius r,
    d = r - sqrt((rho - R)^2 + z^2) with rho the distance to the axis."""
    Z, Y, X = _mesh(n)
    x, y, z = X - centre[0], Y - centre[1], Z - centre[2]
    d = r - np.sqrt((np.sqrt(x * x + y * y) - R) ** 2 + z * z)
    return np.tanh(d / (math.sqrt(2.0) * eps))
