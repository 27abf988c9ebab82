"""Plain FP64 CPU oracle of the discrete curvature phase-field energy F_eps.

TEST INFRASTRUCTURE ONLY. This module exists to check the HIP path. Only the
test suite, the smoke check and the CPU-baseline leg of the benchmark may import
it; the product path never does, and this module imports nothing from the
product package.

What it computes, in the order the paper defines it:

* the matrix field M = -eps Hess u + (W'(u)/eps) n (x) n of eq. (Meps), with the
  double well W(s) = (1 - s^2)^2 / 4 of Sec. 2.3 (Notations);
* the integrand of eq. (Feps), Sec. 3.2, built from Tr M, ||M||^2 and the
  positive part (2||M||^2 - (Tr M)^2)^+;
* the discretisation of Sec. 4.1 (Implementation details): the integral is a
  finite sum over a periodic voxel grid of spacing h, the derivatives are
  classical periodic finite differences, |grad u| is replaced by
  sqrt(|grad u|^2 + xi^2) and 1/|grad u| by 1/sqrt(|grad u|^2 + xi^2) with
  xi = 1e-6, and x^+ is replaced by xi log(1 + exp(x / xi));
* the exact gradient of that finite sum with respect to every voxel value,
  obtained by a hand-derived reverse-mode (adjoint) sweep;
* a mass-preserving descent step: a plain gradient step followed by the L2
  projection back onto the set {mean(u) = m}; the mass (mean) constraint is the
  one Sec. 4.1 imposes on the flow;
* the extensions of Sec. 5.2: the orientation term eps mu (theta . grad u)^2
  and space-dependent coefficients a(x) and mass m(x).

Readings where the paper leaves a choice open (all listed in the design notes):

* finite differences: second-order central differences with periodic wrap;
  the mixed second derivative uses the four diagonal neighbours, so the
  Hessian is the compact 19-point stencil and its trace is the 7-point
  Laplacian;
* the normal n (x) n = grad u grad u^T / (|grad u|^2 + xi^2); the term
  a00 eps |grad u|^2 uses the unregularised |grad u|^2;
* the smoothing scale of the positive part is the same xi = 1e-6;
* the gradient is that of F_h = h^3 sum_i f_i, i.e. the h^3 factor is kept.

Arrays are indexed [z, y, x] (x fastest), a periodic grid of N_z x N_y x N_x
samples with spacing h in every direction.
"""

import numpy as np

# Sec. 4.1 (Implementation details): offset on |grad u| and smoothing scale of x^+.
XI = 1e-6

# Component order used throughout: gradient (x, y, z); Hessian (xx, yy, zz, xy, xz, yz).
_AX = (2, 1, 0)          # numpy axis of x, y, z for arrays indexed [z, y, x]
_PAIRS = ((0, 1), (0, 2), (1, 2))


def _at(u, offsets):
    """Value at i + sum_a offsets[a] e_a with periodic wrap (offsets in x, y, z)."""
    out = u
    for a, k in enumerate(offsets):
        if k:
            out = np.roll(out, -k, axis=_AX[a])
    return out


def _unit(a, k=1):
    off = [0, 0, 0]
    off[a] = k
    return off


def _pair(a, sa, b, sb):
    off = [0, 0, 0]
    off[a] = sa
    off[b] = sb
    return off


# --------------------------------------------------------------------------
# Double well, Sec. 2.3 (Notations)
# --------------------------------------------------------------------------

def double_well(s):
    """W(s) = (1 - s^2)^2 / 4."""
    return 0.25 * (1.0 - s * s) ** 2


def double_well_prime(s):
    """W'(s) = s^3 - s."""
    return s ** 3 - s


# --------------------------------------------------------------------------
# Finite differences, Sec. 4.1 (Implementation details)
# --------------------------------------------------------------------------

def fd_gradient(u, h):
    """Periodic central differences: g_a = (u(i + e_a) - u(i - e_a)) / (2h)."""
    return [(_at(u, _unit(a)) - _at(u, _unit(a, -1))) / (2.0 * h) for a in range(3)]


def fd_hessian(u, h):
    """Compact periodic second differences, order (xx, yy, zz, xy, xz, yz).

    H_aa = (u(i+e_a) - 2u(i) + u(i-e_a)) / h^2,
    H_ab = (u(i+e_a+e_b) - u(i+e_a-e_b) - u(i-e_a+e_b) + u(i-e_a-e_b)) / (4h^2).
    """
    out = [(_at(u, _unit(a)) - 2.0 * u + _at(u, _unit(a, -1))) / (h * h) for a in range(3)]
    for a, b in _PAIRS:
        out.append((_at(u, _pair(a, 1, b, 1)) - _at(u, _pair(a, 1, b, -1))
                    - _at(u, _pair(a, -1, b, 1)) + _at(u, _pair(a, -1, b, -1))) / (4.0 * h * h))
    return out


def fd_laplacian(u, h):
    """7-point periodic Laplacian sum_a (u(i+e_a) - 2u(i) + u(i-e_a)) / h^2."""
    lap = -6.0 * u
    for a in range(3):
        lap = lap + _at(u, _unit(a)) + _at(u, _unit(a, -1))
    return lap / (h * h)


# --------------------------------------------------------------------------
# Coefficients of eq. (Feps)
# --------------------------------------------------------------------------

def feps_coefficients(a, eps):
    """Weights (c1..c6) of the six terms of eq. (Feps), Sec. 3.2.

    a = (a20, a11, a02, a10, a01, a00) in the order of Sec. 3.2.  The integrand
    is c1 ||M||^2 + c2 (Tr M)^2 + c3 Tr M S + c4 |grad u| Tr M
    + c5 |grad u| S + c6 eps |grad u|^2, with S = sqrt((2||M||^2 - (Tr M)^2)^+).
    Each a_k may be a number or a field of the grid's shape (the spatialised
    parameters a(x) of Sec. 5.2); the c_k are then fields too.
    """
    a20, a11, a02, a10, a01, a00 = (np.asarray(v, dtype=np.float64) for v in a)
    return ((a20 + a02 - a11) / (2.0 * eps),
            a11 / (2.0 * eps),
            (a20 - a02) / (2.0 * eps),
            (a10 + a01) / 2.0,
            (a10 - a01) / 2.0,
            a00)


# --------------------------------------------------------------------------
# Smoothed positive part, Sec. 4.1: x^+ ~ xi log(1 + exp(x / xi))
# --------------------------------------------------------------------------

def softplus(x, xi=XI):
    """xi log(1 + exp(x/xi)), evaluated as max(x,0) + xi log1p(exp(-|x|/xi))."""
    return np.maximum(x, 0.0) + xi * np.log1p(np.exp(-np.abs(x) / xi))


def logistic(z):
    """1 / (1 + exp(-z)) without overflow; the derivative of softplus in x/xi."""
    e = np.exp(-np.abs(z))
    return np.where(z >= 0, 1.0 / (1.0 + e), e / (1.0 + e))


def positive_part(x, xi=XI, mode="smooth"):
    """(value, derivative) of the positive part: smoothed (Sec. 4.1) or exact max(x, 0)."""
    if mode == "smooth":
        return softplus(x, xi), logistic(x / xi)
    if mode == "hard":
        return np.maximum(x, 0.0), (x > 0).astype(np.float64)
    raise ValueError("mode must be 'smooth' or 'hard'")


# --------------------------------------------------------------------------
# Forward: pointwise fields and the energy
# --------------------------------------------------------------------------

def pointwise(u, h, eps, a, xi=XI, mode="smooth", orient=None):
    """All per-voxel quantities of eq. (Meps) and eq. (Feps) on the grid.

    Returns a dict with the stencil values g (3), H (6), the matrix M (6, same
    order as H), T = Tr M, N2 = ||M||_F^2, X = 2 N2 - T^2, S = sqrt(X^+ smoothed),
    rho = sqrt(q + xi^2), q = |g|^2, the term fields and the density f.

    orient = (mu, theta) adds the orientation term of Sec. 5.2,
    eps mu (theta . grad u)^2, as a seventh term (theta as given, (x, y, z)).
    """
    u = np.asarray(u, dtype=np.float64)
    c1, c2, c3, c4, c5, c6 = feps_coefficients(a, eps)
    g = fd_gradient(u, h)
    H = fd_hessian(u, h)
    q = g[0] ** 2 + g[1] ** 2 + g[2] ** 2
    r = q + xi * xi
    rho = np.sqrt(r)
    # n (x) n with the offset: g g^T / (|g|^2 + xi^2)
    s = double_well_prime(u) / (eps * r)
    M = [-eps * H[a_] + s * g[a_] * g[a_] for a_ in range(3)]
    for k, (a_, b_) in enumerate(_PAIRS):
        M.append(-eps * H[3 + k] + s * g[a_] * g[b_])
    T = M[0] + M[1] + M[2]
    N2 = M[0] ** 2 + M[1] ** 2 + M[2] ** 2 + 2.0 * (M[3] ** 2 + M[4] ** 2 + M[5] ** 2)
    X = 2.0 * N2 - T * T
    P, dP = positive_part(X, xi, mode)
    S = np.sqrt(P)
    terms = (c1 * N2, c2 * T * T, c3 * T * S, c4 * rho * T, c5 * rho * S, c6 * eps * q)
    f = terms[0] + terms[1] + terms[2] + terms[3] + terms[4] + terms[5]
    tg = None
    if orient is not None:
        mu, th = orient
        tg = th[0] * g[0] + th[1] * g[1] + th[2] * g[2]          # theta . grad u
        terms = terms + (eps * mu * tg * tg,)
        f = f + terms[6]
    return dict(g=g, H=H, M=M, T=T, N2=N2, X=X, P=P, dP=dP, S=S, q=q, r=r, rho=rho,
                s=s, terms=terms, f=f, coeffs=(c1, c2, c3, c4, c5, c6), tg=tg)


def energy(u, h, eps, a, xi=XI, mode="smooth", orient=None):
    """F_h(u) = h^3 sum_i f_i: eq. (Feps) with the integral as a finite sum (Sec. 4.1)."""
    return float(h ** 3 * np.sum(pointwise(u, h, eps, a, xi, mode, orient)["f"]))


def energy_abs(u, h, eps, a, xi=XI, mode="smooth", orient=None):
    """h^3 sum_i sum_k |term_k|: the scale used for relative energy errors when F ~ 0."""
    t = pointwise(u, h, eps, a, xi, mode, orient)["terms"]
    return float(h ** 3 * sum(np.sum(np.abs(x)) for x in t))


# --------------------------------------------------------------------------
# Adjoint: exact gradient of F_h with respect to every voxel value
# --------------------------------------------------------------------------

def adjoint_fields(u, h, eps, a, xi=XI, mode="smooth", orient=None):
    """Per-voxel partial derivatives of f with respect to its stencil inputs.

    Returns (ubar, gamma[3], theta[6], fwd): ubar = df/du at the voxel itself
    (through W'), gamma_a = df/dg_a, theta_k = df/dH_k (k in xx, yy, zz, xy,
    xz, yz), computed by reverse-mode differentiation of the forward chain in
    `pointwise`.
    """
    fw = pointwise(u, h, eps, a, xi, mode, orient)
    c1, c2, c3, c4, c5, c6 = fw["coeffs"]
    g, M, T, S, rho, r, s = fw["g"], fw["M"], fw["T"], fw["S"], fw["rho"], fw["r"], fw["s"]
    u = np.asarray(u, dtype=np.float64)

    # f = c1 N2 + c2 T^2 + c3 T S + c4 rho T + c5 rho S + c6 eps q
    S_bar = c3 * T + c5 * rho
    T_bar = 2.0 * c2 * T + c3 * S + c4 * rho
    rho_bar = c4 * T + c5 * S
    N2_bar = np.full_like(T, c1)
    # S = sqrt(P(X)), X = 2 N2 - T^2; dS/dX := 0 where S == 0
    with np.errstate(divide="ignore", invalid="ignore"):
        dS_dX = np.where(S > 0, fw["dP"] / (2.0 * np.where(S > 0, S, 1.0)), 0.0)
    X_bar = S_bar * dS_dX
    N2_bar = N2_bar + 2.0 * X_bar
    T_bar = T_bar - 2.0 * T * X_bar
    # N2 = sum_a M_aa^2 + 2 sum_{a<b} M_ab^2, T = sum_a M_aa
    M_bar = [2.0 * N2_bar * M[k] + T_bar for k in range(3)]
    M_bar += [4.0 * N2_bar * M[k] for k in range(3, 6)]
    # M_ab = -eps H_ab + s g_a g_b
    theta = [-eps * mb for mb in M_bar]
    s_bar = (M_bar[0] * g[0] * g[0] + M_bar[1] * g[1] * g[1] + M_bar[2] * g[2] * g[2]
             + M_bar[3] * g[0] * g[1] + M_bar[4] * g[0] * g[2] + M_bar[5] * g[1] * g[2])
    # s = W'(u) / (eps r), r = q + xi^2, rho = sqrt(r), q = |g|^2
    q_bar = -s_bar * s / r + rho_bar / (2.0 * rho) + c6 * eps
    ubar = s_bar * (3.0 * u * u - 1.0) / (eps * r)
    gamma = [
        s * (2.0 * M_bar[0] * g[0] + M_bar[3] * g[1] + M_bar[4] * g[2]) + 2.0 * g[0] * q_bar,
        s * (2.0 * M_bar[1] * g[1] + M_bar[3] * g[0] + M_bar[5] * g[2]) + 2.0 * g[1] * q_bar,
        s * (2.0 * M_bar[2] * g[2] + M_bar[4] * g[0] + M_bar[5] * g[1]) + 2.0 * g[2] * q_bar,
    ]
    if orient is not None:
        # d/dg_a of eps mu (theta . g)^2
        mu, th = orient
        gamma = [gamma[a_] + 2.0 * eps * mu * fw["tg"] * th[a_] for a_ in range(3)]
    return ubar, gamma, theta, fw


def energy_grad(u, h, eps, a, xi=XI, mode="smooth", orient=None):
    """(F_h, dF_h/du): energy and its exact gradient, h^3 included.

    The gradient applies the transposes of the stencils to the per-voxel adjoint
    fields: the central difference is anti-self-adjoint on a periodic grid and
    the second and mixed differences are self-adjoint.
    """
    ubar, gamma, theta, fw = adjoint_fields(u, h, eps, a, xi, mode, orient)
    E = float(h ** 3 * np.sum(fw["f"]))
    return E, h ** 3 * transpose_stencils(ubar, gamma, theta, h)


def transpose_stencils(ubar, gamma, theta, h):
    """sum over the stencils' transposes of the per-voxel adjoints: the derivative of
    sum_i f_i with respect to every sample, given df_i/du_i (ubar), df_i/dg_a (gamma)
    and df_i/dH_k (theta) at every voxel i of a periodic grid."""
    grad = ubar.copy()
    for a_ in range(3):
        # transpose of the central difference
        grad -= (_at(gamma[a_], _unit(a_)) - _at(gamma[a_], _unit(a_, -1))) / (2.0 * h)
        # transpose of the second difference (self-adjoint)
        grad += (_at(theta[a_], _unit(a_)) - 2.0 * theta[a_]
                 + _at(theta[a_], _unit(a_, -1))) / (h * h)
    for k, (a_, b_) in enumerate(_PAIRS):
        th = theta[3 + k]
        grad += (_at(th, _pair(a_, 1, b_, 1)) - _at(th, _pair(a_, 1, b_, -1))
                 - _at(th, _pair(a_, -1, b_, 1)) + _at(th, _pair(a_, -1, b_, -1))) / (4.0 * h * h)
    return grad


# --------------------------------------------------------------------------
# Mass-preserving descent (Sec. 4.1: the flow keeps the mean of u fixed)
# --------------------------------------------------------------------------

def mass_projected_step(u, h, eps, a, m, tau, xi=XI, mode="smooth", orient=None):
    """One step u <- P_m(u - tau dF_h/du), P_m(v) = v + (m - mean(v)).

    P_m is the L2-orthogonal projection onto {mean(u) = m}. Returns
    (u_new, F_h(u)), the energy being that of the field before the step.
    """
    E, grad = energy_grad(u, h, eps, a, xi, mode, orient)
    v = np.asarray(u, dtype=np.float64) - tau * grad
    return v + (m - np.mean(v)), E


def descend(u, h, eps, a, m, tau, nsteps, xi=XI, mode="smooth", orient=None):
    """nsteps mass-projected steps; returns (u_final, [F_h before each step])."""
    energies = []
    u = np.asarray(u, dtype=np.float64)
    for _ in range(nsteps):
        u, E = mass_projected_step(u, h, eps, a, m, tau, xi, mode, orient)
        energies.append(E)
    return u, energies


def adam_projected_step(u, m1, m2, t, h, eps, a, m, lr=1e-3, beta1=0.9, beta2=0.999, adam_eps=1e-8,
                        xi=XI, mode="smooth"):
    """One mass-preserving step with Adam, the optimiser of Sec. 4.1 (learning rate,
    betas and no weight decay as stated there; adam_eps is not stated, 1e-8 is read).

    Adam (Kingma & Ba) on the voxel values with step number t >= 1:
    m1 <- beta1 m1 + (1-beta1) g, m2 <- beta2 m2 + (1-beta2) g^2,
    v = u - lr (m1/(1-beta1^t)) / (sqrt(m2/(1-beta2^t)) + adam_eps), then the L2
    projection onto {mean = m}. Returns (u_new, m1, m2, F_h(u)).
    """
    E, grad = energy_grad(u, h, eps, a, xi, mode)
    m1 = beta1 * m1 + (1.0 - beta1) * grad
    m2 = beta2 * m2 + (1.0 - beta2) * grad * grad
    mhat = m1 / (1.0 - beta1 ** t)
    vhat = m2 / (1.0 - beta2 ** t)
    v = np.asarray(u, dtype=np.float64) - lr * mhat / (np.sqrt(vhat) + adam_eps)
    return v + (m - np.mean(v)), m1, m2, E


def descend_adam(u, h, eps, a, m, nsteps, lr=1e-3, beta1=0.9, beta2=0.999, adam_eps=1e-8, xi=XI,
                 mode="smooth"):
    """nsteps Adam steps from zero moments; returns (u_final, [F_h before each step])."""
    u = np.asarray(u, dtype=np.float64)
    m1 = np.zeros_like(u)
    m2 = np.zeros_like(u)
    energies = []
    for t in range(1, nsteps + 1):
        u, m1, m2, E = adam_projected_step(u, m1, m2, t, h, eps, a, m, lr, beta1, beta2, adam_eps, xi, mode)
        energies.append(E)
    return u, energies


# --------------------------------------------------------------------------
# Batched helpers (independent instances, each with its own eps, a, m)
# --------------------------------------------------------------------------

def energy_grad_batch(U, h, eps_list, a_list, xi=XI, mode="smooth"):
    """Per-instance (energies[B], grads[B, ...]) for a stack of independent fields."""
    Es, Gs = [], []
    for b in range(U.shape[0]):
        E, G = energy_grad(U[b], h, eps_list[b], a_list[b], xi, mode)
        Es.append(E)
        Gs.append(G)
    return np.array(Es), np.stack(Gs)


# --------------------------------------------------------------------------
# Algorithm 1 (Sec. 4.1): the H^-1 flow through u = div A + m0, a small
# Gaussian blur, and Adam on the vector field A
# --------------------------------------------------------------------------

def fd_divergence(A, h):
    """div A = sum_a (A_a(i + e_a) - A_a(i - e_a)) / (2h), periodic; A is [3, nz, ny, nx]
    with components (x, y, z) (the same central differences as the gradient)."""
    return sum((_at(A[a_], _unit(a_)) - _at(A[a_], _unit(a_, -1))) / (2.0 * h) for a_ in range(3))


def gaussian_weights(sigma_k):
    """Normalised taps w_j, |j| <= ceil(4 sigma_k), of the sampled Gaussian exp(-j^2 / (2 sigma_k^2));
    sigma_k = 0 gives the identity [1]."""
    if sigma_k <= 0:
        return np.array([1.0])
    r = int(np.ceil(4.0 * sigma_k))
    j = np.arange(-r, r + 1, dtype=np.float64)
    w = np.exp(-j * j / (2.0 * sigma_k * sigma_k))
    return w / w.sum()


def gaussian_blur(u, sigma_k):
    """Separable periodic convolution of u [nz, ny, nx] with the sampled Gaussian along
    x, then y, then z. The kernel is even, so the blur is its own adjoint."""
    w = gaussian_weights(sigma_k)
    r = (len(w) - 1) // 2
    out = np.asarray(u, dtype=np.float64)
    for a_ in range(3):
        acc = np.zeros_like(out)
        for k, wk in enumerate(w):
            acc += wk * _at(out, _unit(a_, k - r))
        out = acc
    return out


def hminus_energy(A, h, eps, a, m0, sigma_k, xi=XI, mode="smooth", orient=None):
    """G_eps(A) = F_h(k * (div A + m0)) (Algorithm 1, with the blur before the energy).
    m0 may be a field m(x) (Sec. 5.2), a may hold fields a(x)."""
    return energy(gaussian_blur(fd_divergence(A, h) + m0, sigma_k), h, eps, a, xi, mode, orient)


def hminus_energy_grad(A, h, eps, a, m0, sigma_k, xi=XI, mode="smooth", orient=None):
    """(G_eps(A), dG/dA, u) with u = k * (div A + m0): the chain rule of Algorithm 1.

    dG/du_b = dF_h/du (at the blurred field), dG/du = k * dG/du_b (even kernel),
    dG/dA_a = -(dG/du(i + e_a) - dG/du(i - e_a)) / (2h) (the central difference is
    anti-self-adjoint on a periodic grid), i.e. dG/dA = -grad dF/du of Sec. 4.1.
    """
    u = gaussian_blur(fd_divergence(A, h) + m0, sigma_k)
    E, gb = energy_grad(u, h, eps, a, xi, mode, orient)
    gu = gaussian_blur(gb, sigma_k)
    gA = np.stack([-(_at(gu, _unit(a_)) - _at(gu, _unit(a_, -1))) / (2.0 * h) for a_ in range(3)])
    return E, gA, u


def hminus_adam_step(A, m1, m2, t, h, eps, a, m0, sigma_k, lr=1e-3, beta1=0.9, beta2=0.999, adam_eps=1e-8,
                     xi=XI, mode="smooth", orient=None):
    """One iteration of Algorithm 1: G and dG/dA at A, then Adam on A (step number t >= 1).
    Returns (A_new, m1, m2, G(A), u) with u the blurred phase field at A."""
    E, gA, u = hminus_energy_grad(A, h, eps, a, m0, sigma_k, xi, mode, orient)
    m1 = beta1 * m1 + (1.0 - beta1) * gA
    m2 = beta2 * m2 + (1.0 - beta2) * gA * gA
    mhat = m1 / (1.0 - beta1 ** t)
    vhat = m2 / (1.0 - beta2 ** t)
    A_new = np.asarray(A, dtype=np.float64) - lr * mhat / (np.sqrt(vhat) + adam_eps)
    return A_new, m1, m2, E, u


def hminus_descend(A, h, eps, a, m0, sigma_k, nsteps, lr=1e-3, beta1=0.9, beta2=0.999, adam_eps=1e-8,
                   xi=XI, mode="smooth", orient=None):
    """nsteps iterations of Algorithm 1 from zero moments. Returns (A, [G before each step], u_final)
    with u_final = k * (div A + m0) at the final A."""
    A = np.asarray(A, dtype=np.float64)
    m1 = np.zeros_like(A)
    m2 = np.zeros_like(A)
    energies = []
    for t in range(1, nsteps + 1):
        A, m1, m2, E, _ = hminus_adam_step(A, m1, m2, t, h, eps, a, m0, sigma_k, lr, beta1, beta2, adam_eps,
                                           xi, mode, orient)
        energies.append(E)
    return A, energies, gaussian_blur(fd_divergence(A, h) + m0, sigma_k)
