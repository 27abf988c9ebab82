/*
 * fe.h - C ABI of the MI355X (gfx950) curvature phase-field energy library.
 *
 * The library evaluates the discrete phase-field energy F_eps of eq. (Feps)
 * (Sec. 3.2), its exact gradient with respect to the phase field u, and a
 * mass-preserving descent step, on periodic 3-D voxel grids, for one or many
 * independent instances at once.
 *
 * Discrete problem (Sec. 4.1, Implementation details). For each instance b
 * with field u on an nz x ny x nx periodic grid of spacing h:
 *
 *   M  = -eps Hess_h u + (W'(u)/eps) g g^T / (|g|^2 + xi^2),  W'(s) = s^3 - s
 *   F_h(u) = h^3 sum_voxels [ c1 ||M||^2 + c2 (Tr M)^2 + c3 Tr M S
 *                             + c4 rho Tr M + c5 rho S + c6 eps |g|^2 ]
 *
 * with g = central-difference gradient, Hess_h = compact 19-point periodic
 * Hessian, rho = sqrt(|g|^2 + xi^2), S = sqrt(softplus_xi(2||M||^2 - (Tr M)^2)),
 * softplus_xi(x) = xi log(1 + exp(x/xi)), xi = 1e-6, and
 *   c1 = (a20 + a02 - a11)/(2 eps), c2 = a11/(2 eps), c3 = (a20 - a02)/(2 eps),
 *   c4 = (a10 + a01)/2, c5 = (a10 - a01)/2, c6 = a00
 * for the polynomial p(k1,k2) = a20 k1^2 + a11 k1 k2 + a02 k2^2 + a10 k1
 * + a01 k2 + a00 of eq. (F) (Sec. 2.1).
 *
 * Layout: every field is a dense, contiguous device array [batch][nz][ny][nx]
 * (x fastest) of float (FE_F32) or double (FE_F64), on the device that was
 * current when the context was created. Field pointers are owned by the
 * caller; the library never frees or reallocates them.
 *
 * Errors: every int-returning call returns FE_OK (0) on success and a
 * negative FE_E* code otherwise; fe_last_error() then describes the failure.
 * No C++ exception crosses this interface. Calls are ordered on the
 * context's stream; only calls that return values into host memory
 * synchronise that stream. One context must not be used from two host
 * threads at the same time.
 */
#ifndef FE_H_
#define FE_H_

#ifdef __cplusplus
extern "C" {
#endif

enum fe_dtype { FE_F32 = 0, FE_F64 = 1 };

enum fe_status {
  FE_OK = 0,
  FE_EINVAL = -1,     /* invalid argument: sizes, NULL pointers, eps <= 0, non-finite values */
  FE_EHIP = -2,       /* a HIP runtime call or kernel launch failed */
  FE_ENOMEM = -3,     /* device or host allocation failed */
  FE_ENONFINITE = -4  /* an energy came out NaN/Inf; outputs were still written */
};

typedef struct fe_grid {
  int nx, ny, nz;   /* samples per axis, each >= 1 */
  int batch;        /* number of independent instances, >= 1 */
  double h;         /* grid spacing (same on every axis), > 0 */
  int dtype;        /* FE_F32 or FE_F64: element type of every field */
} fe_grid;

typedef struct fe_ctx fe_ctx;   /* opaque: parameters, reduction workspace, step buffers, graphs */

/*
 * Create a context for `grid`.
 *   eps      host [batch]: interface width eps_b > 0 of each instance (eq. (Meps)).
 *   p_coeffs host [batch][6]: (a20, a11, a02, a10, a01, a00) of each instance,
 *            the coefficient order of Sec. 3.2; all finite.
 *   stream   hipStream_t to order work on, or NULL for the default stream.
 *   out      receives the new context.
 * Allocates only small device workspaces (O(batch x blocks) doubles); the
 * ping-pong buffer of fe_step is allocated on its first call.
 * Limits: a plane (nx * ny samples) of at most 4 GiB - 64 KiB, the kernels
 * addressing it with 32-bit byte offsets; at most 4e9 samples in all.
 * Returns FE_EINVAL, FE_ENOMEM or FE_EHIP on failure (*out is then NULL).
 */
int fe_create(const fe_grid* grid, const double* eps, const double* p_coeffs,
              void* stream, fe_ctx** out);

/* Replace eps [batch] and p_coeffs [batch][6] (same meaning as fe_create). No allocation. */
int fe_set_params(fe_ctx* ctx, const double* eps, const double* p_coeffs);

/* Order subsequent work on `stream` (hipStream_t, NULL = default stream). */
int fe_set_stream(fe_ctx* ctx, void* stream);

/*
 * Energy only: energy[b] = F_h(u_b) in double.
 *   u       device field [batch][nz][ny][nx], read only.
 *   energy  host [batch], or NULL. Non-NULL synchronises the stream.
 * FE_ENONFINITE if an energy is NaN/Inf (energy[] is still written).
 */
int fe_energy(fe_ctx* ctx, const void* u, double* energy);

/*
 * Energy and gradient: g = dF_h/du, the exact derivative of the h^3-weighted
 * finite sum (the h^3 factor is included), and energy[b] = F_h(u_b).
 *   u       device field, read only.
 *   g       device field, written; must not overlap u.
 *   energy  host [batch] or NULL (non-NULL synchronises the stream).
 */
int fe_energy_grad(fe_ctx* ctx, const void* u, void* g, double* energy);

/*
 * As fe_energy / fe_energy_grad, but the energies go to device memory and
 * nothing synchronises: energy_dev is a device array of `batch` doubles, or NULL.
 * g may be NULL to compute the energy only.
 */
int fe_energy_grad_async(fe_ctx* ctx, const void* u, void* g, double* energy_dev);

/*
 * The gradient alone, scaled per instance: g_b = s_b dF_h/du_b, the backward of
 * an energy whose incoming derivative is s (the chain rule through eq. (Feps)).
 * The density is linear in its coefficients, so the sweep runs with every
 * coefficient of instance b multiplied by s_b (with a coefficient field, the
 * gradient is scaled after the sweep). No energy is formed; stream-ordered,
 * nothing synchronises, nothing is allocated.
 *   u       device field [batch][nz][ny][nx], read only.
 *   g       device field, written; must not overlap u.
 *   gscale  device array of `batch` doubles (s), read in stream order.
 * Equal to s_b times fe_energy_grad's g up to rounding, not bitwise.
 */
int fe_grad_scaled_async(fe_ctx* ctx, const void* u, void* g, const double* gscale);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): fe_energy_grad_async
 * without a context. It allocates nothing and calls nothing that allocates;
 * its per-instance table and block partials live in one static 1 MiB device
 * array that each device holds until the process ends.
 *   grid, eps, p_coeffs  as in fe_create (host memory, read during the call);
 *                        batch <= 16.
 *   u           device field [batch][nz][ny][nx] on the current device, read only.
 *   g           device field, written with dF_h/du (must not overlap u), or NULL.
 *   energy_dev  device array of `batch` doubles receiving F_h(u_b), or NULL
 *               (not both NULL).
 *   stream      hipStream_t the work is ordered on (NULL: default stream).
 * Nothing synchronises; the launch shape is the one a fresh context would
 * choose. FE_EINVAL for a batch above 16, invalid parameters, or a grid whose
 * sweep needs more block partials than the array holds (65280; 256^3 needs 512).
 * Every call on a device shares that device's array (the last call's contents
 * stay there; every value a call reads it has written first in stream order),
 * so calls that overlap on one device - on two streams, or from two host
 * threads - race and must be serialised by the caller.
 */
int fe_energy_grad_noalloc(const fe_grid* grid, const double* eps, const double* p_coeffs, const void* u,
                           void* g, double* energy_dev, void* stream);

/*
 * nsteps mass-preserving descent steps, in place on u (Sec. 4.1 keeps the mean
 * of u fixed along the flow):
 *   u <- v + (mass[b] - mean(v)),  v = u - tau dF_h/du,
 * i.e. a gradient step followed by the L2 projection onto {mean(u_b) = mass[b]}.
 * The first step also moves an initial mean that differs from mass[b] onto it.
 *   u       device field, read and overwritten with the result.
 *   mass    host [batch]: target mean of each instance.
 *   tau     step size (> 0, finite).
 *   nsteps  number of steps, >= 0 (0 is a no-op).
 *   energy  host [batch] or NULL: F_h of the field before the last step
 *           (synchronises the stream when non-NULL).
 * Uses a context-owned ping-pong field of the same size as u (allocated on
 * first use) and replays captured HIP graphs for the step loop.
 */
int fe_step(fe_ctx* ctx, void* u, const double* mass, double tau, int nsteps, double* energy);

/*
 * nsteps mass-preserving steps with the optimiser the paper runs its flows
 * with (Adam, Sec. 4.1: learning rate 1e-3, betas (0.9, 0.999), no weight
 * decay), in place on u:
 *   g = dF_h/du,  m1 <- beta1 m1 + (1 - beta1) g,  m2 <- beta2 m2 + (1 - beta2) g^2,
 *   v = u - lr (m1 / (1 - beta1^t)) / (sqrt(m2 / (1 - beta2^t)) + adam_eps),
 *   u <- v + (mass[b] - mean(v)),  t <- t + 1,
 * per voxel, with the moments m1, m2 and the step number t (starting at 1)
 * kept in the context from one call to the next (fe_adam_reset clears them).
 * The per-voxel normalisation bounds every move by about lr, which keeps the
 * descent stable where dF_h/du spikes near umbilic voxels (it grows like
 * 1/sqrt(2||M||^2 - (Tr M)^2) there when a20 != a02 or a10 != a01).
 *   u, mass, nsteps, energy  as for fe_step.
 *   lr > 0, 0 <= beta1, beta2 < 1, adam_eps > 0, all finite, else FE_EINVAL.
 * Allocates the two moment fields (each the size of u) on first use.
 */
int fe_step_adam(fe_ctx* ctx, void* u, const double* mass, double lr, double beta1, double beta2,
                 double adam_eps, int nsteps, double* energy);

/* Zero the Adam moments and reset the step number to 1. Stream-ordered, no allocation. */
int fe_adam_reset(fe_ctx* ctx);

/*
 * Space-dependent coefficients a(x) of Sec. 5.2. Every later energy, gradient,
 * step, flow and diagnostics call evaluates the density at voxel i with the
 * coefficients a(x_i) instead of the instance's p_coeffs (eps stays per
 * instance).
 *   a_field  device [batch][6][nz][ny][nx] in the context's precision, the six
 *            coefficients in the order (a20, a11, a02, a10, a01, a00); the
 *            library keeps its own scaled copy (one record of six values per
 *            voxel, allocated on first use). NULL returns to the per-instance
 *            coefficients.
 * fe_set_params drops an installed field (its scaling depends on eps); set it
 * again afterwards. Synchronises the stream. FE_EINVAL when nx * ny * 6
 * samples exceed 4 GiB - 64 KiB (the sweeps address a plane of records with
 * 32-bit offsets).
 */
int fe_set_coeff_field(fe_ctx* ctx, const void* a_field);

/*
 * Space-dependent mass m(x) of Sec. 5.2 for fe_hminus_step: u = div A + m(x)
 * replaces u = div A + m0, and m0 may then be NULL (it is ignored).
 *   m_field  device [batch][nz][ny][nx] in the context's precision (copied);
 *            NULL returns to the per-instance m0.
 * The mean of u is then the mean of m(x). The step entry points are not
 * affected (their constraint is the mean).
 */
int fe_set_mass_field(fe_ctx* ctx, const void* m_field);

/*
 * The orientation term of Sec. 5.2: every later energy, gradient, step, flow
 * and diagnostics call adds eps mu (theta . grad u)^2 to the density (with
 * grad u the central differences), i.e. h^3 eps mu sum_i (theta . g_i)^2 to F_h.
 *   mu     host [batch]; 0 switches the term off for that instance (the default).
 *   theta  host [batch][3] (x, y, z), used as given (the paper takes a unit vector).
 * All values must be finite. Does not reallocate; synchronises the stream.
 */
int fe_set_orientation(fe_ctx* ctx, const double* mu, const double* theta);

/*
 * nsteps iterations of the paper's generation algorithm (Algorithm 1, Sec. 4.1):
 * the mass-preserving H^-1 flow written as an L2 flow on a periodic vector
 * field A through u = div A + m0, with a small Gaussian blur before the energy
 * and Adam on A:
 *   u = k * (div A + m0),  G(A) = F_h(u),
 *   dG/dA = -grad (k * dF_h/du)   (div and grad are the periodic central
 *                                   differences; the kernel k is even),
 *   A <- A - lr mhat / (sqrt(vhat) + adam_eps)   (Adam, moments kept in the
 *                                                  context; fe_hminus_reset clears them).
 * mean(u) = m0 holds exactly, since div A has zero mean and k sums to 1.
 *   A        device [batch][3][nz][ny][nx] (components x, y, z), updated in place.
 *   m0       host [batch]: the mass (target mean) of each instance; ignored,
 *            and may be NULL, while a mass field is set (fe_set_mass_field).
 *   sigma_k  blur standard deviation in voxels, 0 <= sigma_k <= 4 (0: no blur);
 *            taps exp(-j^2 / (2 sigma_k^2)), |j| <= ceil(4 sigma_k), normalised.
 *   lr, beta1, beta2, adam_eps  Adam settings (the paper: 1e-3, 0.9, 0.999).
 *   u_out    device field [batch][nz][ny][nx] or NULL: receives k * (div A + m0)
 *            at the final A (the field whose zero level set is the texture).
 *   energy   host [batch] or NULL: G before the last update (synchronises).
 * Requires nz * batch <= 65535, planes (nx * ny samples) under 4 GiB and
 * nz * nx < 2^31 (FE_EINVAL otherwise). Allocates two work fields and
 * the six moment fields of A on first use; replays captured graphs.
 */
int fe_hminus_step(fe_ctx* ctx, void* A, const double* m0, double sigma_k, double lr, double beta1,
                   double beta2, double adam_eps, int nsteps, void* u_out, double* energy);

/* Zero the Adam moments of A and reset their step number to 1. No allocation. */
int fe_hminus_reset(fe_ctx* ctx);

/*
 * Texture diagnostics of u in one sweep over the energy's stencils.
 *   curv   device [batch][4][nz][ny][nx] in the context's precision, or NULL:
 *          the diffuse mean curvature H, Gaussian curvature K and principal
 *          curvatures kappa1 >= kappa2 of eqs. (Heps), (Keps), (kepsa),
 *          (kepsb) (Sec. 3.1), with |grad u| regularised as sqrt(|g|^2 + xi^2).
 *   hist   device double [batch][nbins][nbins], or NULL: histogram of
 *          (kappa1, kappa2), indexed [bin of kappa1][bin of kappa2], each voxel
 *          weighted by h^3 eps |grad u|^2 (the density that concentrates on
 *          the diffuse interface); curvatures are clamped to [-kmax, kmax] and
 *          binned uniformly, bin = min(floor((k + kmax) nbins / (2 kmax)),
 *          nbins - 1), in the context's precision. A mesh-free stand-in for the
 *          curvature diagram of Sec. 4.1. The call zeroes it first. Bins are
 *          summed with floating-point atomics, so their last bits may vary
 *          between calls. 1 <= nbins <= 64, kmax > 0.
 *   stats  host double [batch][5], or NULL: F_h, the Cahn-Hilliard area
 *          A_eps of eq. (CH_eps), the discrepancy of Sec. 4.5 normalised by
 *          A_eps, min u and max u (bitwise deterministic; synchronises).
 */
int fe_diagnostics(fe_ctx* ctx, const void* u, void* curv, double* hist, int nbins, double kmax, double* stats);

/*
 * Algorithm 2 (Sec. 4.2): the L2 flow of F_h(k * u) with replicate boundary
 * conditions, driven by L-BFGS, on one field (the validation flow of the
 * paper's Willmore experiments). The box field [nz][ny][nx] is held inside a
 * padded copy whose padding repeats the nearest box voxel wherever a stencil
 * or the blur reads outside the box; F_h sums the density over the box only,
 * and derivatives that land on padding are added back onto the voxels it
 * copies, so the gradient is exact for that finite sum.
 *
 * L-BFGS (Nocedal and Wright's two-loop recursion, H0 = s'y / y'y, no line
 * search): each step runs up to max_iter inner iterations of fixed length lr
 * (the very first one scaled by min(1, 1/|g|_1)), keeps the last `history`
 * pairs (s, y) with s'y > 1e-10, and stops early on max|g| <= tolerance_grad,
 * g'd > -tolerance_change, max|lr d| <= tolerance_change, a loss change below
 * tolerance_change, or after max_iter * 5 / 4 evaluations. Defaults: lr 1,
 * history 10, max_iter 20 (Sec. 4.2), tolerances 1e-7 and 1e-9.
 */
typedef struct fe_l2 fe_l2;

/* grid: the box (batch must be 1); eps, p_coeffs[6] as in fe_create; blur
 * 0 <= sigma_k <= 4 voxels (0: none). The box padded by max(1, ceil(4 sigma_k))
 * on every side must have ny, nz <= 65535, planes under 4 GiB and
 * nz * nx < 2^31 (FE_EINVAL otherwise). Allocates the padded fields and the
 * optimiser's history on the device. */
int fe_l2_create(const fe_grid* grid, double eps, const double* p_coeffs, double sigma_k, void* stream,
                 fe_l2** out);
/* Optimiser settings (1 <= history <= 64, max_iter >= 1); resets its state. */
int fe_l2_set_lbfgs(fe_l2* flow, double lr, int history, int max_iter, double tolerance_grad,
                    double tolerance_change);
/* Copy the box field u (device, [nz][ny][nx], the grid's precision) in as the
 * variable, and reset the optimiser's state. */
int fe_l2_load(fe_l2* flow, const void* u);
/* Copy the variable out to the box field u (device). */
int fe_l2_store(fe_l2* flow, void* u);
/* Load u, then F_h(k * u) into *energy (host) and its gradient into g (device
 * box field, or NULL). Synchronises. */
int fe_l2_energy_grad(fe_l2* flow, const void* u, void* g, double* energy);
/* nsteps optimiser steps from the current variable and state; energies (host
 * [nsteps] or NULL) receives the loss at the start of each step. */
int fe_l2_step(fe_l2* flow, int nsteps, double* energies);
int fe_l2_set_stream(fe_l2* flow, void* stream);
void fe_l2_destroy(fe_l2* flow);

/*
 * Launch-shape selection. Variants are numbered 0 .. fe_num_variants()-1;
 * fe_variant_info describes one (x and y interior tile, threads per block,
 * element size it supports). fe_set_launch picks a variant and a z-chunk
 * length (planes per block, >= 1; 0 = automatic). FE_EINVAL for a variant
 * that does not support the context's dtype. A new context starts on the
 * leading variant of its dtype whose tiles evaluate the fewest ring voxels on
 * its x-y plane. Its automatic z chunks are the equal chunks whose blocks,
 * dealt out over the compute units, finish first.
 */
int fe_num_variants(void);
int fe_variant_info(int variant, int* tile_x, int* tile_y, int* threads, int* dtype_mask);
int fe_set_launch(fe_ctx* ctx, int variant, int z_chunk);
int fe_get_launch(const fe_ctx* ctx, int* variant, int* z_chunk);

/* What fe_autotune times: the sweep that fe_energy_grad, fe_step or fe_step_adam runs. */
enum fe_tune_kind { FE_TUNE_GRAD = 0, FE_TUNE_STEP = 1, FE_TUNE_ADAM = 2 };

/*
 * Pick the launch shape (variant and z-chunk length) for the sweep that `kind`
 * names, and keep it in the context. The choice depends on the grid, batch,
 * dtype, kind, on whether the instances' p are symmetric in k1, k2 (which
 * per-voxel body the sweep holds), on a coefficient field or box mask, and on
 * the device architecture; a choice made earlier in this process for the same
 * key, or loaded by fe_tune_cache_load, is taken without timing (*cached = 1).
 * Otherwise the workload first runs 50 ms untimed (the clocks settle), then
 * every variant that supports the dtype is timed at a few z-chunk lengths,
 * `iters` launches each, and the fastest is kept and cached.
 *   u        device field, read only.
 *   work     device field of u's size, distinct from u, overwritten (the step
 *            kinds run on a copy of u there and in the context's step buffer).
 *   kind     FE_TUNE_GRAD, FE_TUNE_STEP or FE_TUNE_ADAM (not for a box mask).
 *   iters    launches per candidate, >= 1.
 *   best_us  host, may be NULL: time per launch of the choice, in microseconds.
 *   cached   host, may be NULL: 1 if the choice came from the cache, else 0.
 * FE_TUNE_ADAM times on temporary moments: the context's Adam state is kept.
 * Synchronises the stream. FE_EINVAL on bad arguments.
 */
int fe_autotune(fe_ctx* ctx, const void* u, void* work, int kind, int iters, double* best_us, int* cached);

/*
 * The autotuner's cache, shared by every context of the process: save it to a
 * text file (one "key variant z_chunk us" line per entry), merge a saved file
 * into it (FE_EINVAL, and nothing merged, if a line is malformed or names a
 * variant this library does not have), or empty it.
 */
int fe_tune_cache_save(const char* path);
int fe_tune_cache_load(const char* path);
void fe_tune_cache_clear(void);

/* Release the context and everything it allocated. NULL is a no-op. */
void fe_destroy(fe_ctx* ctx);

/* Text of the last error raised on this host thread ("" if none). */
const char* fe_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FE_H_ */
