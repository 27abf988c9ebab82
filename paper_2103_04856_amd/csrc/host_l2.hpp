// Host side of Algorithm 2 (the L2 flow with replicate boundaries, driven by
// L-BFGS) and its entry points. Included once by fe_api.hip.
#pragma once

// The optimiser state lives in device vectors of the padded layout (zero
// padding); its scalars are FP64 on the host.
struct fe_l2 {
  fe_ctx* ctx = nullptr;         // the padded grid, box mode
  fe::PadBox box{};
  double sigma_k = 0.0;
  int r = 0;                     // blur radius
  size_t n = 0;                  // padded elements
  size_t esz = 0;
  void* x = nullptr;             // the variable u (box plus replicated padding)
  void* g = nullptr;             // dF/du (zero padding)
  void* w0 = nullptr;            // work fields
  void* w1 = nullptr;
  void* w2 = nullptr;
  void* d = nullptr;             // search direction
  void* prev_g = nullptr;
  void* q = nullptr;             // two-loop scratch
  std::vector<void*> S, Y;       // history, oldest first (pointers rotate, memory stays)
  std::vector<double> rho;
  int hist_len = 0;
  double* d_red = nullptr;       // reduction partials, then the scalar slots (kL2Slots)
  // settings
  double lr = 1.0, tol_grad = 1e-7, tol_change = 1e-9;
  int history = 10, max_iter = 20, max_eval = 25;
  // state
  long n_iter = 0;
  double t = 0.0, H_diag = 1.0, prev_loss = 0.0;
};

namespace {

int l2_launch_1d(size_t n) { return (int)std::min<size_t>((n + 255) / 256, 65536); }

// Scalars of the optimiser. Each reduction has a slot: 0 energy, 1 max|g|,
// 2 max|d|, 3 g'd, 4 |g|_1, 5 y's, 6 y'y, 7 and 8 the y_i'd dots of the second
// loop (used in turn, so no pass reads the bank it writes), 9.. the s_i'q dots
// of the first loop of the two-loop recursion (one per history entry). d_red
// holds one bank of kVecBlocks partials per slot, then one value per slot for
// the host (the energy is written there directly).
constexpr int kSlotE = 0, kSlotGmax = 1, kSlotDmax = 2, kSlotGtd = 3, kSlotL1 = 4, kSlotYs = 5, kSlotYy = 6,
              kSlotDot = 7, kSlotDot2 = 8, kSlotAlpha = 9;
constexpr int kL2MaxHistory = 64;
constexpr int kL2Slots = kSlotAlpha + kL2MaxHistory;
constexpr size_t kL2RedDoubles = (size_t)kL2Slots * fe::kVecBlocks + kL2Slots;

double* l2_bank(fe_l2* L, int slot) { return L->d_red + (size_t)slot * fe::kVecBlocks; }
double* l2_vals(fe_l2* L) { return L->d_red + (size_t)kL2Slots * fe::kVecBlocks; }
int l2_slot_op(int slot) { return slot == kSlotGmax || slot == kSlotDmax ? 2 : slot == kSlotL1 ? 1 : 0; }

const dim3 kVecGrid(fe::kVecBlocks), kVecBlock(fe::kVecThreads);

// Reduction of a (and b) into the bank of `slot`, stream-ordered, no sync.
template <typename T>
int l2_reduce_dev(fe_l2* L, int op, const void* a, const void* b, int slot) {
  hipStream_t s = L->ctx->stream;
  const T* pa = static_cast<const T*>(a);
  const T* pb = static_cast<const T*>(b);
  double* bank = l2_bank(L, slot);
  if (op == 0)
    hipLaunchKernelGGL((fe::vec_reduce<T, 0>), kVecGrid, kVecBlock, 0, s, pa, pb, L->n, bank);
  else if (op == 1)
    hipLaunchKernelGGL((fe::vec_reduce<T, 1>), kVecGrid, kVecBlock, 0, s, pa, pb, L->n, bank);
  else
    hipLaunchKernelGGL((fe::vec_reduce<T, 2>), kVecGrid, kVecBlock, 0, s, pa, pb, L->n, bank);
  FE_HIP(hipGetLastError());
  return FE_OK;
}

// Host copies of the values of slots [first, first + count) (one sync): the
// banks among them are combined on the device first.
int l2_read_slots(fe_l2* L, int first, int count, double* out) {
  fe::BankList bl{};
  for (int k = first; k < first + count; ++k) {
    if (k == kSlotE) continue;
    if (bl.count == 4) return set_error(FE_EINVAL, "internal: too many slots in one read");
    bl.bank[bl.count] = l2_bank(L, k);
    bl.out[bl.count] = l2_vals(L) + k;
    bl.op[bl.count] = l2_slot_op(k);
    ++bl.count;
  }
  if (bl.count) {
    hipLaunchKernelGGL(fe::vec_finish, dim3(1), dim3(64), 0, L->ctx->stream, bl);
    FE_HIP(hipGetLastError());
  }
  FE_HIP(hipMemcpyAsync(out, l2_vals(L) + first, sizeof(double) * count, hipMemcpyDeviceToHost, L->ctx->stream));
  FE_HIP(hipStreamSynchronize(L->ctx->stream));
  return FE_OK;
}

// Coefficient ka v(ia) + kb v(ib) + kc of a vector pass, from the values of
// dot-product slots (ia, ib < 0: that term is absent).
struct L2Coef {
  int ia;
  double ka;
  int ib;
  double kb;
  double kc;
};

// y = alpha x (+ y when acc); then, when w is given, w . y into the bank of
// slot `out`. One pass, no sync.
template <typename T>
int l2_update(fe_l2* L, const L2Coef& k, bool acc, const void* x, void* y, const void* w = nullptr, int out = 0) {
  hipStream_t s = L->ctx->stream;
  const fe::VecCoef cf{k.ia >= 0 ? l2_bank(L, k.ia) : nullptr, k.ka, k.ib >= 0 ? l2_bank(L, k.ib) : nullptr, k.kb,
                       k.kc};
  const T* px = static_cast<const T*>(x);
  T* py = static_cast<T*>(y);
  const T* pw = static_cast<const T*>(w);
  double* bank = l2_bank(L, out);
  if (acc)
    hipLaunchKernelGGL((fe::vec_update_dot<T, true>), kVecGrid, kVecBlock, 0, s, cf, px, py, pw, L->n, bank);
  else
    hipLaunchKernelGGL((fe::vec_update_dot<T, false>), kVecGrid, kVecBlock, 0, s, cf, px, py, pw, L->n, bank);
  FE_HIP(hipGetLastError());
  return FE_OK;
}

// y = alpha x (+ y when acc) with a host coefficient
template <typename T>
int l2_scale_add(fe_l2* L, double alpha, const void* x, bool acc, void* y) {
  return l2_update<T>(L, L2Coef{-1, 0.0, -1, 0.0, alpha}, acc, x, y);
}

// The separable blur passes on the padded array (periodic within it):
// in -> tmp1 (x) -> tmp2 (y) -> out (z), or in -> tmp1 (fused x-y) -> out (z)
// for r = 4, 8; in and out may coincide, tmp1/tmp2 not.
template <typename T>
void l2_blur(fe_l2* L, const T* in, T* tmp1, T* tmp2, T* out) {
  const fe::FieldDims d{L->box.nx, L->box.ny, L->box.nz, 1};
  const fe::BlurTaps<T> k = blur_taps<T>(L->sigma_k);
  hipStream_t s = L->ctx->stream;
  if (has_xy_pass(k.r)) {
    blur_xy_pass<T>(s, d, k, in, tmp1);
    blur_axis_pass<T, 2>(s, d, k, tmp1, out);
    return;
  }
  blur_x_pass<T, false>(s, d, k, in, tmp1, nullptr, nullptr, T(0), nullptr, 0.0, 0.0);
  blur_yz<T>(s, d, k, tmp1, tmp2, out);
}

// The padding kernels: replicate padding over the pad shell, and its
// transpose (fixed-width runs for the pad widths 1, 4 and 8).
template <typename T>
void l2_pad(fe_l2* L, T* f) {
  const size_t n = fe::pad_shell_size(L->box);
  if (n == 0) return;
  hipLaunchKernelGGL(fe::pad_replicate<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, L->ctx->stream, f,
                     L->box);
}

template <typename T>
void l2_fold(fe_l2* L, const T* g, T* out) {
  const dim3 grid((unsigned)ceil_div(L->box.nx * L->box.ny, 256), (unsigned)L->box.nz);
  hipStream_t s = L->ctx->stream;
  const int W = L->box.lo[0];
  if (W == 4)
    hipLaunchKernelGGL((fe::fold_pads<T, 4>), grid, dim3(256), 0, s, g, out, L->box);
  else if (W == 8)
    hipLaunchKernelGGL((fe::fold_pads<T, 8>), grid, dim3(256), 0, s, g, out, L->box);
  else if (W == 1)
    hipLaunchKernelGGL((fe::fold_pads<T, 1>), grid, dim3(256), 0, s, g, out, L->box);
  else
    hipLaunchKernelGGL((fe::fold_pads<T, 0>), grid, dim3(256), 0, s, g, out, L->box);
}

// F_h(k * x) with replicate boundaries into the energy slot and g = its
// gradient (zero padding), stream-ordered.
template <typename T>
int l2_eval_dev(fe_l2* L) {
  T* x = static_cast<T*>(L->x);
  T* g = static_cast<T*>(L->g);
  T* w0 = static_cast<T*>(L->w0);
  T* w1 = static_cast<T*>(L->w1);
  T* w2 = static_cast<T*>(L->w2);
  l2_pad<T>(L, x);
  const T* ub = x;
  if (L->r > 0) {
    l2_blur<T>(L, x, w0, w1, w2);             // w2 = k * x
    l2_pad<T>(L, w2);
    ub = w2;
  }
  int rc = sweep_energy(L->ctx, L->ctx->stream, fe::kGrad, ub, w0, l2_vals(L) + kSlotE);   // w0 = g_ext
  if (rc) return rc;
  if (L->r > 0) {
    l2_fold<T>(L, w0, w1);                    // w1 = gb
    l2_blur<T>(L, w1, w0, w2, w1);           // w1 = k * gb (zero-extended)
    l2_fold<T>(L, w1, g);
  } else {
    l2_fold<T>(L, w0, g);
  }
  FE_HIP(hipGetLastError());
  return FE_OK;
}

// As l2_eval_dev, with the loss copied to the host (syncs).
template <typename T>
int l2_eval(fe_l2* L, double& loss) {
  int rc = l2_eval_dev<T>(L);
  if (rc) return rc;
  rc = l2_read_slots(L, kSlotE, 1, &loss);
  if (rc) return rc;
  if (!std::isfinite(loss)) return set_error(FE_ENONFINITE, "energy is not finite");
  return FE_OK;
}

// One optimiser step of L-BFGS without line search (Nocedal and Wright, the
// two-loop recursion with H0 = s'y / y'y): up to max_iter inner iterations,
// each a fixed step t d; the first ever step is scaled by min(1, 1/|g|_1);
// a pair (s, y) enters the history only if s'y > 1e-10. Stops early on
// max|g| <= tol_grad, a non-descent direction (g'd > -tol_change), a step
// max|t d| <= tol_change, or a loss change below tol_change. `loss0` receives
// the loss at the start of the step. The recursion's dot products stay in
// device scalar slots; the host reads scalars only where it branches on them
// (about three syncs per iteration).
template <typename T>
int l2_step(fe_l2* L, double& loss0) {
  int rc = l2_eval_dev<T>(L);
  if (rc) return rc;
  if ((rc = l2_reduce_dev<T>(L, 2, L->g, nullptr, kSlotGmax))) return rc;
  double sc[2];
  if ((rc = l2_read_slots(L, kSlotE, 2, sc))) return rc;
  double loss = sc[0], gmax = sc[1];
  if (!std::isfinite(loss)) return set_error(FE_ENONFINITE, "energy is not finite");
  loss0 = loss;
  int evals = 1;
  if (gmax <= L->tol_grad) return FE_OK;
  bool opt_cond = false;
  for (int it = 1; it <= L->max_iter; ++it) {
    ++L->n_iter;
    if (L->n_iter == 1) {
      if ((rc = l2_scale_add<T>(L, -1.0, L->g, false, L->d))) return rc;
      L->hist_len = 0;
      L->rho.clear();
      L->H_diag = 1.0;
    } else {
      // y = g - prev_g (in q), s = t d (in w0); accept the pair if y's > 1e-10
      hipLaunchKernelGGL(fe::vec_sub<T>, dim3(l2_launch_1d(L->n)), dim3(256), 0, L->ctx->stream,
                         static_cast<const T*>(L->g), static_cast<const T*>(L->prev_g), static_cast<T*>(L->q), L->n);
      FE_HIP(hipGetLastError());
      if ((rc = l2_scale_add<T>(L, L->t, L->d, false, L->w0))) return rc;
      if ((rc = l2_reduce_dev<T>(L, 0, L->q, L->w0, kSlotYs))) return rc;
      if ((rc = l2_reduce_dev<T>(L, 0, L->q, L->q, kSlotYy))) return rc;
      double yy2[2];
      if ((rc = l2_read_slots(L, kSlotYs, 2, yy2))) return rc;
      const double ys = yy2[0], yy = yy2[1];
      if (ys > 1e-10) {
        if (L->hist_len == L->history) {         // drop the oldest: rotate the slots
          std::rotate(L->S.begin(), L->S.begin() + 1, L->S.end());
          std::rotate(L->Y.begin(), L->Y.begin() + 1, L->Y.end());
          L->rho.erase(L->rho.begin());
          --L->hist_len;
        }
        // the new pair takes over the buffers of y and s; theirs become scratch
        std::swap(L->q, L->Y[L->hist_len]);
        std::swap(L->w0, L->S[L->hist_len]);
        L->rho.push_back(1.0 / ys);
        ++L->hist_len;
        L->H_diag = ys / yy;
      }
      // two-loop recursion: q = -g; newest to oldest: a_i = rho_i s_i'q, q -= a_i y_i;
      // d = H_diag q; oldest to newest: b_i = rho_i y_i'd, d += (a_i - b_i) s_i.
      // Each pass updates q (or d) and forms the dot product of the next entry.
      const int m = L->hist_len;
      if ((rc = l2_update<T>(L, L2Coef{-1, 0.0, -1, 0.0, -1.0}, false, L->g, L->q, m > 0 ? L->S[m - 1] : nullptr,
                             m > 0 ? kSlotAlpha + m - 1 : 0)))
        return rc;
      for (int i = m - 1; i >= 0; --i)
        if ((rc = l2_update<T>(L, L2Coef{kSlotAlpha + i, -L->rho[i], -1, 0.0, 0.0}, true, L->Y[i], L->q,
                               i > 0 ? L->S[i - 1] : nullptr, i > 0 ? kSlotAlpha + i - 1 : 0)))
          return rc;
      if ((rc = l2_update<T>(L, L2Coef{-1, 0.0, -1, 0.0, L->H_diag}, false, L->q, L->d, m > 0 ? L->Y[0] : nullptr,
                             kSlotDot)))
        return rc;
      for (int i = 0; i < m; ++i) {
        const int cur = (i & 1) ? kSlotDot2 : kSlotDot, nxt = (i & 1) ? kSlotDot : kSlotDot2;
        if ((rc = l2_update<T>(L, L2Coef{kSlotAlpha + i, L->rho[i], cur, -L->rho[i], 0.0}, true, L->S[i], L->d,
                               i + 1 < m ? L->Y[i + 1] : nullptr, nxt)))
          return rc;
      }
    }
    // prev_g takes over the gradient's buffer; the next evaluation writes g anew
    // (until then the current gradient is prev_g)
    std::swap(L->g, L->prev_g);
    L->prev_loss = loss;
    const bool first = L->n_iter == 1;
    if ((rc = l2_reduce_dev<T>(L, 0, L->prev_g, L->d, kSlotGtd))) return rc;
    if (first && (rc = l2_reduce_dev<T>(L, 1, L->prev_g, nullptr, kSlotL1))) return rc;
    double gl[2];
    if ((rc = l2_read_slots(L, kSlotGtd, first ? 2 : 1, gl))) return rc;
    L->t = first ? std::min(1.0, 1.0 / gl[1]) * L->lr : L->lr;
    const double gtd = gl[0];
    if (gtd > -L->tol_change) break;
    int ls_evals = 0;
    if ((rc = l2_scale_add<T>(L, L->t, L->d, true, L->x))) return rc;
    if ((rc = l2_reduce_dev<T>(L, 2, L->d, nullptr, kSlotDmax))) return rc;
    double dmax = 0.0;
    if (it != L->max_iter) {
      if ((rc = l2_eval_dev<T>(L))) return rc;
      if ((rc = l2_reduce_dev<T>(L, 2, L->g, nullptr, kSlotGmax))) return rc;
      double egd[3];
      if ((rc = l2_read_slots(L, kSlotE, 3, egd))) return rc;
      loss = egd[0];
      if (!std::isfinite(loss)) return set_error(FE_ENONFINITE, "energy is not finite");
      opt_cond = egd[1] <= L->tol_grad;
      dmax = egd[2];
      ls_evals = 1;
    }
    evals += ls_evals;
    if (it == L->max_iter) break;
    if (evals >= L->max_eval) break;
    if (opt_cond) break;
    if (dmax * std::fabs(L->t) <= L->tol_change) break;
    if (std::fabs(loss - L->prev_loss) < L->tol_change) break;
  }
  return FE_OK;
}

int l2_free(fe_l2* L) {
  if (!L) return FE_OK;
  for (void* p : {L->x, L->g, L->w0, L->w1, L->w2, L->d, L->prev_g, L->q, (void*)L->d_red})
    if (p) (void)hipFree(p);
  for (void* p : L->S)
    if (p) (void)hipFree(p);
  for (void* p : L->Y)
    if (p) (void)hipFree(p);
  if (L->ctx) fe_destroy(L->ctx);
  delete L;
  return FE_OK;
}

}  // namespace

extern "C" {

int fe_l2_create(const fe_grid* grid, double eps, const double* p_coeffs, double sigma_k, void* stream,
                 fe_l2** out) {
  g_last_error.clear();
  if (!out) return set_error(FE_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = check_grid(grid);
  if (rc) return rc;
  if (grid->batch != 1) return set_error(FE_EINVAL, "the L2 flow takes one field (batch 1)");
  if (!(sigma_k >= 0.0) || std::ceil(4.0 * sigma_k) > fe::kBlurMaxR)
    return set_error(FE_EINVAL, "sigma_k must lie in [0, %g]", fe::kBlurMaxR / 4.0);
  fe_l2* L = new (std::nothrow) fe_l2();
  if (!L) return set_error(FE_ENOMEM, "host allocation failed");
  L->sigma_k = sigma_k;
  L->r = sigma_k > 0.0 ? (int)std::ceil(4.0 * sigma_k) : 0;
  const int W = std::max(1, L->r);
  fe_grid pg = *grid;
  pg.nx += 2 * W;
  pg.ny += 2 * W;
  pg.nz += 2 * W;
  if ((long)pg.nz > 65535 || (long)pg.ny > 65535) {
    l2_free(L);
    return set_error(FE_EINVAL, "grid too large for the flow kernels");
  }
  rc = fe_create(&pg, &eps, p_coeffs, stream, &L->ctx);
  if (rc) {
    l2_free(L);
    return rc;
  }
  fe_ctx* c = L->ctx;
  c->use_box = true;
  c->variant = sweep_variant(c);
  const int dims[3] = {grid->nx, grid->ny, grid->nz};
  for (int i = 0; i < 3; ++i) {
    c->box_lo[i] = W;
    c->box_hi[i] = W + dims[i];
  }
  L->box = fe::PadBox{pg.nx, pg.ny, pg.nz, {W, W, W}, {W + grid->nx, W + grid->ny, W + grid->nz}};
  L->esz = elem_size(pg);
  L->n = field_elems(pg);
  DeviceGuard dg(c->device);
  for (void** p : {&L->x, &L->g, &L->w0, &L->w1, &L->w2, &L->d, &L->prev_g, &L->q}) {
    if (hipMalloc(p, L->n * L->esz) != hipSuccess) {
      *p = nullptr;
      l2_free(L);
      return set_error(FE_ENOMEM, "L2 flow field allocation failed");
    }
    if (hipMemsetAsync(*p, 0, L->n * L->esz, c->stream) != hipSuccess) {
      l2_free(L);
      return set_error(FE_EHIP, "hipMemsetAsync failed");
    }
  }
  if (hipMalloc((void**)&L->d_red, sizeof(double) * kL2RedDoubles) != hipSuccess) {
    L->d_red = nullptr;
    l2_free(L);
    return set_error(FE_ENOMEM, "L2 flow reduction buffer allocation failed");
  }
  if (hipMemsetAsync(L->d_red, 0, sizeof(double) * kL2RedDoubles, c->stream) != hipSuccess) {
    l2_free(L);
    return set_error(FE_EHIP, "hipMemsetAsync failed");
  }
  rc = fe_l2_set_lbfgs(L, 1.0, 10, 20, 1e-7, 1e-9);
  if (rc) {
    l2_free(L);
    return rc;
  }
  *out = L;
  return FE_OK;
}

int fe_l2_set_lbfgs(fe_l2* L, double lr, int history, int max_iter, double tolerance_grad, double tolerance_change) {
  g_last_error.clear();
  if (!L) return set_error(FE_EINVAL, "flow is NULL");
  if (!(lr > 0.0) || !std::isfinite(lr)) return set_error(FE_EINVAL, "lr must be finite and > 0");
  if (history < 1 || history > kL2MaxHistory)
    return set_error(FE_EINVAL, "history must lie in [1, %d]", kL2MaxHistory);
  if (max_iter < 1) return set_error(FE_EINVAL, "max_iter must be >= 1");
  if (!(tolerance_grad >= 0.0) || !(tolerance_change >= 0.0))
    return set_error(FE_EINVAL, "tolerances must be >= 0");
  DeviceGuard dg(L->ctx->device);
  if (history != (int)L->S.size()) {
    // allocate the new history first, so that a failure leaves the old one intact
    std::vector<void*> S(history, nullptr), Y(history, nullptr);
    bool ok = true;
    for (int i = 0; i < history && ok; ++i)
      ok = hipMalloc(&S[i], L->n * L->esz) == hipSuccess && hipMalloc(&Y[i], L->n * L->esz) == hipSuccess;
    if (!ok) {
      for (void* p : S)
        if (p) (void)hipFree(p);
      for (void* p : Y)
        if (p) (void)hipFree(p);
      return set_error(FE_ENOMEM, "L-BFGS history allocation failed");
    }
    for (void* p : L->S)
      if (p) (void)hipFree(p);
    for (void* p : L->Y)
      if (p) (void)hipFree(p);
    L->S.swap(S);
    L->Y.swap(Y);
  }
  L->lr = lr;
  L->history = history;
  L->max_iter = max_iter;
  L->max_eval = max_iter * 5 / 4;
  L->tol_grad = tolerance_grad;
  L->tol_change = tolerance_change;
  L->n_iter = 0;
  L->hist_len = 0;
  L->rho.clear();
  return FE_OK;
}

int fe_l2_load(fe_l2* L, const void* u) {
  g_last_error.clear();
  if (!L) return set_error(FE_EINVAL, "flow is NULL");
  if (!u) return set_error(FE_EINVAL, "u is NULL");
  DeviceGuard dg(L->ctx->device);
  const size_t nbox = (size_t)(L->box.hi[0] - L->box.lo[0]) * (L->box.hi[1] - L->box.lo[1]) *
                      (L->box.hi[2] - L->box.lo[2]);
  const int nb = l2_launch_1d(nbox);
  if (L->ctx->grid.dtype == FE_F32)
    hipLaunchKernelGGL(fe::box_copy<float>, dim3(nb), dim3(256), 0, L->ctx->stream, static_cast<const float*>(u),
                       static_cast<float*>(L->x), L->box, 1);
  else
    hipLaunchKernelGGL(fe::box_copy<double>, dim3(nb), dim3(256), 0, L->ctx->stream,
                       static_cast<const double*>(u), static_cast<double*>(L->x), L->box, 1);
  FE_HIP(hipGetLastError());
  L->n_iter = 0;
  L->hist_len = 0;
  L->rho.clear();
  return FE_OK;
}

int fe_l2_store(fe_l2* L, void* u) {
  g_last_error.clear();
  if (!L) return set_error(FE_EINVAL, "flow is NULL");
  if (!u) return set_error(FE_EINVAL, "u is NULL");
  DeviceGuard dg(L->ctx->device);
  const size_t nbox = (size_t)(L->box.hi[0] - L->box.lo[0]) * (L->box.hi[1] - L->box.lo[1]) *
                      (L->box.hi[2] - L->box.lo[2]);
  const int nb = l2_launch_1d(nbox);
  if (L->ctx->grid.dtype == FE_F32)
    hipLaunchKernelGGL(fe::box_copy<float>, dim3(nb), dim3(256), 0, L->ctx->stream,
                       static_cast<const float*>(L->x), static_cast<float*>(u), L->box, 0);
  else
    hipLaunchKernelGGL(fe::box_copy<double>, dim3(nb), dim3(256), 0, L->ctx->stream,
                       static_cast<const double*>(L->x), static_cast<double*>(u), L->box, 0);
  FE_HIP(hipGetLastError());
  return FE_OK;
}

int fe_l2_energy_grad(fe_l2* L, const void* u, void* g, double* energy) {
  int rc = fe_l2_load(L, u);
  if (rc) return rc;
  DeviceGuard dg(L->ctx->device);
  double E = 0.0;
  rc = L->ctx->grid.dtype == FE_F32 ? l2_eval<float>(L, E) : l2_eval<double>(L, E);
  if (rc) return rc;
  if (energy) *energy = E;
  if (g) {
    const size_t nbox = (size_t)(L->box.hi[0] - L->box.lo[0]) * (L->box.hi[1] - L->box.lo[1]) *
                        (L->box.hi[2] - L->box.lo[2]);
    const int nb = l2_launch_1d(nbox);
    if (L->ctx->grid.dtype == FE_F32)
      hipLaunchKernelGGL(fe::box_copy<float>, dim3(nb), dim3(256), 0, L->ctx->stream,
                         static_cast<const float*>(L->g), static_cast<float*>(g), L->box, 0);
    else
      hipLaunchKernelGGL(fe::box_copy<double>, dim3(nb), dim3(256), 0, L->ctx->stream,
                         static_cast<const double*>(L->g), static_cast<double*>(g), L->box, 0);
    FE_HIP(hipGetLastError());
  }
  return FE_OK;
}

int fe_l2_step(fe_l2* L, int nsteps, double* energies) {
  g_last_error.clear();
  if (!L) return set_error(FE_EINVAL, "flow is NULL");
  if (nsteps < 0) return set_error(FE_EINVAL, "nsteps must be >= 0");
  DeviceGuard dg(L->ctx->device);
  for (int k = 0; k < nsteps; ++k) {
    double E = 0.0;
    const int rc = L->ctx->grid.dtype == FE_F32 ? l2_step<float>(L, E) : l2_step<double>(L, E);
    if (rc) return rc;
    if (energies) energies[k] = E;
  }
  return FE_OK;
}

int fe_l2_set_stream(fe_l2* L, void* stream) {
  g_last_error.clear();
  if (!L) return set_error(FE_EINVAL, "flow is NULL");
  return fe_set_stream(L->ctx, stream);
}

void fe_l2_destroy(fe_l2* L) { l2_free(L); }

}  // extern "C"
