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
  std::vector<double> SY, YY;    // [history][history]: s_a . y_b (a <= b) and y_a . y_b of the history
  std::vector<double> pgS, pgY;  // prev_g . s_a and prev_g . y_a for the current history
  int hist_len = 0;
  double* d_red = nullptr;       // reduction banks, then their values (kL2Banks each)
  // settings
  double lr = 1.0, tol_grad = 1e-7, tol_change = 1e-9;
  int history = 10, max_iter = 20, max_eval = 25;
  // state
  long n_iter = 0;
  double t = 0.0, H_diag = 1.0, prev_loss = 0.0;
};

namespace {

int l2_launch_1d(size_t n) { return (int)std::min<size_t>((n + 255) / 256, 65536); }

// Scalars of the optimiser. Named slots: 0 energy, 1 max|g|, 2 max|d|, 3 g'd
// and 4 |g|_1 (first iteration); then the inner products of the Gram pass
// (y.y, y.s, y.g, g.g, g.s, then g.V_k for each history vector). d_red
// holds one bank of kVecBlocks partials per slot, then one value per slot for
// the host (the energy is written there directly).
constexpr int kSlotE = 0, kSlotGmax = 1, kSlotDmax = 2, kSlotGtd = 3, kSlotL1 = 4, kSlotGram = 5;
constexpr int kL2MaxHistory = 64;
constexpr int kL2Banks = kSlotGram + 5 + 2 * kL2MaxHistory;
constexpr size_t kL2RedDoubles = (size_t)kL2Banks * fe::kVecBlocks + kL2Banks;

double* l2_bank(fe_l2* L, int slot) { return L->d_red + (size_t)slot * fe::kVecBlocks; }
double* l2_vals(fe_l2* L) { return L->d_red + (size_t)kL2Banks * fe::kVecBlocks; }
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

// Host copies of the values of named slots [first, first + count) (one sync):
// the banks among them are combined on the device first.
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

// out = sum_k c[k] v[k] (+ out when acc), in passes of up to kCombVecs vectors;
// with dmax, the last pass leaves max |out| in the bank of kSlotDmax. No sync.
template <typename T>
int l2_lincomb(fe_l2* L, const std::vector<const void*>& v, const std::vector<double>& c, bool acc, void* out,
               bool dmax, void* x = nullptr, double t = 0.0) {
  const size_t K = v.size();
  for (size_t k0 = 0; k0 < K; k0 += fe::kCombVecs) {
    fe::CombList<T> cl{};
    cl.count = (int)std::min<size_t>(fe::kCombVecs, K - k0);
    // pass widths 1, 4, 8, 16 or 24; the padding repeats the first vector with c = 0
    const int w = cl.count == 1 ? 1 : cl.count <= 4 ? 4 : cl.count <= 8 ? 8 : cl.count <= 16 ? 16 : fe::kCombVecs;
    for (int k = 0; k < w; ++k) {
      cl.v[k] = static_cast<const T*>(v[k < cl.count ? k0 + k : k0]);
      cl.c[k] = k < cl.count ? c[k0 + k] : 0.0;
    }
    const int a = (acc || k0 > 0) ? 1 : 0;
    const bool last = k0 + fe::kCombVecs >= K;
    double* dm = (dmax && last) ? l2_bank(L, kSlotDmax) : nullptr;
    T* px = last ? static_cast<T*>(x) : nullptr;
    T* po = static_cast<T*>(out);
    hipStream_t s = L->ctx->stream;
    if (w == 1)
      hipLaunchKernelGGL((fe::vec_lincomb<T, 1>), kVecGrid, kVecBlock, 0, s, cl, po, a, L->n, dm, px, t);
    else if (w == 4)
      hipLaunchKernelGGL((fe::vec_lincomb<T, 4>), kVecGrid, kVecBlock, 0, s, cl, po, a, L->n, dm, px, t);
    else if (w == 8)
      hipLaunchKernelGGL((fe::vec_lincomb<T, 8>), kVecGrid, kVecBlock, 0, s, cl, po, a, L->n, dm, px, t);
    else if (w == 16)
      hipLaunchKernelGGL((fe::vec_lincomb<T, 16>), kVecGrid, kVecBlock, 0, s, cl, po, a, L->n, dm, px, t);
    else
      hipLaunchKernelGGL((fe::vec_lincomb<T, fe::kCombVecs>), kVecGrid, kVecBlock, 0, s, cl, po, a, L->n, dm, px, t);
    FE_HIP(hipGetLastError());
  }
  return FE_OK;
}

// y = alpha x (+ y when acc) with a host coefficient
template <typename T>
int l2_scale_add(fe_l2* L, double alpha, const void* x, bool acc, void* y) {
  return l2_lincomb<T>(L, {x}, {alpha}, acc, y, false);
}

// The Gram pass: y = g - prev_g into L->q, s = t d into L->w0, and the inner
// products y.y, y.s, y.g, g.g, g.s and, for every vector v of `hist`, g.v,
// copied to `out` in that order (one sync). Up to kDotVecs history vectors go
// through one pass; a list of 8, 16 or 24 entries, the unused ones pointing at g.
template <typename T>
void gram_launch(fe_l2* L, bool form, const fe::DotList<T>& dl, int bank) {
  hipStream_t s = L->ctx->stream;
  const T* g = static_cast<const T*>(L->g);
  const T* pg = static_cast<const T*>(L->prev_g);
  const T* d = static_cast<const T*>(L->d);
  T* y = static_cast<T*>(L->q);
  T* sv = static_cast<T*>(L->w0);
  double* bk = l2_bank(L, bank);
  const dim3 grid = kVecGrid, blk(fe::gram_threads<T>());
  const int nl = dl.count == 0 ? 0 : dl.count <= 8 ? 8 : dl.count <= 16 ? 16 : fe::kDotVecs;
  if (form) {
    if (nl == 0)
      hipLaunchKernelGGL((fe::vec_gram<T, true, 0>), grid, blk, 0, s, g, pg, d, L->t, y, sv, dl, L->n, bk);
    else if (nl == 8)
      hipLaunchKernelGGL((fe::vec_gram<T, true, 8>), grid, blk, 0, s, g, pg, d, L->t, y, sv, dl, L->n, bk);
    else if (nl == 16)
      hipLaunchKernelGGL((fe::vec_gram<T, true, 16>), grid, blk, 0, s, g, pg, d, L->t, y, sv, dl, L->n, bk);
    else
      hipLaunchKernelGGL((fe::vec_gram<T, true, fe::kDotVecs>), grid, blk, 0, s, g, pg, d, L->t, y, sv, dl, L->n,
                         bk);
  } else {
    if (nl == 8)
      hipLaunchKernelGGL((fe::vec_gram<T, false, 8>), grid, blk, 0, s, g, nullptr, nullptr, 0.0, nullptr, nullptr, dl,
                         L->n, bk);
    else if (nl == 16)
      hipLaunchKernelGGL((fe::vec_gram<T, false, 16>), grid, blk, 0, s, g, nullptr, nullptr, 0.0, nullptr, nullptr,
                         dl, L->n, bk);
    else
      hipLaunchKernelGGL((fe::vec_gram<T, false, fe::kDotVecs>), grid, blk, 0, s, g, nullptr, nullptr, 0.0, nullptr,
                         nullptr, dl, L->n, bk);
  }
}

template <typename T>
int l2_gram(fe_l2* L, const std::vector<const void*>& hist, std::vector<double>& out) {
  hipStream_t s = L->ctx->stream;
  const T* g = static_cast<const T*>(L->g);
  const size_t K = hist.size();
  int bank = kSlotGram;
  size_t k0 = 0;
  do {
    fe::DotList<T> dl{};
    dl.count = (int)std::min<size_t>(fe::kDotVecs, K - k0);
    for (int k = 0; k < fe::kDotVecs; ++k) dl.v[k] = k < dl.count ? static_cast<const T*>(hist[k0 + k]) : g;
    gram_launch<T>(L, k0 == 0, dl, bank);
    FE_HIP(hipGetLastError());
    bank += (k0 == 0 ? 5 : 0) + dl.count;
    k0 += dl.count;
  } while (k0 < K);
  const int nv = bank - kSlotGram;
  hipLaunchKernelGGL(fe::vec_finish_sums, dim3(nv), dim3(64), 0, s, (const double*)l2_bank(L, kSlotGram),
                     l2_vals(L) + kSlotGram);
  FE_HIP(hipGetLastError());
  out.resize(nv);
  FE_HIP(hipMemcpyAsync(out.data(), l2_vals(L) + kSlotGram, sizeof(double) * nv, hipMemcpyDeviceToHost, s));
  FE_HIP(hipStreamSynchronize(s));
  return FE_OK;
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
// transpose (fixed-width runs for the pad widths 1, 4 and 8 on boxes at least
// 2 voxels thick, general runs otherwise).
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
  // the fixed-width forms need a box at least 2 voxels thick on every axis
  bool thick = true;
  for (int a = 0; a < 3; ++a) thick = thick && L->box.hi[a] - L->box.lo[a] >= 2;
  const int W = thick ? L->box.lo[0] : 0;
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
    const bool first = L->n_iter == 1;
    double gtd = 0.0, gl1 = 0.0;
    bool moved = false;   // x already advanced by the direction pass
    if (first) {
      if ((rc = l2_lincomb<T>(L, {L->g}, {-1.0}, false, L->d, true))) return rc;   // d = -g
      L->hist_len = 0;
      L->rho.clear();
      L->pgS.clear();
      L->pgY.clear();
      L->H_diag = 1.0;
      if ((rc = l2_reduce_dev<T>(L, 0, L->g, L->d, kSlotGtd))) return rc;
      if ((rc = l2_reduce_dev<T>(L, 1, L->g, nullptr, kSlotL1))) return rc;
      double gl[2];
      if ((rc = l2_read_slots(L, kSlotGtd, 2, gl))) return rc;
      gtd = gl[0];
      gl1 = gl[1];
    } else {
      // The Gram pass: y = g - prev_g (in q), s = t d (in w0), the inner
      // products of y and g with each other and with s, and g with every
      // history vector; y with a history vector is g.v - prev_g.v, the latter
      // kept from the previous pass (prev_g was that pass's g).
      int m = L->hist_len;
      const int H = L->history;
      std::vector<const void*> hist;
      for (int i = 0; i < m; ++i) hist.push_back(L->S[i]);
      for (int i = 0; i < m; ++i) hist.push_back(L->Y[i]);
      std::vector<double> gv;
      if ((rc = l2_gram<T>(L, hist, gv))) return rc;
      const double yy = gv[0], ys = gv[1], yg = gv[2], gg = gv[3], gs = gv[4];
      if ((int)L->pgS.size() != m || (int)L->pgY.size() != m)
        return set_error(FE_EINVAL, "L-BFGS state out of step with its history");
      std::vector<double> yS(m), gS(m), yY(m), gY(m);
      for (int i = 0; i < m; ++i) {
        gS[i] = gv[5 + i];
        gY[i] = gv[5 + m + i];
        yS[i] = gS[i] - L->pgS[i];
        yY[i] = gY[i] - L->pgY[i];
      }
      double* SY = L->SY.data();
      double* YY = L->YY.data();
      // accept the pair if y's > 1e-10 (the oldest leaves a full history)
      if (ys > 1e-10) {
        if (m == H) {
          std::rotate(L->S.begin(), L->S.begin() + 1, L->S.end());
          std::rotate(L->Y.begin(), L->Y.begin() + 1, L->Y.end());
          L->rho.erase(L->rho.begin());
          for (int a = 0; a + 1 < m; ++a)
            for (int b = 0; b + 1 < m; ++b) {
              SY[a * H + b] = SY[(a + 1) * H + b + 1];
              YY[a * H + b] = YY[(a + 1) * H + b + 1];
            }
          for (auto* v : {&yS, &gS, &yY, &gY}) v->erase(v->begin());
          --m;
        }
        // the new pair takes over the buffers of y and s; theirs become scratch
        std::swap(L->q, L->Y[m]);
        std::swap(L->w0, L->S[m]);
        for (int a = 0; a < m; ++a) {
          SY[a * H + m] = yS[a];                 // s_a . y_new
          YY[a * H + m] = YY[m * H + a] = yY[a];
        }
        SY[m * H + m] = ys;
        YY[m * H + m] = yy;
        gS.push_back(gs);
        gY.push_back(yg);
        L->rho.push_back(1.0 / ys);
        L->hist_len = ++m;
        L->H_diag = ys / yy;
      }
      // g becomes prev_g below: keep its products with the history as it now stands
      L->pgS = gS;
      L->pgY = gY;
      // The two-loop recursion on the inner products, newest to oldest:
      //   a_i = rho_i s_i.q with q = -g - sum_{j>i} a_j y_j,
      // then r = H q (q = -g - sum_j a_j y_j), oldest to newest:
      //   b_i = rho_i y_i.r with r = H q + sum_{j<i} (a_j - b_j) s_j,
      // and d = H q + sum_i (a_i - b_i) s_i = -H g - H sum_j a_j y_j + sum_i (a_i - b_i) s_i.
      const double Hd = L->H_diag;
      std::vector<double> al(m), be(m);
      for (int i = m - 1; i >= 0; --i) {
        double sq = -gS[i];
        for (int j = i + 1; j < m; ++j) sq -= al[j] * SY[i * H + j];
        al[i] = L->rho[i] * sq;
      }
      for (int i = 0; i < m; ++i) {
        double yq = -gY[i];
        for (int j = 0; j < m; ++j) yq -= al[j] * YY[i * H + j];
        double yr = Hd * yq;
        for (int j = 0; j < i; ++j) yr += (al[j] - be[j]) * SY[j * H + i];
        be[i] = L->rho[i] * yr;
      }
      std::vector<const void*> vv{L->g};
      std::vector<double> cc{-Hd};
      gtd = -Hd * gg;
      for (int i = 0; i < m; ++i) {
        vv.push_back(L->S[i]);
        cc.push_back(al[i] - be[i]);
        gtd += (al[i] - be[i]) * gS[i];
      }
      for (int j = 0; j < m; ++j) {
        vv.push_back(L->Y[j]);
        cc.push_back(-Hd * al[j]);
        gtd += -Hd * al[j] * gY[j];
      }
      // when the step will be taken (t = lr, g'd below -tol_change), the pass
      // that forms d also moves x
      moved = !(gtd > -L->tol_change);
      if ((rc = l2_lincomb<T>(L, vv, cc, false, L->d, true, moved ? L->x : nullptr, L->lr))) return rc;
    }
    // prev_g takes over the gradient's buffer; the next evaluation writes g anew
    std::swap(L->g, L->prev_g);
    L->prev_loss = loss;
    L->t = first ? std::min(1.0, 1.0 / gl1) * L->lr : L->lr;
    if (gtd > -L->tol_change) break;
    int ls_evals = 0;
    if (!moved && (rc = l2_scale_add<T>(L, L->t, L->d, true, L->x))) return rc;   // max |d| is in its slot already
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
  if ((long)pg.nz > 65535 || (long)pg.ny > 65535 || !flow_dims_ok(pg)) {
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
  L->pgS.clear();
  L->pgY.clear();
  L->SY.assign((size_t)history * history, 0.0);
  L->YY.assign((size_t)history * history, 0.0);
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
  L->pgS.clear();
  L->pgY.clear();
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
