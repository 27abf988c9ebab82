// Host side of Algorithm 1 (the H^-1 flow on a vector field): the blur
// passes, the iteration, and its entry points. Included once by fe_api.hip.
#pragma once

namespace {

template <typename T>
fe::BlurTaps<T> blur_taps(double sigma_k) {
  fe::BlurTaps<T> k{};
  k.r = sigma_k > 0.0 ? (int)std::ceil(4.0 * sigma_k) : 0;
  double w[2 * fe::kBlurMaxR + 1];
  double sum = 0.0;
  for (int j = -k.r; j <= k.r; ++j) {
    w[j + k.r] = k.r ? std::exp(-(double)j * j / (2.0 * sigma_k * sigma_k)) : 1.0;
    sum += w[j + k.r];
  }
  for (int j = 0; j <= 2 * k.r; ++j) k.w[j] = T(w[j] / sum);
  return k;
}

struct FlowRule {
  double sigma_k, lr, beta1, beta2, adam_eps;
};

// Launch shapes of the flow kernels.
dim3 x_grid(const fe::FieldDims& d) { return dim3(ceil_div(d.nx, 64), ceil_div(d.ny, fe::kBlurRows), d.nz * d.batch); }
dim3 axis_grid(const fe::FieldDims& d, int axis) {
  return axis == 1 ? dim3(ceil_div(d.nz * d.nx, 256), ceil_div(d.ny, fe::kAxisChunk), d.batch)
                   : dim3(ceil_div(d.nx * d.ny, 256), ceil_div(d.nz, fe::kAxisChunk), d.batch);
}
// The flow kernels address a plane with 32-bit byte offsets and number the
// columns of the y pass (nz * nx of them) in 32-bit integers.
bool flow_dims_ok(const fe_grid& g) {
  return (double)g.nx * g.ny * elem_size(g) < 4294967296.0 && (double)g.nz * g.nx < 2147483392.0;
}

// flat runs of 256 voxels of a plane, one plane per grid z
dim3 plane_grid(const fe::FieldDims& d) { return dim3(ceil_div(d.nx * d.ny, 256), 1, d.nz * d.batch); }

// Whole rows staged per block (the ROWS forms) when a row and its halo fit
// the 128 staged values.
bool rows_fit(const fe::FieldDims& d, int r) { return d.nx + 2 * r <= fe::kRowsMax; }

// The x pass (with the divergence when DIV), dispatched to the fixed-radius
// instantiation when there is one, and to its ROWS form when the rows fit.
template <typename T, bool DIV>
void blur_x_pass(hipStream_t s, const fe::FieldDims& d, const fe::BlurTaps<T>& k, const T* in, T* out,
                 const double* m0, const T* mfield, T inv2h, fe::FlowClock* clk, double beta1, double beta2) {
  const dim3 g = x_grid(d), b(64, 4);
  const dim3 gr(1, g.y, g.z);
  if (k.r == 4 && rows_fit(d, 4))
    hipLaunchKernelGGL((fe::blur_x<T, DIV, 4, true>), gr, b, 0, s, in, out, m0, mfield, d, inv2h, k, clk, beta1,
                       beta2);
  else if (k.r == 8 && rows_fit(d, 8))
    hipLaunchKernelGGL((fe::blur_x<T, DIV, 8, true>), gr, b, 0, s, in, out, m0, mfield, d, inv2h, k, clk, beta1,
                       beta2);
  else if (k.r == 4)
    hipLaunchKernelGGL((fe::blur_x<T, DIV, 4>), g, b, 0, s, in, out, m0, mfield, d, inv2h, k, clk, beta1, beta2);
  else if (k.r == 8)
    hipLaunchKernelGGL((fe::blur_x<T, DIV, 8>), g, b, 0, s, in, out, m0, mfield, d, inv2h, k, clk, beta1, beta2);
  else
    hipLaunchKernelGGL((fe::blur_x<T, DIV>), g, b, 0, s, in, out, m0, mfield, d, inv2h, k, clk, beta1, beta2);
}

// The fused x-then-y pass, for the radii that have one (r = 4 and 8).
bool has_xy_pass(int r) { return r == 4 || r == 8; }
dim3 xy_grid(const fe::FieldDims& d) { return dim3(ceil_div(d.nx, 64), ceil_div(d.ny, fe::kXYRows), d.nz * d.batch); }

template <typename T>
void blur_xy_pass(hipStream_t s, const fe::FieldDims& d, const fe::BlurTaps<T>& k, const T* in, T* out) {
  const dim3 g = xy_grid(d), b(64, 8);
  const dim3 gr(1, g.y, g.z);
  if (k.r == 4 && rows_fit(d, 4))
    hipLaunchKernelGGL((fe::blur_xy<T, 4, true>), gr, b, 0, s, in, out, d, k);
  else if (k.r == 4)
    hipLaunchKernelGGL((fe::blur_xy<T, 4>), g, b, 0, s, in, out, d, k);
  else if (rows_fit(d, 8))
    hipLaunchKernelGGL((fe::blur_xy<T, 8, true>), gr, b, 0, s, in, out, d, k);
  else
    hipLaunchKernelGGL((fe::blur_xy<T, 8>), g, b, 0, s, in, out, d, k);
}

template <typename T, int AXIS>
void blur_axis_pass(hipStream_t s, const fe::FieldDims& d, const fe::BlurTaps<T>& k, const T* in, T* out) {
  const dim3 g = axis_grid(d, AXIS), b(256);
  if (k.r == 4)
    hipLaunchKernelGGL((fe::blur_axis<T, AXIS, 4>), g, b, 0, s, in, out, d, k);
  else if (k.r == 8)
    hipLaunchKernelGGL((fe::blur_axis<T, AXIS, 8>), g, b, 0, s, in, out, d, k);
  else
    hipLaunchKernelGGL((fe::blur_axis<T, AXIS>), g, b, 0, s, in, out, d, k);
}

// out = k * f along y then z, through `tmp` (f is left as it was; out may be f).
template <typename T>
void blur_yz(hipStream_t s, const fe::FieldDims& d, const fe::BlurTaps<T>& k, const T* f, T* tmp, T* out) {
  blur_axis_pass<T, 1>(s, d, k, f, tmp);
  blur_axis_pass<T, 2>(s, d, k, tmp, out);
}

// u = k * (div A + m0) into `out` (a user field or the work field w0, never
// w1): x pass into w0, y pass into w1, z pass into out. `clk` advances the
// flow clock (iterations only). The fused x-y pass is not used here: with the
// divergence its staging costs more than the pass it saves once the grid
// outgrows one wave of blocks (16 x 100^3: 162 us against 93 + 47 us).
template <typename T>
int flow_field(fe_ctx* c, hipStream_t s, const void* A, T* out, double sigma_k, fe::FlowClock* clk,
               double beta1, double beta2) {
  const fe::FieldDims d{c->grid.nx, c->grid.ny, c->grid.nz, c->grid.batch};
  const fe::BlurTaps<T> k = blur_taps<T>(sigma_k);
  const T inv2h = T(1.0 / (2.0 * c->grid.h));
  T* w0 = static_cast<T*>(c->d_w0);
  const T* mf = c->use_mfield ? static_cast<const T*>(c->d_mfield) : nullptr;
  if (k.r == 0) {
    blur_x_pass<T, true>(s, d, k, (const T*)A, out, c->d_mass, mf, inv2h, clk, beta1, beta2);
  } else {
    blur_x_pass<T, true>(s, d, k, (const T*)A, w0, c->d_mass, mf, inv2h, clk, beta1, beta2);
    blur_yz<T>(s, d, k, w0, static_cast<T*>(c->d_w1), out);
  }
  FE_HIP(hipGetLastError());
  return FE_OK;
}

// One iteration of Algorithm 1 on A (in place); the energy of its field stays
// in the block partials (partials_buf 0) for finish_sums.
template <typename T>
int flow_iteration(fe_ctx* c, hipStream_t s, void* A, const FlowRule& fr) {
  T* w0 = static_cast<T*>(c->d_w0);
  T* w1 = static_cast<T*>(c->d_w1);
  const fe::FieldDims d{c->grid.nx, c->grid.ny, c->grid.nz, c->grid.batch};
  const fe::BlurTaps<T> k = blur_taps<T>(fr.sigma_k);
  // ub = k * (div A + m0) in w0
  int rc = flow_field<T>(c, s, A, w0, fr.sigma_k, c->d_flow_clk, fr.beta1, fr.beta2);
  if (rc) return rc;
  // gb = dF/du at ub, in w1 (the energy of ub stays in the block partials)
  const StepRule none{fe::kGrad, 0.0, 0.0, 0.0, 0.0};
  rc = sweep(c, s, fe::kGrad, w0, w1, nullptr, partials_buf(c, 0), none);
  if (rc) return rc;
  const T inv2h = T(1.0 / (2.0 * c->grid.h));
  const fe::FlowClock* clk = c->d_flow_clk;
  // gu = k * gb: for r = 4, 8 the x-y pass into w0 and the z pass into w1;
  // otherwise the x pass into w0, the y pass into w1, the z pass into w0
  const T* gu = w1;
  if (has_xy_pass(k.r)) {
    blur_xy_pass<T>(s, d, k, (const T*)w1, w0);
    blur_axis_pass<T, 2>(s, d, k, (const T*)w0, w1);
  } else if (k.r > 0) {
    blur_x_pass<T, false>(s, d, k, (const T*)w1, w0, nullptr, nullptr, T(0), nullptr, 0.0, 0.0);
    blur_yz<T>(s, d, k, w0, w1, w0);
    gu = w0;
  }
  hipLaunchKernelGGL(fe::adam_vector_field<T>, plane_grid(d), dim3(256), 0, s, gu, (T*)A, (T*)c->d_am1,
                     (T*)c->d_am2, d, inv2h, T(fr.lr), T(fr.beta1), T(fr.beta2), T(fr.adam_eps), clk);
  FE_HIP(hipGetLastError());
  return FE_OK;
}

int flow_iteration_any(fe_ctx* c, hipStream_t s, void* A, const FlowRule& fr) {
  return c->grid.dtype == FE_F32 ? flow_iteration<float>(c, s, A, fr) : flow_iteration<double>(c, s, A, fr);
}

int flow_reset_launch(fe_ctx* c) {
  const size_t n = 3 * field_elems(c->grid);
  const int nblk = (int)std::min<size_t>((n + 255) / 256, 65536);
  if (c->grid.dtype == FE_F32)
    hipLaunchKernelGGL(fe::flow_reset<float>, dim3(nblk), dim3(256), 0, c->stream, (float*)c->d_am1,
                       (float*)c->d_am2, n, c->d_flow_clk);
  else
    hipLaunchKernelGGL(fe::flow_reset<double>, dim3(nblk), dim3(256), 0, c->stream, (double*)c->d_am1,
                       (double*)c->d_am2, n, c->d_flow_clk);
  FE_HIP(hipGetLastError());
  return FE_OK;
}

}  // namespace

extern "C" {

int fe_hminus_step(fe_ctx* c, void* A, const double* m0, double sigma_k, double lr, double beta1, double beta2,
                   double adam_eps, int nsteps, void* u_out, double* energy) {
  g_last_error.clear();
  if (!c) return set_error(FE_EINVAL, "ctx is NULL");
  if (!A) return set_error(FE_EINVAL, "A is NULL");
  if (!m0 && !c->use_mfield) return set_error(FE_EINVAL, "m0 is NULL and no mass field is set");
  if (nsteps < 0) return set_error(FE_EINVAL, "nsteps must be >= 0");
  if (!(sigma_k >= 0.0) || std::ceil(4.0 * sigma_k) > fe::kBlurMaxR)
    return set_error(FE_EINVAL, "sigma_k must lie in [0, %g]", fe::kBlurMaxR / 4.0);
  if (!(lr > 0.0) || !std::isfinite(lr)) return set_error(FE_EINVAL, "lr must be finite and > 0");
  if (!(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0))
    return set_error(FE_EINVAL, "beta1 and beta2 must lie in [0, 1)");
  if (!(adam_eps > 0.0) || !std::isfinite(adam_eps)) return set_error(FE_EINVAL, "adam_eps must be finite and > 0");
  if ((long)c->grid.nz * c->grid.batch > 65535)
    return set_error(FE_EINVAL, "nz * batch must be <= 65535 for the flow kernels");
  if (!flow_dims_ok(c->grid)) return set_error(FE_EINVAL, "planes of 4 GiB or more (or nz * nx >= 2^31) are too large for the flow kernels");
  if (u_out == A) return set_error(FE_EINVAL, "u_out must not alias A");
  for (int b = 0; b < c->grid.batch; ++b)
    if (m0 && !std::isfinite(m0[b])) return set_error(FE_EINVAL, "m0[%d] is not finite", b);
  DeviceGuard dg(c->device);
  const size_t bytes = field_elems(c->grid) * elem_size(c->grid);
  if (!c->d_w0) {
    if (hipMalloc(&c->d_w0, bytes) != hipSuccess || hipMalloc(&c->d_w1, bytes) != hipSuccess ||
        hipMalloc(&c->d_am1, 3 * bytes) != hipSuccess || hipMalloc(&c->d_am2, 3 * bytes) != hipSuccess ||
        hipMalloc((void**)&c->d_flow_clk, sizeof(fe::FlowClock)) != hipSuccess) {
      for (void** p : {&c->d_w0, &c->d_w1, &c->d_am1, &c->d_am2, (void**)&c->d_flow_clk}) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
      }
      return set_error(FE_ENOMEM, "H^-1 flow workspace allocation failed");
    }
    int rc = flow_reset_launch(c);
    if (rc) return rc;
  }
  if (m0) FE_HIP(hipMemcpyAsync(c->d_mass, m0, sizeof(double) * c->grid.batch, hipMemcpyHostToDevice, c->stream));
  const FlowRule fr{sigma_k, lr, beta1, beta2, adam_eps};
  constexpr int kGraphIters = 8;
  const int gi = nsteps >= kGraphIters ? kGraphIters : 0;
  for (int i = 0; i < (gi ? nsteps % gi : nsteps); ++i) {
    int rc = flow_iteration_any(c, c->stream, A, fr);
    if (rc) return rc;
  }
  if (gi > 0) {
    GraphKey key{A, kFlowMode, lr, beta1, beta2, adam_eps, sigma_k, gi, sweep_variant(c), c->lz, fields_in_use(c)};
    auto it = c->graphs.find(key);
    hipGraphExec_t exec = nullptr;
    if (it == c->graphs.end()) {
      hipGraph_t graph = nullptr;
      FE_HIP(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
      int rc = FE_OK;
      for (int i = 0; i < gi && rc == FE_OK; ++i) rc = flow_iteration_any(c, c->cap_stream, A, fr);
      hipError_t ec = hipStreamEndCapture(c->cap_stream, &graph);
      if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
      }
      if (ec != hipSuccess) return set_error(FE_EHIP, "graph capture failed: %s", hipGetErrorString(ec));
      hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ei != hipSuccess) return set_error(FE_EHIP, "graph instantiate failed: %s", hipGetErrorString(ei));
      if (c->graphs.size() > 16) drop_graphs(c);
      c->graphs[key] = exec;
    } else {
      exec = it->second;
    }
    for (int r = 0; r < nsteps / gi; ++r) FE_HIP(hipGraphLaunch(exec, c->stream));
  }
  if (u_out) {
    int rc = c->grid.dtype == FE_F32
                 ? flow_field<float>(c, c->stream, A, (float*)u_out, sigma_k, nullptr, 0.0, 0.0)
                 : flow_field<double>(c, c->stream, A, (double*)u_out, sigma_k, nullptr, 0.0, 0.0);
    if (rc) return rc;
  }
  if (nsteps == 0) {
    if (energy) for (int b = 0; b < c->grid.batch; ++b) energy[b] = 0.0;
    return FE_OK;
  }
  int rc = finish_sums(c, c->stream, partials_buf(c, 0), c->d_energy, nullptr, fe::kGrad);   // the last iteration's G
  if (rc) return rc;
  return copy_energy_out(c, energy);
}

int fe_hminus_reset(fe_ctx* c) {
  g_last_error.clear();
  if (!c) return set_error(FE_EINVAL, "ctx is NULL");
  if (!c->d_am1) return FE_OK;
  DeviceGuard dg(c->device);
  return flow_reset_launch(c);
}

}  // extern "C"
