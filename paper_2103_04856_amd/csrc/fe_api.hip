// Host side of the C ABI declared in include/fe.h: argument validation,
// per-instance constants, launch-shape selection, the graph-replayed step
// loop and the autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "fe.h"
#include "fe_flow.hpp"
#include "fe_diag.hpp"
#include "fe_l2flow.hpp"
#include "fe_kernels.hpp"

namespace {

thread_local std::string g_last_error;

int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

#define FE_HIP(call)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return set_error(FE_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));          \
  } while (0)

constexpr double kXi = 1e-6;   // Sec. 4.1: offset of |grad u| and scale of the smoothed x^+
constexpr int kGraphPairs = 8;  // descent steps per captured graph: 2 x kGraphPairs

// ---------------------------------------------------------------------------
// Launch variants: interior tile (TX x TY) and threads per block.
// ---------------------------------------------------------------------------

template <typename T>
using SweepFn = void (*)(fe::SweepArgs<T>);

template <typename T>
struct Kernels {
  SweepFn<T> grad = nullptr;
  SweepFn<T> step = nullptr;
  SweepFn<T> adam = nullptr;
  SweepFn<T> energy = nullptr;
};

struct Variant {
  int tx, ty, nt;
  int dtype_mask;   // bit 0: FE_F32, bit 1: FE_F64
  Kernels<float> k32;
  Kernels<double> k64;
  Kernels<float> k32sp;    // with a coefficient field (only some variants have them)
  Kernels<double> k64sp;
  SweepFn<float> k32box = nullptr;    // gradient with a box mask (padded, non-periodic fields)
  SweepFn<double> k64box = nullptr;
};

template <typename T, int TX, int TY, int NT, bool SP = false>
Kernels<T> make_kernels() {
  Kernels<T> k;
  k.grad = fe::grad_sweep<T, TX, TY, NT, fe::kGrad, SP>;
  k.step = fe::grad_sweep<T, TX, TY, NT, fe::kStepGD, SP>;
  k.adam = fe::grad_sweep<T, TX, TY, NT, fe::kStepAdam, SP>;
  k.energy = fe::energy_sweep<T, TX, TY, NT, SP>;
  return k;
}

// Static LDS of grad_sweep is (4 (TX+4)(TY+4) + 7 (TX+2)(TY+2)) sizeof(T) plus
// 16 bytes per wave; gfx950 allows up to 160 KiB per workgroup. The block size
// need not divide the tile (the last round of a thread may be idle).
const std::vector<Variant>& variants() {
  static const std::vector<Variant> v = [] {
    std::vector<Variant> r;
    auto add32 = [&](int tx, int ty, int nt, Kernels<float> k, Kernels<float> ksp = {},
                     SweepFn<float> kbox = nullptr) {
      Variant x{tx, ty, nt, 1, k, {}, ksp, {}, kbox, nullptr};
      r.push_back(x);
    };
    auto add64 = [&](int tx, int ty, int nt, Kernels<double> k, Kernels<double> ksp = {},
                     SweepFn<double> kbox = nullptr) {
      Variant x{tx, ty, nt, 2, {}, k, {}, ksp, nullptr, kbox};
      r.push_back(x);
    };
    // the coefficient-field kernels exist for one large, one small and the
    // smallest tile of each precision
    add32(64, 16, 512, make_kernels<float, 64, 16, 512>(), make_kernels<float, 64, 16, 512, true>(),
          fe::grad_sweep<float, 64, 16, 512, fe::kGrad, false, true>);
    add32(64, 32, 1024, make_kernels<float, 64, 32, 1024>());
    add32(32, 32, 512, make_kernels<float, 32, 32, 512>());
    add32(64, 32, 768, make_kernels<float, 64, 32, 768>());
    add32(64, 16, 1024, make_kernels<float, 64, 16, 1024>());
    add32(64, 8, 512, make_kernels<float, 64, 8, 512>());
    add32(32, 16, 512, make_kernels<float, 32, 16, 512>());
    add32(32, 8, 256, make_kernels<float, 32, 8, 256>(), make_kernels<float, 32, 8, 256, true>(),
          fe::grad_sweep<float, 32, 8, 256, fe::kGrad, false, true>);
    add32(16, 16, 256, make_kernels<float, 16, 16, 256>());
    add32(16, 8, 128, make_kernels<float, 16, 8, 128>());
    add32(8, 8, 64, make_kernels<float, 8, 8, 64>(), make_kernels<float, 8, 8, 64, true>(),
          fe::grad_sweep<float, 8, 8, 64, fe::kGrad, false, true>);
    add64(32, 16, 512, make_kernels<double, 32, 16, 512>(), make_kernels<double, 32, 16, 512, true>(),
          fe::grad_sweep<double, 32, 16, 512, fe::kGrad, false, true>);
    add64(32, 8, 256, make_kernels<double, 32, 8, 256>());
    add64(16, 16, 256, make_kernels<double, 16, 16, 256>());
    add64(16, 8, 128, make_kernels<double, 16, 8, 128>(), make_kernels<double, 16, 8, 128, true>(),
          fe::grad_sweep<double, 16, 8, 128, fe::kGrad, false, true>);
    add64(8, 8, 64, make_kernels<double, 8, 8, 64>(), make_kernels<double, 8, 8, 64, true>(),
          fe::grad_sweep<double, 8, 8, 64, fe::kGrad, false, true>);
    return r;
  }();
  return v;
}

template <typename T>
const Kernels<T>& kernels_of(const Variant& v, bool sp = false);
template <>
const Kernels<float>& kernels_of<float>(const Variant& v, bool sp) { return sp ? v.k32sp : v.k32; }
template <>
const Kernels<double>& kernels_of<double>(const Variant& v, bool sp) { return sp ? v.k64sp : v.k64; }
template <typename T>
SweepFn<T> box_kernel_of(const Variant& v);
template <>
SweepFn<float> box_kernel_of<float>(const Variant& v) { return v.k32box; }
template <>
SweepFn<double> box_kernel_of<double>(const Variant& v) { return v.k64box; }

int ceil_div(int a, int b) { return (a + b - 1) / b; }

}  // namespace

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------

// Step-rule hyper-parameters (baked into captured graphs).
struct StepRule {
  int mode;        // fe::kStepGD or fe::kStepAdam
  double tau;      // GD step size or Adam learning rate
  double beta1, beta2, adam_eps;
};

struct GraphKey {
  void* u;                      // the field (or vector field) the graph updates in place
  int mode;                     // fe::SweepMode of a step loop, or kFlowMode
  double tau, beta1, beta2, adam_eps, sigma;
  int pairs;                    // step pairs (or flow iterations) per graph
  int variant;
  int lz;
  int fields;                   // bit 0: coefficient field in use, bit 1: mass field in use
  bool operator<(const GraphKey& o) const {
    return std::tie(u, mode, tau, beta1, beta2, adam_eps, sigma, pairs, variant, lz, fields) <
           std::tie(o.u, o.mode, o.tau, o.beta1, o.beta2, o.adam_eps, o.sigma, o.pairs, o.variant, o.lz,
                    o.fields);
  }
};
constexpr int kFlowMode = 100;

struct fe_ctx {
  fe_grid grid{};
  int device = 0;
  hipStream_t stream = nullptr;       // caller's stream (may be null = default)
  hipStream_t cap_stream = nullptr;   // private stream used only to capture graphs
  std::vector<double> eps, coeffs;    // host copies [batch], [batch][6]
  std::vector<double> mu, theta;      // orientation term [batch], [batch][3] (mu = 0: off)
  void* d_prm = nullptr;              // InstParams<T>[batch]
  double* d_partials = nullptr;       // [batch][max_blocks][2]
  int* d_counters = nullptr;          // [batch + 1] finished-block counters (zero between launches)
  double* d_energy = nullptr;         // [batch]
  double* d_mass = nullptr;           // [batch]
  double* d_shift = nullptr;          // [2][batch]
  void* d_pingpong = nullptr;         // one field, allocated by the first fe_step
  void* d_m1 = nullptr;               // Adam moments, allocated by the first fe_step_adam
  void* d_m2 = nullptr;
  int* d_adam_t = nullptr;            // Adam step number (device)
  void* d_w0 = nullptr;               // H^-1 flow: two scalar work fields
  void* d_w1 = nullptr;
  void* d_am1 = nullptr;              // H^-1 flow: Adam moments of A ([batch][3] fields each)
  void* d_am2 = nullptr;
  fe::FlowClock* d_flow_clk = nullptr; // H^-1 flow: Adam step number and bias corrections (device)
  double* d_diag = nullptr;           // diagnostics: per-instance constants, stats, block partials
  size_t diag_bytes = 0;
  void* d_cfield = nullptr;           // scaled coefficient field [batch][6][nz][ny][nx] (Sec. 5.2)
  bool use_cfield = false;
  void* d_mfield = nullptr;           // mass field m(x) [batch][nz][ny][nx] of the flow (Sec. 5.2)
  bool use_mfield = false;
  bool use_box = false;               // padded non-periodic field: density only inside the box
  int box_lo[3] = {0, 0, 0}, box_hi[3] = {0, 0, 0};
  size_t max_blocks = 0;              // per instance, over all variants and z chunks
  int variant = -1;
  int lz = 0;                         // 0 = automatic
  int num_cu = 256;                   // compute units of the device
  std::map<GraphKey, hipGraphExec_t> graphs;
};

namespace {

size_t elem_size(const fe_grid& g) { return g.dtype == FE_F64 ? 8 : 4; }
size_t field_elems(const fe_grid& g) { return (size_t)g.nx * g.ny * g.nz * g.batch; }

int check_grid(const fe_grid* g) {
  if (!g) return set_error(FE_EINVAL, "grid is NULL");
  if (g->nx < 1 || g->ny < 1 || g->nz < 1)
    return set_error(FE_EINVAL, "grid sizes must be >= 1 (got %d x %d x %d)", g->nx, g->ny, g->nz);
  if (g->batch < 1) return set_error(FE_EINVAL, "batch must be >= 1 (got %d)", g->batch);
  if (!(g->h > 0.0) || !std::isfinite(g->h)) return set_error(FE_EINVAL, "h must be finite and > 0");
  if (g->dtype != FE_F32 && g->dtype != FE_F64) return set_error(FE_EINVAL, "dtype must be FE_F32 or FE_F64");
  const double n = (double)g->nx * g->ny * g->nz;
  if (n * g->batch > 4.0e9 || (double)g->nx * g->ny > 2.0e9)
    return set_error(FE_EINVAL, "grid too large for 32-bit plane indexing");
  return FE_OK;
}

int check_params(int batch, const double* eps, const double* a) {
  if (!eps || !a) return set_error(FE_EINVAL, "eps and p_coeffs must not be NULL");
  for (int b = 0; b < batch; ++b) {
    if (!(eps[b] > 0.0) || !std::isfinite(eps[b]))
      return set_error(FE_EINVAL, "eps[%d] must be finite and > 0", b);
    for (int i = 0; i < 6; ++i)
      if (!std::isfinite(a[6 * b + i])) return set_error(FE_EINVAL, "p_coeffs[%d][%d] is not finite", b, i);
  }
  return FE_OK;
}

// Per-instance constants: c1..c6 of eq. (Feps) folded with the unit scales of
// the raw-difference formulation (s = eps/h^2, 1/(2h), h^3, eps/(4h^2)).
template <typename T>
void fill_params(const fe_ctx* c, std::vector<fe::InstParams<T>>& out) {
  const double h = c->grid.h, h3 = h * h * h;
  out.resize(c->grid.batch);
  for (int b = 0; b < c->grid.batch; ++b) {
    const double e = c->eps[b];
    const double* a = &c->coeffs[6 * b];
    const double a20 = a[0], a11 = a[1], a02 = a[2], a10 = a[3], a01 = a[4], a00 = a[5];
    const double c1 = (a20 + a02 - a11) / (2.0 * e), c2 = a11 / (2.0 * e), c3 = (a20 - a02) / (2.0 * e);
    const double c4 = (a10 + a01) / 2.0, c5 = (a10 - a01) / 2.0, c6 = a00;
    const double sc = e / (h * h);
    fe::InstParams<T>& p = out[b];
    p.lam_d = 1.0 / (e * sc);
    p.lam = T(p.lam_d);
    p.C1 = T(h3 * c1 * sc * sc);
    p.C2 = T(h3 * c2 * sc * sc);
    p.C3 = T(h3 * c3 * sc * sc);
    p.C4 = T(h3 * c4 * sc / (2.0 * h));
    p.C5 = T(h3 * c5 * sc / (2.0 * h));
    p.C6 = T(h3 * c6 * e / (4.0 * h * h));
    p.xi = T(kXi / (sc * sc));
    p.inv_xi = T(sc * sc / kXi);
    p.Co = T(h3 * e * c->mu[b] / (4.0 * h * h));
    p.thx = T(c->theta[3 * b]);
    p.thy = T(c->theta[3 * b + 1]);
    p.thz = T(c->theta[3 * b + 2]);
  }
}

template <typename T>
fe::GridConsts<T> grid_consts(double h) {
  fe::GridConsts<T> k;
  k.reg_d = 4.0 * h * h * kXi * kXi;
  k.reg = T(k.reg_d);
  return k;
}

int upload_params(fe_ctx* c) {
  if (c->grid.dtype == FE_F32) {
    std::vector<fe::InstParams<float>> p;
    fill_params(c, p);
    FE_HIP(hipMemcpyAsync(c->d_prm, p.data(), p.size() * sizeof(p[0]), hipMemcpyHostToDevice, c->stream));
  } else {
    std::vector<fe::InstParams<double>> p;
    fill_params(c, p);
    FE_HIP(hipMemcpyAsync(c->d_prm, p.data(), p.size() * sizeof(p[0]), hipMemcpyHostToDevice, c->stream));
  }
  // the host vectors die here: make sure the copies have consumed them
  FE_HIP(hipStreamSynchronize(c->stream));
  return FE_OK;
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
    else prev = -1;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

bool variant_ok(int v, int dtype) {
  if (v < 0 || v >= (int)variants().size()) return false;
  return variants()[v].dtype_mask & (dtype == FE_F64 ? 2 : 1);
}

// Launch geometry of the chosen variant.
struct Geometry {
  int ntx, nty, nzc, lz, per_inst;
};

// Blocks of the step sweep of `variant` that one compute unit holds at once.
int block_slots(const fe_ctx* c, int variant) {
  const Variant& v = variants()[variant];
  const void* fn = c->grid.dtype == FE_F32 ? (const void*)v.k32.step : (const void*)v.k64.step;
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, v.nt, 0) != hipSuccess || n < 1) n = 1;
  return n;
}

Geometry geometry(const fe_ctx* c, int variant, int lz_req) {
  const Variant& v = variants()[variant];
  Geometry g;
  g.ntx = ceil_div(c->grid.nx, v.tx);
  g.nty = ceil_div(c->grid.ny, v.ty);
  int lz = lz_req;
  if (lz <= 0) {
    // the longest power-of-two chunk (fewest recomputed boundary planes) that
    // still fills every resident block slot of the device, and at least 4 planes
    const double cols = (double)g.ntx * g.nty * c->grid.batch;
    const double slots = (double)c->num_cu * block_slots(c, variant);
    lz = 4;
    while (2 * lz <= c->grid.nz && cols * ceil_div(c->grid.nz, 2 * lz) >= slots) lz *= 2;
  }
  lz = std::min(std::max(lz, 1), c->grid.nz);
  g.lz = lz;
  g.nzc = ceil_div(c->grid.nz, lz);
  g.per_inst = g.ntx * g.nty * g.nzc;
  return g;
}

bool has_sp(int v, int dtype) {
  const Variant& x = variants()[v];
  return dtype == FE_F32 ? x.k32sp.grad != nullptr : x.k64sp.grad != nullptr;
}

bool has_box(int v, int dtype) {
  const Variant& x = variants()[v];
  return dtype == FE_F32 ? x.k32box != nullptr : x.k64box != nullptr;
}

// The variant a sweep launches: the chosen one, unless a coefficient field is
// in use and that variant has no coefficient-field kernels; then the first
// one that has them and whose tile the grid fills.
int sweep_variant(const fe_ctx* c) {
  auto ok = [&](int v) {
    return (!c->use_cfield || has_sp(v, c->grid.dtype)) && (!c->use_box || has_box(v, c->grid.dtype));
  };
  if (ok(c->variant)) return c->variant;
  int last = c->variant;
  for (int v = 0; v < (int)variants().size(); ++v) {
    if (!variant_ok(v, c->grid.dtype) || !ok(v)) continue;
    const Variant& x = variants()[v];
    if (x.tx <= std::max(c->grid.nx, 8) && x.ty <= std::max(c->grid.ny, 8)) return v;
    last = v;
  }
  return last;
}

int fields_in_use(const fe_ctx* c) { return (c->use_cfield ? 1 : 0) | (c->use_mfield ? 2 : 0); }

int default_variant(const fe_grid& g) {
  const int dt = g.dtype;
  // variants are listed best-first for large grids: take the first whose tile
  // the grid fills
  for (int v = 0; v < (int)variants().size(); ++v) {
    if (!variant_ok(v, dt)) continue;
    const Variant& x = variants()[v];
    if (x.tx <= std::max(g.nx, 8) && x.ty <= std::max(g.ny, 8)) return v;
  }
  for (int v = (int)variants().size() - 1; v >= 0; --v)
    if (variant_ok(v, dt)) return v;
  return 0;
}

// kind: -1 energy only, else a fe::SweepMode. One launch computes the sweep and
// its per-instance sums: energy_dev[b] and, for steps, shift_out[b].
template <typename T>
int launch_sweep(fe_ctx* c, hipStream_t s, int kind, const void* src, void* dst, const double* shift_in,
                 double* shift_out, double* energy_dev, const StepRule& rule) {
  const int vi = sweep_variant(c);
  const Geometry geo = geometry(c, vi, c->lz);
  if ((size_t)geo.per_inst > c->max_blocks) return set_error(FE_EINVAL, "internal: partials workspace too small");
  const Variant& v = variants()[vi];
  const Kernels<T>& k = kernels_of<T>(v, c->use_cfield);
  fe::SweepArgs<T> a;
  a.src = static_cast<const T*>(src);
  a.dst = static_cast<T*>(dst);
  a.prm = static_cast<const fe::InstParams<T>*>(c->d_prm);
  a.shift_in = shift_in;
  a.partials = c->d_partials;
  a.counters = c->d_counters;
  a.energy = energy_dev;
  a.mass = c->d_mass;
  a.shift_out = shift_out;
  a.inv_nvox = 1.0 / ((double)c->grid.nx * c->grid.ny * c->grid.nz);
  a.k = grid_consts<T>(c->grid.h);
  a.m1 = static_cast<T*>(c->d_m1);
  a.m2 = static_cast<T*>(c->d_m2);
  a.adam_t = c->d_adam_t;
  a.cfield = c->use_cfield ? static_cast<const T*>(c->d_cfield) : nullptr;
  a.tau = T(rule.tau);
  a.beta1 = T(rule.beta1);
  a.beta2 = T(rule.beta2);
  a.adam_eps = T(rule.adam_eps);
  a.nx = c->grid.nx;
  a.ny = c->grid.ny;
  a.nz = c->grid.nz;
  a.ntx = geo.ntx;
  a.nty = geo.nty;
  a.nzc = geo.nzc;
  a.lz = geo.lz;
  a.batch = c->grid.batch;
  const dim3 grid((unsigned)(geo.per_inst * c->grid.batch));
  const dim3 block((unsigned)v.nt);
  SweepFn<T> fn = kind < 0 ? k.energy
                 : kind == fe::kGrad ? k.grad
                 : kind == fe::kStepGD ? k.step : k.adam;
  if (c->use_box) {
    if (kind != fe::kGrad || c->use_cfield) return set_error(FE_EINVAL, "internal: box sweeps are gradient-only");
    fn = box_kernel_of<T>(v);
    for (int i = 0; i < 3; ++i) {
      a.box_lo[i] = c->box_lo[i];
      a.box_hi[i] = c->box_hi[i];
    }
  }
  hipLaunchKernelGGL(fn, grid, block, 0, s, a);
  FE_HIP(hipGetLastError());
  return FE_OK;
}

int sweep(fe_ctx* c, hipStream_t s, int kind, const void* src, void* dst, const double* shift_in,
          double* shift_out, double* energy_dev, const StepRule& rule) {
  return c->grid.dtype == FE_F32
             ? launch_sweep<float>(c, s, kind, src, dst, shift_in, shift_out, energy_dev, rule)
             : launch_sweep<double>(c, s, kind, src, dst, shift_in, shift_out, energy_dev, rule);
}

int copy_energy_out(fe_ctx* c, double* energy) {
  if (!energy) return FE_OK;
  FE_HIP(hipMemcpyAsync(energy, c->d_energy, sizeof(double) * c->grid.batch, hipMemcpyDeviceToHost, c->stream));
  FE_HIP(hipStreamSynchronize(c->stream));
  for (int b = 0; b < c->grid.batch; ++b)
    if (!std::isfinite(energy[b])) return set_error(FE_ENONFINITE, "energy[%d] is not finite", b);
  return FE_OK;
}

void drop_graphs(fe_ctx* c) {
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  c->graphs.clear();
}

// One descent step: src (+ shift_in) -> dst, then shift_out = mass - mean(dst).
int step_once(fe_ctx* c, hipStream_t s, const void* src, void* dst, const double* shift_in, double* shift_out,
              const StepRule& rule) {
  return sweep(c, s, rule.mode, src, dst, shift_in, shift_out, c->d_energy, rule);
}

int adam_reset_launch(fe_ctx* c) {
  const size_t n = field_elems(c->grid);
  const int nblk = (int)std::min<size_t>((n + 255) / 256, 65536);
  if (c->grid.dtype == FE_F32)
    hipLaunchKernelGGL(fe::adam_reset<float>, dim3(nblk), dim3(256), 0, c->stream, (float*)c->d_m1,
                       (float*)c->d_m2, n, c->d_adam_t);
  else
    hipLaunchKernelGGL(fe::adam_reset<double>, dim3(nblk), dim3(256), 0, c->stream, (double*)c->d_m1,
                       (double*)c->d_m2, n, c->d_adam_t);
  FE_HIP(hipGetLastError());
  return FE_OK;
}

int run_steps(fe_ctx* c, void* u, const double* mass, const StepRule& rule, int nsteps, double* energy);

// ---- H^-1 flow (Algorithm 1) ---------------------------------------------

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
dim3 row_grid(const fe::FieldDims& d) { return dim3(ceil_div(d.nx, 64), ceil_div(d.ny, 4), d.nz * d.batch); }
dim3 x_grid(const fe::FieldDims& d) { return dim3(ceil_div(d.nx, 64), ceil_div(d.ny, fe::kBlurRows), d.nz * d.batch); }
dim3 axis_grid(const fe::FieldDims& d, int axis) {
  return axis == 1 ? dim3(ceil_div(d.nx, 64), ceil_div(d.ny, fe::kAxisChunk), ceil_div(d.nz, 4) * d.batch)
                   : dim3(ceil_div(d.nx, 64), ceil_div(d.nz, fe::kAxisChunk), ceil_div(d.ny, 4) * d.batch);
}

// The x pass (with the divergence when DIV), dispatched to the fixed-radius
// instantiation when there is one.
template <typename T, bool DIV>
void blur_x_pass(hipStream_t s, const fe::FieldDims& d, const fe::BlurTaps<T>& k, const T* in, T* out,
                 const double* m0, const T* mfield, T inv2h, fe::FlowClock* clk, double beta1, double beta2) {
  const dim3 g = x_grid(d), b(64, 4);
  if (k.r == 4)
    hipLaunchKernelGGL((fe::blur_x<T, DIV, 4>), g, b, 0, s, in, out, m0, mfield, d, inv2h, k, clk, beta1, beta2);
  else if (k.r == 8)
    hipLaunchKernelGGL((fe::blur_x<T, DIV, 8>), g, b, 0, s, in, out, m0, mfield, d, inv2h, k, clk, beta1, beta2);
  else
    hipLaunchKernelGGL((fe::blur_x<T, DIV>), g, b, 0, s, in, out, m0, mfield, d, inv2h, k, clk, beta1, beta2);
}

template <typename T, int AXIS>
void blur_axis_pass(hipStream_t s, const fe::FieldDims& d, const fe::BlurTaps<T>& k, const T* in, T* out) {
  const dim3 g = axis_grid(d, AXIS), b(64, 4);
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
// flow clock (iterations only).
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

// One iteration of Algorithm 1 on A (in place), energies into d_energy.
template <typename T>
int flow_iteration(fe_ctx* c, hipStream_t s, void* A, const FlowRule& fr) {
  T* w0 = static_cast<T*>(c->d_w0);
  T* w1 = static_cast<T*>(c->d_w1);
  const fe::FieldDims d{c->grid.nx, c->grid.ny, c->grid.nz, c->grid.batch};
  const fe::BlurTaps<T> k = blur_taps<T>(fr.sigma_k);
  // ub = k * (div A + m0) in w0
  int rc = flow_field<T>(c, s, A, w0, fr.sigma_k, c->d_flow_clk, fr.beta1, fr.beta2);
  if (rc) return rc;
  // gb = dF/du at ub, in w1 (energy of ub into d_energy)
  const StepRule none{fe::kGrad, 0.0, 0.0, 0.0, 0.0};
  rc = sweep(c, s, fe::kGrad, w0, w1, nullptr, nullptr, c->d_energy, none);
  if (rc) return rc;
  // gu = k * gb: x pass into w0, y pass into w1, z pass into w0
  T* gu = w1;
  if (k.r > 0) {
    blur_x_pass<T, false>(s, d, k, (const T*)w1, w0, nullptr, nullptr, T(0), nullptr, 0.0, 0.0);
    blur_yz<T>(s, d, k, w0, w1, w0);
    gu = w0;
  }
  hipLaunchKernelGGL(fe::adam_vector_field<T>, row_grid(d), dim3(64, 4), 0, s, (const T*)gu, (T*)A,
                     (T*)c->d_am1, (T*)c->d_am2, d, T(1.0 / (2.0 * c->grid.h)), T(fr.lr), T(fr.beta1),
                     T(fr.beta2), T(fr.adam_eps), (const fe::FlowClock*)c->d_flow_clk);
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

// The diagnostics sweep: one tile shape for both precisions, z chunks of up to 32.
constexpr int kDiagTX = 64, kDiagTY = 8, kDiagNT = 512, kDiagLZ = 32;

template <typename T>
int diagnostics(fe_ctx* c, const void* u, void* curv, double* hist, int nbins, double kmax, double* stats) {
  const int B = c->grid.batch;
  const int ntx = ceil_div(c->grid.nx, kDiagTX), nty = ceil_div(c->grid.ny, kDiagTY);
  // the longest z chunk (fewest recomputed halo planes) that still gives every
  // compute unit two blocks
  int lz = kDiagLZ;
  while (lz > 4 && (double)ntx * nty * ceil_div(c->grid.nz, lz) * B < 2.0 * c->num_cu) lz /= 2;
  lz = std::min(lz, c->grid.nz);
  const int nzc = ceil_div(c->grid.nz, lz);
  const size_t per_inst = (size_t)ntx * nty * nzc;
  // layout of d_diag: DiagInst[B] | stats[B][5] | partials[B][per_inst][5]
  const size_t need = sizeof(fe::DiagInst) * B + sizeof(double) * fe::kDiagStats * B * (1 + per_inst);
  if (c->diag_bytes < need) {
    if (c->d_diag) (void)hipFree(c->d_diag);
    c->d_diag = nullptr;
    c->diag_bytes = 0;
    if (hipMalloc((void**)&c->d_diag, need) != hipSuccess) {
      c->d_diag = nullptr;
      return set_error(FE_ENOMEM, "diagnostics workspace allocation failed");
    }
    c->diag_bytes = need;
  }
  const double h = c->grid.h;
  std::vector<fe::DiagInst> di(B);
  for (int b = 0; b < B; ++b) {
    const double eps = c->eps[b];
    di[b] = fe::DiagInst{eps * h / 8.0, h * h * h / (4.0 * eps), eps * h / 4.0};
  }
  fe::DiagInst* d_inst = reinterpret_cast<fe::DiagInst*>(c->d_diag);
  double* d_stats = reinterpret_cast<double*>(d_inst + B);
  double* d_part = d_stats + (size_t)fe::kDiagStats * B;
  FE_HIP(hipMemcpyAsync(d_inst, di.data(), sizeof(fe::DiagInst) * B, hipMemcpyHostToDevice, c->stream));
  if (hist) {
    const int n = B * nbins * nbins;
    hipLaunchKernelGGL(fe::fill_f64, dim3(ceil_div(n, 64)), dim3(64), 0, c->stream, hist, n, 0.0);
  }
  fe::SweepArgs<T> a{};
  a.src = static_cast<const T*>(u);
  a.prm = static_cast<const fe::InstParams<T>*>(c->d_prm);
  a.cfield = c->use_cfield ? static_cast<const T*>(c->d_cfield) : nullptr;
  a.k = grid_consts<T>(h);
  a.nx = c->grid.nx;
  a.ny = c->grid.ny;
  a.nz = c->grid.nz;
  a.ntx = ntx;
  a.nty = nty;
  a.nzc = nzc;
  a.lz = lz;
  a.batch = B;
  fe::DiagArgs<T> d{};
  d.inst = d_inst;
  d.curv = static_cast<T*>(curv);
  d.hist = hist;
  d.partials = d_part;
  d.nbins = hist ? nbins : 0;
  d.kmax = T(kmax);
  d.bin_scale = T(hist ? nbins / (2.0 * kmax) : 0.0);
  d.inv_h = T(1.0 / h);
  d.inv_h2 = T(1.0 / (h * h));
  hipLaunchKernelGGL((fe::diag_sweep<T, kDiagTX, kDiagTY, kDiagNT>), dim3((unsigned)(per_inst * B)),
                     dim3(kDiagNT), 0, c->stream, a, d);
  hipLaunchKernelGGL(fe::diag_finish, dim3(B), dim3(256), 0, c->stream, (const double*)d_part, (int)per_inst,
                     d_stats);
  FE_HIP(hipGetLastError());
  if (stats) {
    FE_HIP(hipMemcpyAsync(stats, d_stats, sizeof(double) * fe::kDiagStats * B, hipMemcpyDeviceToHost, c->stream));
    FE_HIP(hipStreamSynchronize(c->stream));
  }
  return FE_OK;
}

int run_steps(fe_ctx* c, void* u, const double* mass, const StepRule& rule, int nsteps, double* energy) {
  if (!u) return set_error(FE_EINVAL, "u is NULL");
  if (!mass) return set_error(FE_EINVAL, "mass is NULL");
  if (nsteps < 0) return set_error(FE_EINVAL, "nsteps must be >= 0");
  for (int b = 0; b < c->grid.batch; ++b)
    if (!std::isfinite(mass[b])) return set_error(FE_EINVAL, "mass[%d] is not finite", b);
  if (nsteps == 0) return FE_OK;
  DeviceGuard dg(c->device);
  const int B = c->grid.batch;
  if (!c->d_pingpong) {
    if (hipMalloc(&c->d_pingpong, field_elems(c->grid) * elem_size(c->grid)) != hipSuccess) {
      c->d_pingpong = nullptr;
      return set_error(FE_ENOMEM, "ping-pong field allocation failed");
    }
  }
  FE_HIP(hipMemcpyAsync(c->d_mass, mass, sizeof(double) * B, hipMemcpyHostToDevice, c->stream));
  double* s0 = c->d_shift;        // shift of the ping-pong field
  double* s1 = c->d_shift + B;    // shift of u
  hipLaunchKernelGGL(fe::fill_f64, dim3(ceil_div(B, 64)), dim3(64), 0, c->stream, s1, B, 0.0);
  FE_HIP(hipGetLastError());
  void* A = c->d_pingpong;

  // pairs of steps u -> A -> u: whole blocks of kGraphPairs pairs are replayed
  // from one captured graph (the same graph for any nsteps), the rest launch
  // directly
  const int npairs = nsteps / 2;
  const int gpairs = npairs >= kGraphPairs ? kGraphPairs : 0;
  for (int i = 0; i < (gpairs ? npairs % gpairs : npairs); ++i) {
    int rc = step_once(c, c->stream, u, A, s1, s0, rule);
    if (rc == FE_OK) rc = step_once(c, c->stream, A, u, s0, s1, rule);
    if (rc) return rc;
  }
  if (gpairs > 0) {
    GraphKey key{u,      rule.mode,           rule.tau, rule.beta1,     rule.beta2, rule.adam_eps, 0.0,
                 gpairs, sweep_variant(c), c->lz,    fields_in_use(c)};
    auto it = c->graphs.find(key);
    hipGraphExec_t exec = nullptr;
    if (it == c->graphs.end()) {
      hipGraph_t graph = nullptr;
      FE_HIP(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
      int rc = FE_OK;
      for (int i = 0; i < gpairs && rc == FE_OK; ++i) {
        rc = step_once(c, c->cap_stream, u, A, s1, s0, rule);
        if (rc == FE_OK) rc = step_once(c, c->cap_stream, A, u, s0, s1, rule);
      }
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
    for (int r = 0; r < npairs / gpairs; ++r) FE_HIP(hipGraphLaunch(exec, c->stream));
  }
  const size_t per_inst = (size_t)c->grid.nx * c->grid.ny * c->grid.nz;
  const int nblk = (int)std::min<size_t>((field_elems(c->grid) + 255) / 256, 65536);
  const void* last = u;
  const double* shift = s1;
  if (nsteps % 2) {
    int rc = step_once(c, c->stream, u, A, s1, s0, rule);
    if (rc) return rc;
    last = A;
    shift = s0;
  }
  if (c->grid.dtype == FE_F32)
    hipLaunchKernelGGL(fe::add_shift<float>, dim3(nblk), dim3(256), 0, c->stream, (const float*)last, (float*)u,
                       shift, per_inst, B);
  else
    hipLaunchKernelGGL(fe::add_shift<double>, dim3(nblk), dim3(256), 0, c->stream, (const double*)last,
                       (double*)u, shift, per_inst, B);
  FE_HIP(hipGetLastError());
  return copy_energy_out(c, energy);
}


// ---------------------------------------------------------------------------
// Algorithm 2: the L2 flow with replicate boundaries and L-BFGS
// ---------------------------------------------------------------------------

}  // namespace

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

// Scalar slots after the partials in d_red: 0 energy, 1 max|g|, 2 max|d|, 3 g'd,
// 4 |g|_1, 5 y's, 6 y'y, 7 scratch dot, 8.. the s_i'q dots of the two-loop
// recursion (one per history entry).
constexpr int kSlotE = 0, kSlotGmax = 1, kSlotDmax = 2, kSlotGtd = 3, kSlotL1 = 4, kSlotYs = 5, kSlotYy = 6,
              kSlotDot = 7, kSlotAlpha = 8;
constexpr int kL2MaxHistory = 64;
constexpr int kL2Slots = kSlotAlpha + kL2MaxHistory;

// Reduction of a (and b) into scalar slot `slot`, stream-ordered, no sync.
template <typename T>
int l2_reduce_dev(fe_l2* L, int op, const void* a, const void* b, int slot) {
  hipStream_t s = L->ctx->stream;
  const T* pa = static_cast<const T*>(a);
  const T* pb = static_cast<const T*>(b);
  double* part = L->d_red;
  double* res = L->d_red + fe::kVecBlocks + slot;
  if (op == 0)
    hipLaunchKernelGGL((fe::vec_reduce<T, 0>), dim3(fe::kVecBlocks), dim3(256), 0, s, pa, pb, L->n, part);
  else if (op == 1)
    hipLaunchKernelGGL((fe::vec_reduce<T, 1>), dim3(fe::kVecBlocks), dim3(256), 0, s, pa, pb, L->n, part);
  else
    hipLaunchKernelGGL((fe::vec_reduce<T, 2>), dim3(fe::kVecBlocks), dim3(256), 0, s, pa, pb, L->n, part);
  if (op == 2)
    hipLaunchKernelGGL(fe::vec_finish<2>, dim3(1), dim3(256), 0, s, (const double*)part, fe::kVecBlocks, res);
  else
    hipLaunchKernelGGL(fe::vec_finish<0>, dim3(1), dim3(256), 0, s, (const double*)part, fe::kVecBlocks, res);
  FE_HIP(hipGetLastError());
  return FE_OK;
}

// Host copies of scalar slots [first, first + count) (one sync).
int l2_read_slots(fe_l2* L, int first, int count, double* out) {
  FE_HIP(hipMemcpyAsync(out, L->d_red + fe::kVecBlocks + first, sizeof(double) * count, hipMemcpyDeviceToHost,
                        L->ctx->stream));
  FE_HIP(hipStreamSynchronize(L->ctx->stream));
  return FE_OK;
}

// y += (ka sc[ia] + kb sc[ib]) x with device scalars
template <typename T>
int l2_axpy_dev(fe_l2* L, int ia, double ka, int ib, double kb, const void* x, void* y) {
  hipLaunchKernelGGL(fe::vec_axpy_dev<T>, dim3(l2_launch_1d(L->n)), dim3(256), 0, L->ctx->stream,
                     (const double*)(L->d_red + fe::kVecBlocks), ia, ka, ib, kb, static_cast<const T*>(x),
                     static_cast<T*>(y), L->n);
  FE_HIP(hipGetLastError());
  return FE_OK;
}

// y = alpha x + beta y
template <typename T>
int l2_axpby(fe_l2* L, double alpha, const void* x, double beta, void* y) {
  hipLaunchKernelGGL(fe::vec_axpby<T>, dim3(l2_launch_1d(L->n)), dim3(256), 0, L->ctx->stream, T(alpha),
                     static_cast<const T*>(x), T(beta), static_cast<T*>(y), L->n);
  FE_HIP(hipGetLastError());
  return FE_OK;
}

template <typename T>
int l2_copy(fe_l2* L, const void* src, void* dst) {
  FE_HIP(hipMemcpyAsync(dst, src, L->n * sizeof(T), hipMemcpyDeviceToDevice, L->ctx->stream));
  return FE_OK;
}

// The three separable blur passes on the padded array (periodic within it):
// in -> tmp1 (x) -> tmp2 (y) -> out (z); in and out may coincide, tmp1/tmp2 not.
template <typename T>
void l2_blur(fe_l2* L, const T* in, T* tmp1, T* tmp2, T* out) {
  const fe::FieldDims d{L->box.nx, L->box.ny, L->box.nz, 1};
  const fe::BlurTaps<T> k = blur_taps<T>(L->sigma_k);
  hipStream_t s = L->ctx->stream;
  blur_x_pass<T, false>(s, d, k, in, tmp1, nullptr, nullptr, T(0), nullptr, 0.0, 0.0);
  blur_yz<T>(s, d, k, tmp1, tmp2, out);
}

// F_h(k * x) with replicate boundaries into the energy slot and g = its
// gradient (zero padding), stream-ordered.
template <typename T>
int l2_eval_dev(fe_l2* L) {
  hipStream_t s = L->ctx->stream;
  const int nb = l2_launch_1d(L->n);
  T* x = static_cast<T*>(L->x);
  T* g = static_cast<T*>(L->g);
  T* w0 = static_cast<T*>(L->w0);
  T* w1 = static_cast<T*>(L->w1);
  T* w2 = static_cast<T*>(L->w2);
  hipLaunchKernelGGL(fe::pad_replicate<T>, dim3(nb), dim3(256), 0, s, x, L->box);
  const T* ub = x;
  if (L->r > 0) {
    l2_blur<T>(L, x, w0, w1, w2);             // w2 = k * x
    hipLaunchKernelGGL(fe::pad_replicate<T>, dim3(nb), dim3(256), 0, s, w2, L->box);
    ub = w2;
  }
  const StepRule none{fe::kGrad, 0.0, 0.0, 0.0, 0.0};
  int rc = sweep(L->ctx, s, fe::kGrad, ub, w0, nullptr, nullptr, L->ctx->d_energy, none);   // w0 = g_ext
  if (rc) return rc;
  if (L->r > 0) {
    hipLaunchKernelGGL(fe::fold_pads<T>, dim3(nb), dim3(256), 0, s, (const T*)w0, w1, L->box);   // w1 = gb
    l2_blur<T>(L, w1, w0, w2, w1);           // w1 = k * gb (zero-extended)
    hipLaunchKernelGGL(fe::fold_pads<T>, dim3(nb), dim3(256), 0, s, (const T*)w1, g, L->box);
  } else {
    hipLaunchKernelGGL(fe::fold_pads<T>, dim3(nb), dim3(256), 0, s, (const T*)w0, g, L->box);
  }
  FE_HIP(hipGetLastError());
  FE_HIP(hipMemcpyAsync(L->d_red + fe::kVecBlocks + kSlotE, L->ctx->d_energy, sizeof(double),
                        hipMemcpyDeviceToDevice, s));
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
      if ((rc = l2_axpby<T>(L, -1.0, L->g, 0.0, L->d))) return rc;
      L->hist_len = 0;
      L->rho.clear();
      L->H_diag = 1.0;
    } else {
      // y = g - prev_g (in q), s = t d (in w0); accept the pair if y's > 1e-10
      hipLaunchKernelGGL(fe::vec_sub<T>, dim3(l2_launch_1d(L->n)), dim3(256), 0, L->ctx->stream,
                         static_cast<const T*>(L->g), static_cast<const T*>(L->prev_g), static_cast<T*>(L->q), L->n);
      FE_HIP(hipGetLastError());
      if ((rc = l2_axpby<T>(L, L->t, L->d, 0.0, L->w0))) return rc;
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
        if ((rc = l2_copy<T>(L, L->q, L->Y[L->hist_len]))) return rc;
        if ((rc = l2_copy<T>(L, L->w0, L->S[L->hist_len]))) return rc;
        L->rho.push_back(1.0 / ys);
        ++L->hist_len;
        L->H_diag = ys / yy;
      }
      // two-loop recursion: q = -g; newest to oldest: a_i = rho_i s_i'q, q -= a_i y_i;
      // d = H_diag q; oldest to newest: b_i = rho_i y_i'd, d += (a_i - b_i) s_i
      if ((rc = l2_axpby<T>(L, -1.0, L->g, 0.0, L->q))) return rc;
      for (int i = L->hist_len - 1; i >= 0; --i) {
        if ((rc = l2_reduce_dev<T>(L, 0, L->S[i], L->q, kSlotAlpha + i))) return rc;
        if ((rc = l2_axpy_dev<T>(L, kSlotAlpha + i, -L->rho[i], -1, 0.0, L->Y[i], L->q))) return rc;
      }
      if ((rc = l2_axpby<T>(L, L->H_diag, L->q, 0.0, L->d))) return rc;
      for (int i = 0; i < L->hist_len; ++i) {
        if ((rc = l2_reduce_dev<T>(L, 0, L->Y[i], L->d, kSlotDot))) return rc;
        if ((rc = l2_axpy_dev<T>(L, kSlotAlpha + i, L->rho[i], kSlotDot, -L->rho[i], L->S[i], L->d))) return rc;
      }
    }
    if ((rc = l2_copy<T>(L, L->g, L->prev_g))) return rc;
    L->prev_loss = loss;
    const bool first = L->n_iter == 1;
    if ((rc = l2_reduce_dev<T>(L, 0, L->g, L->d, kSlotGtd))) return rc;
    if (first && (rc = l2_reduce_dev<T>(L, 1, L->g, nullptr, kSlotL1))) return rc;
    double gl[2];
    if ((rc = l2_read_slots(L, kSlotGtd, first ? 2 : 1, gl))) return rc;
    L->t = first ? std::min(1.0, 1.0 / gl[1]) * L->lr : L->lr;
    const double gtd = gl[0];
    if (gtd > -L->tol_change) break;
    int ls_evals = 0;
    if ((rc = l2_axpby<T>(L, L->t, L->d, 1.0, L->x))) return rc;
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

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

int fe_create(const fe_grid* grid, const double* eps, const double* p_coeffs, void* stream, fe_ctx** out) {
  g_last_error.clear();
  if (!out) return set_error(FE_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = check_grid(grid);
  if (rc) return rc;
  rc = check_params(grid->batch, eps, p_coeffs);
  if (rc) return rc;

  fe_ctx* c = new (std::nothrow) fe_ctx();
  if (!c) return set_error(FE_ENOMEM, "host allocation failed");
  c->grid = *grid;
  c->stream = static_cast<hipStream_t>(stream);
  c->eps.assign(eps, eps + grid->batch);
  c->coeffs.assign(p_coeffs, p_coeffs + 6 * grid->batch);
  c->mu.assign(grid->batch, 0.0);
  c->theta.assign(3 * grid->batch, 0.0);
  c->variant = default_variant(*grid);
  c->lz = 0;

  auto fail = [&](int code) {
    fe_destroy(c);
    return code;
  };
  if (hipGetDevice(&c->device) != hipSuccess) return fail(set_error(FE_EHIP, "hipGetDevice failed"));
  {
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device) == hipSuccess && ncu > 0)
      c->num_cu = ncu;
  }
  if (hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess)
    return fail(set_error(FE_EHIP, "hipStreamCreateWithFlags failed"));

  // partials workspace: the largest per-instance block count of any variant at z chunk 1
  size_t mb = 0;
  for (int v = 0; v < (int)variants().size(); ++v) {
    if (!variant_ok(v, grid->dtype)) continue;
    const Variant& x = variants()[v];
    mb = std::max(mb, (size_t)ceil_div(grid->nx, x.tx) * ceil_div(grid->ny, x.ty) * grid->nz);
  }
  c->max_blocks = mb;
  const size_t prm_bytes = grid->dtype == FE_F32 ? sizeof(fe::InstParams<float>) : sizeof(fe::InstParams<double>);
  if (hipMalloc(&c->d_prm, prm_bytes * grid->batch) != hipSuccess ||
      hipMalloc((void**)&c->d_partials, sizeof(double) * 2 * mb * grid->batch) != hipSuccess ||
      hipMalloc((void**)&c->d_energy, sizeof(double) * grid->batch) != hipSuccess ||
      hipMalloc((void**)&c->d_mass, sizeof(double) * grid->batch) != hipSuccess ||
      hipMalloc((void**)&c->d_shift, sizeof(double) * 2 * grid->batch) != hipSuccess ||
      hipMalloc((void**)&c->d_counters, sizeof(int) * (grid->batch + 1)) != hipSuccess)
    return fail(set_error(FE_ENOMEM, "device workspace allocation failed"));
  hipLaunchKernelGGL(fe::fill_i32, dim3(ceil_div(grid->batch + 1, 64)), dim3(64), 0, c->stream, c->d_counters,
                     grid->batch + 1, 0);
  if (hipGetLastError() != hipSuccess) return fail(set_error(FE_EHIP, "counter initialisation failed"));
  rc = upload_params(c);
  if (rc) return fail(rc);
  *out = c;
  return FE_OK;
}

int fe_set_params(fe_ctx* c, const double* eps, const double* p_coeffs) {
  g_last_error.clear();
  if (!c) return set_error(FE_EINVAL, "ctx is NULL");
  int rc = check_params(c->grid.batch, eps, p_coeffs);
  if (rc) return rc;
  DeviceGuard dg(c->device);
  c->eps.assign(eps, eps + c->grid.batch);
  c->coeffs.assign(p_coeffs, p_coeffs + 6 * c->grid.batch);
  c->use_cfield = false;   // its scaling depends on eps: the caller sets it again
  return upload_params(c);
}

int fe_set_orientation(fe_ctx* c, const double* mu, const double* theta) {
  g_last_error.clear();
  if (!c) return set_error(FE_EINVAL, "ctx is NULL");
  if (!mu || !theta) return set_error(FE_EINVAL, "mu and theta must not be NULL");
  for (int b = 0; b < c->grid.batch; ++b) {
    if (!std::isfinite(mu[b])) return set_error(FE_EINVAL, "mu[%d] is not finite", b);
    for (int k = 0; k < 3; ++k)
      if (!std::isfinite(theta[3 * b + k])) return set_error(FE_EINVAL, "theta[%d] is not finite", b);
  }
  DeviceGuard dg(c->device);
  c->mu.assign(mu, mu + c->grid.batch);
  c->theta.assign(theta, theta + 3 * c->grid.batch);
  return upload_params(c);
}

int fe_set_coeff_field(fe_ctx* c, const void* a_field) {
  g_last_error.clear();
  if (!c) return set_error(FE_EINVAL, "ctx is NULL");
  if (!a_field) {
    c->use_cfield = false;
    return FE_OK;
  }
  DeviceGuard dg(c->device);
  const size_t n = field_elems(c->grid);
  if (!c->d_cfield && hipMalloc(&c->d_cfield, 6 * n * elem_size(c->grid)) != hipSuccess) {
    c->d_cfield = nullptr;
    return set_error(FE_ENOMEM, "coefficient field allocation failed");
  }
  const double h = c->grid.h, h3 = h * h * h;
  const int B = c->grid.batch;
  std::vector<double> k(3 * B);
  for (int b = 0; b < B; ++b) {
    const double e = c->eps[b], sc = e / (h * h);
    k[3 * b] = h3 * sc * sc / (2.0 * e);
    k[3 * b + 1] = h3 * sc / (4.0 * h);
    k[3 * b + 2] = h3 * e / (4.0 * h * h);
  }
  double* d_k = nullptr;
  if (hipMalloc((void**)&d_k, sizeof(double) * k.size()) != hipSuccess)
    return set_error(FE_ENOMEM, "coefficient factor allocation failed");
  hipError_t e1 = hipMemcpyAsync(d_k, k.data(), sizeof(double) * k.size(), hipMemcpyHostToDevice, c->stream);
  const size_t vol = n / B;
  const int nblk = (int)std::min<size_t>((n + 255) / 256, 65536);
  if (e1 == hipSuccess) {
    if (c->grid.dtype == FE_F32)
      hipLaunchKernelGGL(fe::scale_coeff_field<float>, dim3(nblk), dim3(256), 0, c->stream,
                         static_cast<const float*>(a_field), static_cast<float*>(c->d_cfield), vol, B,
                         (const double*)d_k);
    else
      hipLaunchKernelGGL(fe::scale_coeff_field<double>, dim3(nblk), dim3(256), 0, c->stream,
                         static_cast<const double*>(a_field), static_cast<double*>(c->d_cfield), vol, B,
                         (const double*)d_k);
    e1 = hipGetLastError();
  }
  // the factors (and the host vector) must outlive the conversion
  const hipError_t e2 = hipStreamSynchronize(c->stream);
  (void)hipFree(d_k);
  if (e1 != hipSuccess) return set_error(FE_EHIP, "coefficient field conversion failed: %s", hipGetErrorString(e1));
  if (e2 != hipSuccess) return set_error(FE_EHIP, "hipStreamSynchronize failed: %s", hipGetErrorString(e2));
  c->use_cfield = true;
  return FE_OK;
}

int fe_set_mass_field(fe_ctx* c, const void* m_field) {
  g_last_error.clear();
  if (!c) return set_error(FE_EINVAL, "ctx is NULL");
  if (!m_field) {
    c->use_mfield = false;
    return FE_OK;
  }
  DeviceGuard dg(c->device);
  const size_t bytes = field_elems(c->grid) * elem_size(c->grid);
  if (!c->d_mfield && hipMalloc(&c->d_mfield, bytes) != hipSuccess) {
    c->d_mfield = nullptr;
    return set_error(FE_ENOMEM, "mass field allocation failed");
  }
  FE_HIP(hipMemcpyAsync(c->d_mfield, m_field, bytes, hipMemcpyDeviceToDevice, c->stream));
  c->use_mfield = true;
  return FE_OK;
}

int fe_set_stream(fe_ctx* c, void* stream) {
  g_last_error.clear();
  if (!c) return set_error(FE_EINVAL, "ctx is NULL");
  c->stream = static_cast<hipStream_t>(stream);
  return FE_OK;
}

int fe_energy_grad_async(fe_ctx* c, const void* u, void* g, double* energy_dev) {
  g_last_error.clear();
  if (!c) return set_error(FE_EINVAL, "ctx is NULL");
  if (!u) return set_error(FE_EINVAL, "u is NULL");
  if (g == u) return set_error(FE_EINVAL, "g must not alias u");
  DeviceGuard dg(c->device);
  const StepRule none{fe::kGrad, 0.0, 0.0, 0.0, 0.0};
  return sweep(c, c->stream, g ? fe::kGrad : -1, u, g, nullptr, nullptr, energy_dev ? energy_dev : c->d_energy,
               none);
}

int fe_energy(fe_ctx* c, const void* u, double* energy) {
  int rc = fe_energy_grad_async(c, u, nullptr, c ? c->d_energy : nullptr);
  if (rc) return rc;
  DeviceGuard dg(c->device);
  return copy_energy_out(c, energy);
}

int fe_energy_grad(fe_ctx* c, const void* u, void* g, double* energy) {
  if (c && !g) return set_error(FE_EINVAL, "g is NULL (use fe_energy for the energy only)");
  int rc = fe_energy_grad_async(c, u, g, c ? c->d_energy : nullptr);
  if (rc) return rc;
  DeviceGuard dg(c->device);
  return copy_energy_out(c, energy);
}

int fe_step(fe_ctx* c, void* u, const double* mass, double tau, int nsteps, double* energy) {
  g_last_error.clear();
  if (!c) return set_error(FE_EINVAL, "ctx is NULL");
  if (!(tau > 0.0) || !std::isfinite(tau)) return set_error(FE_EINVAL, "tau must be finite and > 0");
  const StepRule rule{fe::kStepGD, tau, 0.0, 0.0, 0.0};
  return run_steps(c, u, mass, rule, nsteps, energy);
}

int fe_step_adam(fe_ctx* c, void* u, const double* mass, double lr, double beta1, double beta2, double adam_eps,
                 int nsteps, double* energy) {
  g_last_error.clear();
  if (!c) return set_error(FE_EINVAL, "ctx is NULL");
  if (!(lr > 0.0) || !std::isfinite(lr)) return set_error(FE_EINVAL, "lr must be finite and > 0");
  if (!(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0))
    return set_error(FE_EINVAL, "beta1 and beta2 must lie in [0, 1)");
  if (!(adam_eps > 0.0) || !std::isfinite(adam_eps)) return set_error(FE_EINVAL, "adam_eps must be finite and > 0");
  if (!c->d_m1) {
    DeviceGuard dg(c->device);
    const size_t bytes = field_elems(c->grid) * elem_size(c->grid);
    if (hipMalloc(&c->d_m1, bytes) != hipSuccess || hipMalloc(&c->d_m2, bytes) != hipSuccess ||
        hipMalloc((void**)&c->d_adam_t, sizeof(int)) != hipSuccess) {
      if (c->d_m1) (void)hipFree(c->d_m1);
      if (c->d_m2) (void)hipFree(c->d_m2);
      if (c->d_adam_t) (void)hipFree(c->d_adam_t);
      c->d_m1 = c->d_m2 = nullptr;
      c->d_adam_t = nullptr;
      return set_error(FE_ENOMEM, "Adam moment allocation failed");
    }
    int rc = adam_reset_launch(c);
    if (rc) return rc;
  }
  const StepRule rule{fe::kStepAdam, lr, beta1, beta2, adam_eps};
  return run_steps(c, u, mass, rule, nsteps, energy);
}

int fe_adam_reset(fe_ctx* c) {
  g_last_error.clear();
  if (!c) return set_error(FE_EINVAL, "ctx is NULL");
  if (!c->d_m1) return FE_OK;   // nothing allocated yet: the first fe_step_adam starts from zero
  DeviceGuard dg(c->device);
  return adam_reset_launch(c);
}

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
  if ((long)c->grid.nz * c->grid.batch > 65535 || (long)c->grid.ny * c->grid.batch > 65535)
    return set_error(FE_EINVAL, "nz * batch and ny * batch must be <= 65535 for the flow kernels");
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
  return copy_energy_out(c, energy);
}

int fe_diagnostics(fe_ctx* c, const void* u, void* curv, double* hist, int nbins, double kmax, double* stats) {
  g_last_error.clear();
  if (!c) return set_error(FE_EINVAL, "ctx is NULL");
  if (!u) return set_error(FE_EINVAL, "u is NULL");
  if (curv == u) return set_error(FE_EINVAL, "curv must not alias u");
  if (hist) {
    if (nbins < 1 || nbins > fe::kDiagMaxBins)
      return set_error(FE_EINVAL, "nbins must lie in [1, %d] (got %d)", fe::kDiagMaxBins, nbins);
    if (!(kmax > 0.0) || !std::isfinite(kmax)) return set_error(FE_EINVAL, "kmax must be finite and > 0");
  }
  DeviceGuard dg(c->device);
  return c->grid.dtype == FE_F32 ? diagnostics<float>(c, u, curv, hist, nbins, kmax, stats)
                                 : diagnostics<double>(c, u, curv, hist, nbins, kmax, stats);
}

int fe_hminus_reset(fe_ctx* c) {
  g_last_error.clear();
  if (!c) return set_error(FE_EINVAL, "ctx is NULL");
  if (!c->d_am1) return FE_OK;
  DeviceGuard dg(c->device);
  return flow_reset_launch(c);
}

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
  if (hipMalloc((void**)&L->d_red, sizeof(double) * (fe::kVecBlocks + kL2Slots)) != hipSuccess) {
    L->d_red = nullptr;
    l2_free(L);
    return set_error(FE_ENOMEM, "L2 flow reduction buffer allocation failed");
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

int fe_num_variants(void) { return (int)variants().size(); }

int fe_variant_info(int variant, int* tile_x, int* tile_y, int* threads, int* dtype_mask) {
  if (variant < 0 || variant >= (int)variants().size()) return set_error(FE_EINVAL, "no variant %d", variant);
  const Variant& v = variants()[variant];
  if (tile_x) *tile_x = v.tx;
  if (tile_y) *tile_y = v.ty;
  if (threads) *threads = v.nt;
  if (dtype_mask) *dtype_mask = v.dtype_mask;
  return FE_OK;
}

int fe_set_launch(fe_ctx* c, int variant, int z_chunk) {
  g_last_error.clear();
  if (!c) return set_error(FE_EINVAL, "ctx is NULL");
  if (!variant_ok(variant, c->grid.dtype))
    return set_error(FE_EINVAL, "variant %d does not exist or does not support this dtype", variant);
  if (z_chunk < 0) return set_error(FE_EINVAL, "z_chunk must be >= 0");
  c->variant = variant;
  c->lz = z_chunk;
  return FE_OK;
}

int fe_get_launch(const fe_ctx* c, int* variant, int* z_chunk) {
  if (!c) return set_error(FE_EINVAL, "ctx is NULL");
  if (variant) *variant = c->variant;
  if (z_chunk) *z_chunk = geometry(c, c->variant, c->lz).lz;
  return FE_OK;
}

int fe_autotune(fe_ctx* c, const void* u, void* g, int iters, double* best_us) {
  g_last_error.clear();
  if (!c) return set_error(FE_EINVAL, "ctx is NULL");
  if (!u || !g || u == g) return set_error(FE_EINVAL, "u and g must be distinct device fields");
  if (iters < 1) return set_error(FE_EINVAL, "iters must be >= 1");
  DeviceGuard dg(c->device);
  const int keep_v = c->variant, keep_lz = c->lz;
  hipEvent_t e0, e1;
  FE_HIP(hipEventCreate(&e0));
  FE_HIP(hipEventCreate(&e1));
  double best = 1e300;
  int best_v = keep_v, best_lz = keep_lz;
  const int lzs[] = {4, 8, 16, 32, 64, 128};
  int rc = FE_OK;
  for (int v = 0; v < (int)variants().size() && rc == FE_OK; ++v) {
    if (!variant_ok(v, c->grid.dtype)) continue;
    const Variant& x = variants()[v];
    if (x.tx > 2 * c->grid.nx || x.ty > 2 * c->grid.ny) continue;
    for (int lz : lzs) {
      if (lz > c->grid.nz) continue;
      c->variant = v;
      c->lz = lz;
      rc = fe_energy_grad_async(c, u, g, nullptr);   // warm-up
      if (rc) break;
      if (hipEventRecord(e0, c->stream) != hipSuccess) { rc = set_error(FE_EHIP, "hipEventRecord failed"); break; }
      for (int i = 0; i < iters && rc == FE_OK; ++i) rc = fe_energy_grad_async(c, u, g, nullptr);
      if (rc) break;
      if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
        rc = set_error(FE_EHIP, "event timing failed");
        break;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      const double us = 1000.0 * ms / iters;
      if (us < best) {
        best = us;
        best_v = v;
        best_lz = lz;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->variant = best_v;
  c->lz = best_lz;
  if (rc) return rc;
  if (best_us) *best_us = best;
  return FE_OK;
}

void fe_destroy(fe_ctx* c) {
  if (!c) return;
  DeviceGuard dg(c->device);
  drop_graphs(c);
  if (c->d_prm) (void)hipFree(c->d_prm);
  if (c->d_partials) (void)hipFree(c->d_partials);
  if (c->d_energy) (void)hipFree(c->d_energy);
  if (c->d_mass) (void)hipFree(c->d_mass);
  if (c->d_shift) (void)hipFree(c->d_shift);
  if (c->d_counters) (void)hipFree(c->d_counters);
  if (c->d_pingpong) (void)hipFree(c->d_pingpong);
  if (c->d_m1) (void)hipFree(c->d_m1);
  if (c->d_m2) (void)hipFree(c->d_m2);
  if (c->d_adam_t) (void)hipFree(c->d_adam_t);
  for (void* p : {c->d_w0, c->d_w1, c->d_am1, c->d_am2, (void*)c->d_flow_clk, (void*)c->d_diag, c->d_cfield,
                  c->d_mfield})
    if (p) (void)hipFree(p);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  delete c;
}

const char* fe_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
