// Core host side of the C ABI: errors, launch variants, the context, the
// per-instance constants, the sweeps, the graph-replayed step loops, the
// autotuner, and the entry points for them. Included once by fe_api.hip.
#pragma once

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

// The sweep kernels of one launch shape: [fe::SweepBody] for the gradient, the
// plain step and the Adam step (the single-body ones only for the leading
// shapes; nullptr where not built).
template <typename T>
struct Kernels {
  SweepFn<T> grad[3] = {nullptr, nullptr, nullptr};
  SweepFn<T> step[3] = {nullptr, nullptr, nullptr};
  SweepFn<T> adam[3] = {nullptr, nullptr, nullptr};
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
  bool lead = false;   // a default candidate: chosen by the ring work its tiles cover a grid with
};

template <typename T, int TX, int TY, int NT, bool SP = false, bool BODIES = false>
Kernels<T> make_kernels() {
  Kernels<T> k;
  k.grad[fe::kBodyAny] = fe::grad_sweep<T, TX, TY, NT, fe::kGrad, SP>;
  k.step[fe::kBodyAny] = fe::grad_sweep<T, TX, TY, NT, fe::kStepGD, SP>;
  k.adam[fe::kBodyAny] = fe::grad_sweep<T, TX, TY, NT, fe::kStepAdam, SP>;
  if constexpr (BODIES && !SP) {
    k.grad[fe::kBodyNoS] = fe::grad_sweep<T, TX, TY, NT, fe::kGrad, false, false, fe::kBodyNoS>;
    k.step[fe::kBodyNoS] = fe::grad_sweep<T, TX, TY, NT, fe::kStepGD, false, false, fe::kBodyNoS>;
    k.adam[fe::kBodyNoS] = fe::grad_sweep<T, TX, TY, NT, fe::kStepAdam, false, false, fe::kBodyNoS>;
    k.grad[fe::kBodyFull] = fe::grad_sweep<T, TX, TY, NT, fe::kGrad, false, false, fe::kBodyFull>;
    k.step[fe::kBodyFull] = fe::grad_sweep<T, TX, TY, NT, fe::kStepGD, false, false, fe::kBodyFull>;
    k.adam[fe::kBodyFull] = fe::grad_sweep<T, TX, TY, NT, fe::kStepAdam, false, false, fe::kBodyFull>;
  }
  k.energy = fe::energy_sweep<T, TX, TY, NT, SP>;
  return k;
}

// The kernel of `kind` (a fe::SweepMode) for a batch whose instances all take
// `body`, or the per-instance one where no single-body kernel is built.
template <typename T>
SweepFn<T> sweep_kernel(const Kernels<T>& k, int kind, int body) {
  const SweepFn<T>* f = kind == fe::kGrad ? k.grad : kind == fe::kStepGD ? k.step : k.adam;
  return f[body] ? f[body] : f[fe::kBodyAny];
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
    // the coefficient-field and box kernels exist for a few large tiles, one
    // small and the smallest tile of each precision (not for 50 x 20 with a
    // coefficient field: 134 VGPRs, one block per CU). 32 x 32 and 50 x 20 lead
    // the FP32 list: the same block (512 threads, three u loads and three ring
    // voxels per thread, 48 KiB of LDS, two blocks per CU) over a tile whose
    // ring is 1.13 or 1.14 of it. 32 x 32 covers power-of-two planes exactly,
    // 50 x 20 planes of 100, 200 or 600 (where 32 x 32 computes 1.85x the
    // plane at 100^2). 256^3 step, symmetric p: 94 us against 95 (64 x 16)
    // and 97 (64 x 32 / 1024).
    add32(32, 32, 512, make_kernels<float, 32, 32, 512, false, true>());
    r.back().lead = true;
    add32(50, 20, 512, make_kernels<float, 50, 20, 512, false, true>(), {},
          fe::grad_sweep<float, 50, 20, 512, fe::kGrad, false, true>);
    r.back().lead = true;
    add32(64, 16, 512, make_kernels<float, 64, 16, 512>(), make_kernels<float, 64, 16, 512, true>(),
          fe::grad_sweep<float, 64, 16, 512, fe::kGrad, false, true>);
    add32(64, 32, 1024, make_kernels<float, 64, 32, 1024>());
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
    add64(32, 16, 512, make_kernels<double, 32, 16, 512, false, true>(), make_kernels<double, 32, 16, 512, true>(),
          fe::grad_sweep<double, 32, 16, 512, fe::kGrad, false, true>);
    r.back().lead = true;
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

// Ring voxels one plane of the sweep evaluates when v's tiles cover an nx x ny
// plane, ragged tiles included (their wrapped columns are evaluated too).
double ring_work(const Variant& v, int nx, int ny) {
  return (double)ceil_div(nx, v.tx) * ceil_div(ny, v.ty) * (v.tx + 2) * (v.ty + 2);
}

bool tile_fits(const Variant& v, int nx, int ny) { return v.tx <= std::max(nx, 8) && v.ty <= std::max(ny, 8); }

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
  int body;                     // the per-voxel body the sweeps hold (fe::SweepBody)
  bool operator<(const GraphKey& o) const {
    return std::tie(u, mode, tau, beta1, beta2, adam_eps, sigma, pairs, variant, lz, fields, body) <
           std::tie(o.u, o.mode, o.tau, o.beta1, o.beta2, o.adam_eps, o.sigma, o.pairs, o.variant, o.lz,
                    o.fields, o.body);
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
  void* d_prm_scaled = nullptr;       // InstParams<T>[batch] with the coefficients scaled (fe_grad_scaled_async)
  const void* prm_active = nullptr;   // the table sweeps read while set (else d_prm)
  double* d_partials = nullptr;       // [2][batch][max_blocks][2]: block partials of two sweeps (steps alternate)
  double* d_energy = nullptr;         // [batch]
  double* d_mass = nullptr;           // [batch]
  double* d_shift = nullptr;          // [batch]: the shift of the last step's output
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
  void* d_cfield = nullptr;           // scaled coefficient field, [batch][nz][ny][nx] records of six (Sec. 5.2)
  bool use_cfield = false;
  void* d_mfield = nullptr;           // mass field m(x) [batch][nz][ny][nx] of the flow (Sec. 5.2)
  bool use_mfield = false;
  bool use_box = false;               // padded non-periodic field: density only inside the box
  int box_lo[3] = {0, 0, 0}, box_hi[3] = {0, 0, 0};
  size_t max_blocks = 0;              // per instance, over all variants and z chunks
  int variant = -1;
  int lz = 0;                         // 0 = automatic
  int body = 0;                       // fe::SweepBody every instance takes (kBodyAny: they differ)
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
  const double plane_bytes = (double)g->nx * g->ny * (g->dtype == FE_F64 ? 8.0 : 4.0);
  if (n * g->batch > 4.0e9 || plane_bytes > 4294901760.0)
    return set_error(FE_EINVAL, "grid too large for 32-bit plane indexing (planes must be at most 4 GiB - 64 KiB)");
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
// One instance's constants: spacing h, width e, coefficients a[6], orientation
// term mu (0: off) along theta[3].
template <typename T>
fe::InstParams<T> inst_params(double h, double e, const double* a, double mu, const double* theta) {
  const double h3 = h * h * h;
  const double a20 = a[0], a11 = a[1], a02 = a[2], a10 = a[3], a01 = a[4], a00 = a[5];
  const double c1 = (a20 + a02 - a11) / (2.0 * e), c2 = a11 / (2.0 * e), c3 = (a20 - a02) / (2.0 * e);
  const double c4 = (a10 + a01) / 2.0, c5 = (a10 - a01) / 2.0, c6 = a00;
  const double sc = e / (h * h);
  fe::InstParams<T> p;
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
  p.Co = T(h3 * e * mu / (4.0 * h * h));
  p.thx = T(theta[0]);
  p.thy = T(theta[1]);
  p.thz = T(theta[2]);
  return p;
}

template <typename T>
void fill_params(const fe_ctx* c, std::vector<fe::InstParams<T>>& out) {
  out.resize(c->grid.batch);
  for (int b = 0; b < c->grid.batch; ++b)
    out[b] = inst_params<T>(c->grid.h, c->eps[b], &c->coeffs[6 * b], c->mu[b], &c->theta[3 * b]);
}

template <typename T>
fe::GridConsts<T> grid_consts(double h) {
  fe::GridConsts<T> k;
  k.reg_d = 4.0 * h * h * kXi * kXi;
  k.reg = T(k.reg_d);
  return k;
}

// The body every instance of `p` takes (fe::has_s_terms on the typed constants,
// as the kernels decide it), or kBodyAny if they differ.
template <typename T>
int batch_body(const fe::InstParams<T>* p, int batch) {
  int nos = 0;
  for (int b = 0; b < batch; ++b) nos += (p[b].C3 == T(0) && p[b].C5 == T(0)) ? 1 : 0;
  return nos == batch ? fe::kBodyNoS : nos == 0 ? fe::kBodyFull : fe::kBodyAny;
}

int upload_params(fe_ctx* c) {
  if (c->grid.dtype == FE_F32) {
    std::vector<fe::InstParams<float>> p;
    fill_params(c, p);
    c->body = batch_body(p.data(), c->grid.batch);
    FE_HIP(hipMemcpyAsync(c->d_prm, p.data(), p.size() * sizeof(p[0]), hipMemcpyHostToDevice, c->stream));
  } else {
    std::vector<fe::InstParams<double>> p;
    fill_params(c, p);
    c->body = batch_body(p.data(), c->grid.batch);
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

// Time of a sweep whose busiest compute unit runs k = ceil(blocks / num_cu)
// blocks of L planes, `slots` at a time, in units of one plane of a block in a
// full CU: a full group of `slots` blocks costs 1 per plane, a CU left with
// r < slots blocks (r / slots)^0.6 per plane (0.66 for one of two: alone it
// hides less latency, yet finishes sooner). Fitted to the step sweep on 100^3
// to 256^3 grids, one and 16 instances, two blocks per CU.
double sweep_cost(long blocks, int num_cu, int slots, int L) {
  const long k = (blocks + num_cu - 1) / num_cu;
  const long rest = k % slots;
  double t = (double)(k / slots) * L;
  if (rest) t += L * std::pow((double)rest / slots, 0.6);
  return t;
}

// The z chunk length of a halo-1 sweep (the energy-only and diagnostics sweeps)
// over `cols` tile columns that sweep_cost finishes first, a chunk of l planes
// costing about l + 1 (its two halo planes are loads only).
int halo1_chunk(long cols, int nz, int num_cu, int slots) {
  double best = 0.0;
  int lz = 0;
  for (int nzc = 1; nzc <= nz; ++nzc) {
    const int l = ceil_div(nz, nzc);
    if (nzc > 1 && l == ceil_div(nz, nzc - 1)) continue;
    const double t = sweep_cost(cols * ceil_div(nz, l), num_cu, slots, l + 1);
    if (lz <= 0 || t < best) {
      best = t;
      lz = l;
    }
  }
  return lz;
}

// `slots`: blocks of the launched kernel that one compute unit holds at once
// (used when lz_req is 0, automatic).
Geometry geometry_of(const fe_grid& grid, int num_cu, int variant, int lz_req, int slots) {
  const Variant& v = variants()[variant];
  Geometry g;
  g.ntx = ceil_div(grid.nx, v.tx);
  g.nty = ceil_div(grid.ny, v.ty);
  int lz = lz_req;
  if (lz <= 0) {
    // the equal z chunks whose sweep sweep_cost finishes first: longer chunks
    // recompute fewer boundary planes, more of them fill more compute units,
    // and a last round of blocks that fills only some CUs costs most of a
    // round (256^3 in 32 x 32 tiles: 32 planes, 512 blocks; 200^3 in 50 x 20
    // tiles: 17 planes, 480 blocks, 73 us against 102 us for 16 planes)
    const int nz = grid.nz;
    const long cols = (long)g.ntx * g.nty * grid.batch;
    double best = 0.0;
    for (int nzc = 1; nzc <= nz; ++nzc) {
      const int l = ceil_div(nz, nzc);
      if (nzc > 1 && l == ceil_div(nz, nzc - 1)) continue;   // the same chunks as nzc - 1
      const double t = sweep_cost(cols * ceil_div(nz, l), num_cu, slots, l + 2);
      if (lz <= 0 || t < best) {
        best = t;
        lz = l;
      }
    }
  }
  lz = std::min(std::max(lz, 1), grid.nz);
  g.lz = lz;
  g.nzc = ceil_div(grid.nz, lz);
  g.per_inst = g.ntx * g.nty * g.nzc;
  return g;
}

// The kernel launch_sweep runs for `kind` (-1: energy only, else a
// fe::SweepMode) with `variant` on this context.
template <typename T>
SweepFn<T> sweep_fn(const fe_ctx* c, const Variant& v, int kind) {
  if (c->use_box) return box_kernel_of<T>(v);
  const Kernels<T>& k = kernels_of<T>(v, c->use_cfield);
  return kind < 0 ? k.energy : sweep_kernel<T>(k, kind, c->use_cfield ? (int)fe::kBodyAny : c->body);
}

// Blocks of that kernel one compute unit holds at once: its registers and LDS
// decide it (the symmetric step body at 32 x 32 takes three, the bodies with the
// S terms two), and the automatic z chunks follow it.
int launch_slots(const fe_ctx* c, int variant, int kind) {
  const Variant& v = variants()[variant];
  const void* fn = c->grid.dtype == FE_F32 ? (const void*)sweep_fn<float>(c, v, kind)
                                           : (const void*)sweep_fn<double>(c, v, kind);
  int n = 0;
  if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, v.nt, 0) != hipSuccess || n < 1) n = 1;
  return n;
}

// Launch geometry of a sweep of `kind` with `variant` on this context.
Geometry geometry(const fe_ctx* c, int variant, int lz_req, int kind) {
  return geometry_of(c->grid, c->num_cu, variant, lz_req, lz_req > 0 ? 1 : launch_slots(c, variant, kind));
}

bool has_sp(int v, int dtype) {
  const Variant& x = variants()[v];
  return dtype == FE_F32 ? x.k32sp.grad[fe::kBodyAny] != nullptr : x.k64sp.grad[fe::kBodyAny] != nullptr;
}

bool has_box(int v, int dtype) {
  const Variant& x = variants()[v];
  return dtype == FE_F32 ? x.k32box != nullptr : x.k64box != nullptr;
}

// The variant a sweep launches: the chosen one, unless a coefficient field or
// a box mask is in use and that variant has no such kernels; then, of those
// that have them and whose tile the grid fills, the one with the chosen
// block size that evaluates the least ring (else the first).
int sweep_variant(const fe_ctx* c) {
  auto ok = [&](int v) {
    return (!c->use_cfield || has_sp(v, c->grid.dtype)) && (!c->use_box || has_box(v, c->grid.dtype));
  };
  if (ok(c->variant)) return c->variant;
  const int nt = variants()[c->variant].nt;
  int first = -1, best = -1, last = c->variant;
  for (int v = 0; v < (int)variants().size(); ++v) {
    if (!variant_ok(v, c->grid.dtype) || !ok(v)) continue;
    last = v;
    const Variant& x = variants()[v];
    if (!tile_fits(x, c->grid.nx, c->grid.ny)) continue;
    if (first < 0) first = v;
    if (x.nt == nt &&
        (best < 0 || ring_work(x, c->grid.nx, c->grid.ny) < ring_work(variants()[best], c->grid.nx, c->grid.ny)))
      best = v;
  }
  return best >= 0 ? best : first >= 0 ? first : last;
}

int fields_in_use(const fe_ctx* c) { return (c->use_cfield ? 1 : 0) | (c->use_mfield ? 2 : 0); }

int default_variant(const fe_grid& g) {
  const int dt = g.dtype;
  // of the leading variants whose tile the grid fills, the one that evaluates
  // the least ring per plane (ties: the earlier)
  int best = -1;
  for (int v = 0; v < (int)variants().size(); ++v) {
    const Variant& x = variants()[v];
    if (!variant_ok(v, dt) || !x.lead || !tile_fits(x, g.nx, g.ny)) continue;
    if (best < 0 || ring_work(x, g.nx, g.ny) < ring_work(variants()[best], g.nx, g.ny)) best = v;
  }
  if (best >= 0) return best;
  // else, variants being listed largest tile first, the first whose tile the
  // grid fills
  for (int v = 0; v < (int)variants().size(); ++v) {
    if (!variant_ok(v, dt)) continue;
    if (tile_fits(variants()[v], g.nx, g.ny)) return v;
  }
  for (int v = (int)variants().size() - 1; v >= 0; --v)
    if (variant_ok(v, dt)) return v;
  return 0;
}

// Block-partial buffer i (0 or 1) of the context.
double* partials_buf(fe_ctx* c, int i) { return c->d_partials + (size_t)i * 2 * c->max_blocks * c->grid.batch; }

// kind: -1 energy only, else a fe::SweepMode. One launch; the block partials go
// to `partials`. Steps add to src the shift formed from prev_partials (the
// partials of the step that wrote src; null: no shift); Adam steps use the
// step number t0 + t_add.
template <typename T>
int launch_sweep(fe_ctx* c, hipStream_t s, int kind, const void* src, void* dst, const double* prev_partials,
                 double* partials, const StepRule& rule, int t_add) {
  const int vi = sweep_variant(c);
  const Geometry geo = geometry(c, vi, c->lz, kind);
  if ((size_t)geo.per_inst > c->max_blocks) return set_error(FE_EINVAL, "internal: partials workspace too small");
  const Variant& v = variants()[vi];
  fe::SweepArgs<T> a;
  a.src = static_cast<const T*>(src);
  a.dst = static_cast<T*>(dst);
  a.prm = static_cast<const fe::InstParams<T>*>(c->prm_active ? c->prm_active : c->d_prm);
  a.prev_partials = prev_partials;
  a.partials = partials;
  a.mass = c->d_mass;
  a.inv_nvox = 1.0 / ((double)c->grid.nx * c->grid.ny * c->grid.nz);
  a.k = grid_consts<T>(c->grid.h);
  a.m1 = static_cast<T*>(c->d_m1);
  a.m2 = static_cast<T*>(c->d_m2);
  a.adam_t = c->d_adam_t;
  a.t_add = t_add;
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
  if (c->use_box && (kind != fe::kGrad || c->use_cfield))
    return set_error(FE_EINVAL, "internal: box sweeps are gradient-only");
  const SweepFn<T> fn = sweep_fn<T>(c, v, kind);
  if (c->use_box) {
    for (int i = 0; i < 3; ++i) {
      a.box_lo[i] = c->box_lo[i];
      a.box_hi[i] = c->box_hi[i];
    }
  }
  hipLaunchKernelGGL(fn, grid, block, 0, s, a);
  FE_HIP(hipGetLastError());
  return FE_OK;
}

int sweep(fe_ctx* c, hipStream_t s, int kind, const void* src, void* dst, const double* prev_partials,
          double* partials, const StepRule& rule, int t_add = 0) {
  return c->grid.dtype == FE_F32 ? launch_sweep<float>(c, s, kind, src, dst, prev_partials, partials, rule, t_add)
                                 : launch_sweep<double>(c, s, kind, src, dst, prev_partials, partials, rule, t_add);
}

// Per-instance totals of the sweep of `kind` that wrote `partials` (same launch
// shape): energy_dev[b] and, when shift is given, shift[b] = mass[b] - mean of
// its field.
int finish_sums(fe_ctx* c, hipStream_t s, const double* partials, double* energy_dev, double* shift, int kind) {
  const Geometry geo = geometry(c, sweep_variant(c), c->lz, kind);
  hipLaunchKernelGGL(fe::sweep_finish, dim3(c->grid.batch), dim3(64), 0, s, partials, geo.per_inst, energy_dev,
                     (const double*)c->d_mass, 1.0 / ((double)c->grid.nx * c->grid.ny * c->grid.nz), shift);
  FE_HIP(hipGetLastError());
  return FE_OK;
}

// The energy-only sweep (fe::energy_sweep_cols): one x column per lane, 64-wide
// tiles of 8 waves, 2 rows per thread in FP32 (64 x 16 tiles, 106 VGPRs), 1 in
// FP64 (64 x 8, 119 VGPRs): two blocks per CU. 256^3 FP32, measured against 3
// and 4 rows per thread, 4 and 16 waves per block and chunks of 8 to 64
// planes: 31.5 us (symmetric p) and 47 us (full body) at 32-plane chunks, the
// makespan model's choice, within 2% of the fastest of those shapes.
constexpr int kEnergyWaves = 8;
int energy_rows(int dtype) { return dtype == FE_F32 ? 2 : 1; }

const void* energy_cols_kernel(int dtype) {
  return dtype == FE_F32 ? (const void*)fe::energy_sweep_cols<float, 2, kEnergyWaves>
                         : (const void*)fe::energy_sweep_cols<double, 1, kEnergyWaves>;
}

// Launch geometry of the energy-only sweep: tiles as above, z chunks by the
// makespan model of the gradient sweep (a chunk of lz planes costs about lz + 1,
// its two halo planes being loads only).
Geometry energy_geometry(const fe_grid& grid, int num_cu) {
  Geometry g;
  g.ntx = ceil_div(grid.nx, 64);
  g.nty = ceil_div(grid.ny, energy_rows(grid.dtype) * kEnergyWaves);
  int slots = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&slots, energy_cols_kernel(grid.dtype), 64 * kEnergyWaves, 0) !=
          hipSuccess || slots < 1)
    slots = 1;
  g.lz = halo1_chunk((long)g.ntx * g.nty * grid.batch, grid.nz, num_cu, slots);
  g.nzc = ceil_div(grid.nz, g.lz);
  g.per_inst = g.ntx * g.nty * g.nzc;
  return g;
}

// One energy-only sweep of u: block partials into `partials`; returns its geometry.
template <typename T>
int launch_energy_cols(const fe_grid& grid, const Geometry& geo, const void* u, const void* prm, double* partials,
                       hipStream_t s) {
  fe::SweepArgs<T> a{};
  a.src = static_cast<const T*>(u);
  a.prm = static_cast<const fe::InstParams<T>*>(prm);
  a.partials = partials;
  a.inv_nvox = 1.0 / ((double)grid.nx * grid.ny * grid.nz);
  a.k = grid_consts<T>(grid.h);
  a.nx = grid.nx;
  a.ny = grid.ny;
  a.nz = grid.nz;
  a.ntx = geo.ntx;
  a.nty = geo.nty;
  a.nzc = geo.nzc;
  a.lz = geo.lz;
  a.batch = grid.batch;
  const dim3 blocks((unsigned)(geo.per_inst * grid.batch)), threads(64 * kEnergyWaves);
  constexpr int V = std::is_same<T, float>::value ? 2 : 1;
  hipLaunchKernelGGL((fe::energy_sweep_cols<T, V, kEnergyWaves>), blocks, threads, 0, s, a);
  FE_HIP(hipGetLastError());
  return FE_OK;
}

int launch_energy_cols_any(const fe_grid& grid, const Geometry& geo, const void* u, const void* prm,
                           double* partials, hipStream_t s) {
  return grid.dtype == FE_F32 ? launch_energy_cols<float>(grid, geo, u, prm, partials, s)
                              : launch_energy_cols<double>(grid, geo, u, prm, partials, s);
}

// A gradient (or energy-only, kind -1) sweep and its energies into energy_dev.
int sweep_energy(fe_ctx* c, hipStream_t s, int kind, const void* src, void* dst, double* energy_dev) {
  if (kind < 0 && !c->use_cfield && !c->use_box) {
    const Geometry geo = energy_geometry(c->grid, c->num_cu);
    if ((size_t)geo.per_inst > c->max_blocks) return set_error(FE_EINVAL, "internal: partials workspace too small");
    int rc = launch_energy_cols_any(c->grid, geo, src, c->d_prm, partials_buf(c, 0), s);
    if (rc) return rc;
    hipLaunchKernelGGL(fe::sweep_finish, dim3(c->grid.batch), dim3(64), 0, s, (const double*)partials_buf(c, 0),
                       geo.per_inst, energy_dev, (const double*)c->d_mass,
                       1.0 / ((double)c->grid.nx * c->grid.ny * c->grid.nz), (double*)nullptr);
    FE_HIP(hipGetLastError());
    return FE_OK;
  }
  const StepRule none{fe::kGrad, 0.0, 0.0, 0.0, 0.0};
  int rc = sweep(c, s, kind, src, dst, nullptr, partials_buf(c, 0), none);
  return rc ? rc : finish_sums(c, s, partials_buf(c, 0), energy_dev, nullptr, kind);
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

// u = last + shift per instance (last may be u): 16-byte accesses when both
// fields are 16-byte aligned and an instance is a whole number of groups.
int launch_add_shift(fe_ctx* c, const void* last, void* u, const double* shift) {
  const size_t per_inst = (size_t)c->grid.nx * c->grid.ny * c->grid.nz;
  const size_t w = 16 / elem_size(c->grid);
  const bool vec = per_inst % w == 0 && (uintptr_t)last % 16 == 0 && (uintptr_t)u % 16 == 0;
  const size_t work = vec ? (per_inst / w + 3) / 4 : per_inst;     // per thread: 4 groups, or 1 voxel
  const dim3 blocks((unsigned)std::max<size_t>(1, std::min<size_t>((work + 255) / 256, 4096)),
                    (unsigned)c->grid.batch);
  const bool f32 = c->grid.dtype == FE_F32;
  if (f32 && vec)
    hipLaunchKernelGGL((fe::add_shift<float, true>), blocks, dim3(256), 0, c->stream, (const float*)last, (float*)u,
                       shift, per_inst);
  else if (f32)
    hipLaunchKernelGGL((fe::add_shift<float, false>), blocks, dim3(256), 0, c->stream, (const float*)last,
                       (float*)u, shift, per_inst);
  else if (vec)
    hipLaunchKernelGGL((fe::add_shift<double, true>), blocks, dim3(256), 0, c->stream, (const double*)last,
                       (double*)u, shift, per_inst);
  else
    hipLaunchKernelGGL((fe::add_shift<double, false>), blocks, dim3(256), 0, c->stream, (const double*)last,
                       (double*)u, shift, per_inst);
  FE_HIP(hipGetLastError());
  return FE_OK;
}

int adam_tick_launch(fe_ctx* c, hipStream_t s, int n) {
  hipLaunchKernelGGL(fe::adam_tick, dim3(1), dim3(64), 0, s, c->d_adam_t, n);
  FE_HIP(hipGetLastError());
  return FE_OK;
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
  void* A = c->d_pingpong;
  double* P0 = partials_buf(c, 0);
  double* P1 = partials_buf(c, 1);
  const bool adam = rule.mode == fe::kStepAdam;
  // Steps launched since the Adam step number was last advanced; step j of
  // them uses t0 + j.
  int pending = 0;
  auto step = [&](hipStream_t s, const void* src, void* dst, const double* prev, double* out, int t_add) {
    return sweep(c, s, rule.mode, src, dst, prev, out, rule, t_add);
  };
  auto tick = [&](hipStream_t s, int n) { return adam && n > 0 ? adam_tick_launch(c, s, n) : FE_OK; };

  // The first step, u -> A, takes u as it is; every later step adds the shift
  // that the partials of its predecessor give. The rest come in pairs A -> u
  // (partials P1), u -> A (partials P0): whole blocks of kGraphPairs pairs are
  // replayed from one captured graph (the same graph for any nsteps), the
  // others launch directly.
  int rc = step(c->stream, u, A, nullptr, P0, pending++);
  if (rc) return rc;
  const int npairs = (nsteps - 1) / 2;
  const int gpairs = npairs >= kGraphPairs ? kGraphPairs : 0;
  for (int i = 0; i < (gpairs ? npairs % gpairs : npairs); ++i) {
    rc = step(c->stream, A, u, P0, P1, pending++);
    if (rc == FE_OK) rc = step(c->stream, u, A, P1, P0, pending++);
    if (rc) return rc;
  }
  if (gpairs > 0) {
    if ((rc = tick(c->stream, pending))) return rc;
    pending = 0;
    GraphKey key{u,      rule.mode,           rule.tau, rule.beta1,       rule.beta2, rule.adam_eps, 0.0,
                 gpairs, sweep_variant(c), c->lz,    fields_in_use(c), c->body};
    auto it = c->graphs.find(key);
    hipGraphExec_t exec = nullptr;
    if (it == c->graphs.end()) {
      hipGraph_t graph = nullptr;
      FE_HIP(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
      for (int i = 0; i < gpairs && rc == FE_OK; ++i) {
        rc = step(c->cap_stream, A, u, P0, P1, 2 * i);
        if (rc == FE_OK) rc = step(c->cap_stream, u, A, P1, P0, 2 * i + 1);
      }
      if (rc == FE_OK) rc = tick(c->cap_stream, 2 * gpairs);
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
  const void* last = A;
  const double* last_p = P0;
  if ((nsteps - 1) % 2) {
    if ((rc = step(c->stream, A, u, P0, P1, pending++))) return rc;
    last = u;
    last_p = P1;
  }
  if ((rc = tick(c->stream, pending))) return rc;
  // the energy of the last step's input and the shift of its output
  double* shift = c->d_shift;
  if ((rc = finish_sums(c, c->stream, last_p, c->d_energy, shift, rule.mode))) return rc;
  if ((rc = launch_add_shift(c, last, u, shift))) return rc;
  return copy_energy_out(c, energy);
}

// Launch shapes chosen by fe_autotune, kept for the process (and saved to or
// loaded from a text file on request), keyed by what the choice depends on.
struct TuneEntry {
  int variant = 0, lz = 0;
  double us = 0.0;
};
std::map<std::string, TuneEntry> g_tune_cache;
std::mutex g_tune_mu;

// "<nx>x<ny>x<nz>x<batch>:<f32|f64>:<grad|step|adam>:<body>:<field|box|->:<device arch>"
// (the key holds no spaces).
int tune_key(const fe_ctx* c, int kind, std::string& key) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c->device) != hipSuccess)
    return set_error(FE_EHIP, "hipGetDeviceProperties failed");
  std::string arch = prop.gcnArchName;
  for (char& ch : arch)
    if (ch == ' ') ch = '_';
  static const char* kinds[] = {"grad", "step", "adam"};
  static const char* bodies[] = {"any", "nos", "full"};
  char buf[320];
  std::snprintf(buf, sizeof(buf), "%dx%dx%dx%d:%s:%s:%s:%s:%s", c->grid.nx, c->grid.ny, c->grid.nz, c->grid.batch,
                c->grid.dtype == FE_F32 ? "f32" : "f64", kinds[kind], bodies[c->body],
                c->use_box ? "box" : c->use_cfield ? "field" : "-", arch.c_str());
  key = buf;
  return FE_OK;
}

bool tune_lookup(const std::string& key, TuneEntry& out) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  auto it = g_tune_cache.find(key);
  if (it == g_tune_cache.end()) return false;
  out = it->second;
  return true;
}

void tune_store(const std::string& key, const TuneEntry& e) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune_cache[key] = e;
}

}  // namespace

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
  mb = std::max(mb, (size_t)ceil_div(grid->nx, 64) * ceil_div(grid->ny, energy_rows(grid->dtype) * kEnergyWaves) *
                        grid->nz);
  c->max_blocks = mb;
  const size_t prm_bytes = grid->dtype == FE_F32 ? sizeof(fe::InstParams<float>) : sizeof(fe::InstParams<double>);
  if (hipMalloc(&c->d_prm, prm_bytes * grid->batch) != hipSuccess ||
      hipMalloc(&c->d_prm_scaled, prm_bytes * grid->batch) != hipSuccess ||
      hipMalloc((void**)&c->d_partials, sizeof(double) * 4 * mb * grid->batch) != hipSuccess ||
      hipMalloc((void**)&c->d_energy, sizeof(double) * grid->batch) != hipSuccess ||
      hipMalloc((void**)&c->d_mass, sizeof(double) * grid->batch) != hipSuccess ||
      hipMalloc((void**)&c->d_shift, sizeof(double) * grid->batch) != hipSuccess)
    return fail(set_error(FE_ENOMEM, "device workspace allocation failed"));
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
  // the sweeps address a plane of six-value records with 32-bit byte offsets
  if ((double)c->grid.nx * c->grid.ny * 6.0 * (double)elem_size(c->grid) > 4294901760.0)
    return set_error(FE_EINVAL, "coefficient field too large: nx * ny * 6 samples must be at most 4 GiB - 64 KiB");
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
  return sweep_energy(c, c->stream, g ? fe::kGrad : -1, u, g, energy_dev ? energy_dev : c->d_energy);
}

int fe_grad_scaled_async(fe_ctx* c, const void* u, void* g, const double* gscale) {
  g_last_error.clear();
  if (!c) return set_error(FE_EINVAL, "ctx is NULL");
  if (!u || !g || !gscale) return set_error(FE_EINVAL, "u, g and gscale must not be NULL");
  if (g == u) return set_error(FE_EINVAL, "g must not alias u");
  DeviceGuard dg(c->device);
  const StepRule none{fe::kGrad, 0.0, 0.0, 0.0, 0.0};
  const bool f32 = c->grid.dtype == FE_F32;
  if (c->use_cfield) {
    // the coefficients vary per voxel: the plain sweep, then g_b *= s_b
    int rc = sweep(c, c->stream, fe::kGrad, u, g, nullptr, partials_buf(c, 0), none);
    if (rc) return rc;
    const size_t per = (size_t)c->grid.nx * c->grid.ny * c->grid.nz;
    const dim3 blocks((unsigned)std::min<size_t>((per + 255) / 256, 4096), (unsigned)c->grid.batch);
    if (f32)
      hipLaunchKernelGGL(fe::scale_per_instance<float>, blocks, dim3(256), 0, c->stream, (float*)g, per, gscale);
    else
      hipLaunchKernelGGL(fe::scale_per_instance<double>, blocks, dim3(256), 0, c->stream, (double*)g, per, gscale);
    FE_HIP(hipGetLastError());
    return FE_OK;
  }
  if (f32)
    hipLaunchKernelGGL(fe::scale_params<float>, dim3(1), dim3(64), 0, c->stream,
                       (const fe::InstParams<float>*)c->d_prm, (fe::InstParams<float>*)c->d_prm_scaled, gscale,
                       c->grid.batch);
  else
    hipLaunchKernelGGL(fe::scale_params<double>, dim3(1), dim3(64), 0, c->stream,
                       (const fe::InstParams<double>*)c->d_prm, (fe::InstParams<double>*)c->d_prm_scaled, gscale,
                       c->grid.batch);
  FE_HIP(hipGetLastError());
  c->prm_active = c->d_prm_scaled;
  const int rc = sweep(c, c->stream, fe::kGrad, u, g, nullptr, partials_buf(c, 0), none);
  c->prm_active = nullptr;
  return rc;
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
  if (z_chunk) *z_chunk = geometry(c, c->variant, c->lz, fe::kStepGD).lz;
  return FE_OK;
}

int fe_autotune(fe_ctx* c, const void* u, void* work, int kind, int iters, double* best_us, int* cached) {
  g_last_error.clear();
  if (!c) return set_error(FE_EINVAL, "ctx is NULL");
  if (!u || !work || u == work) return set_error(FE_EINVAL, "u and work must be distinct device fields");
  if (iters < 1) return set_error(FE_EINVAL, "iters must be >= 1");
  if (kind != FE_TUNE_GRAD && kind != FE_TUNE_STEP && kind != FE_TUNE_ADAM)
    return set_error(FE_EINVAL, "kind must be FE_TUNE_GRAD, FE_TUNE_STEP or FE_TUNE_ADAM");
  if (kind != FE_TUNE_GRAD && c->use_box) return set_error(FE_EINVAL, "a box-masked context has no step sweeps");
  DeviceGuard dg(c->device);
  if (cached) *cached = 0;
  std::string key;
  int rc = tune_key(c, kind, key);
  if (rc) return rc;
  TuneEntry hit;
  if (tune_lookup(key, hit)) {
    c->variant = hit.variant;
    c->lz = hit.lz;
    if (best_us) *best_us = hit.us;
    if (cached) *cached = 1;
    return FE_OK;
  }
  const int keep_v = c->variant, keep_lz = c->lz;
  // the field the sweeps run on: u itself for the gradient sweep (read only);
  // for steps, a copy in `work` that ping-pongs with the context's buffer
  const size_t bytes = field_elems(c->grid) * elem_size(c->grid);
  void* tmp_m1 = nullptr;
  void* tmp_m2 = nullptr;
  int* tmp_t = nullptr;
  void* keep_m1 = c->d_m1;
  void* keep_m2 = c->d_m2;
  int* keep_t = c->d_adam_t;
  auto restore = [&]() {
    c->d_m1 = keep_m1;
    c->d_m2 = keep_m2;
    c->d_adam_t = keep_t;
    (void)hipStreamSynchronize(c->stream);
    for (void* p : {tmp_m1, tmp_m2, (void*)tmp_t})
      if (p) (void)hipFree(p);
  };
  if (kind != FE_TUNE_GRAD) {
    if (!c->d_pingpong && hipMalloc(&c->d_pingpong, bytes) != hipSuccess) {
      c->d_pingpong = nullptr;
      return set_error(FE_ENOMEM, "ping-pong field allocation failed");
    }
    FE_HIP(hipMemcpyAsync(work, u, bytes, hipMemcpyDeviceToDevice, c->stream));
  }
  if (kind == FE_TUNE_ADAM) {
    // temporary moments: the context's optimiser state is left as it is
    if (hipMalloc(&tmp_m1, bytes) != hipSuccess || hipMalloc(&tmp_m2, bytes) != hipSuccess ||
        hipMalloc((void**)&tmp_t, sizeof(int)) != hipSuccess) {
      restore();
      return set_error(FE_ENOMEM, "temporary Adam moment allocation failed");
    }
    c->d_m1 = tmp_m1;
    c->d_m2 = tmp_m2;
    c->d_adam_t = tmp_t;
    if ((rc = adam_reset_launch(c))) {
      restore();
      return rc;
    }
  }
  const StepRule rule{kind == FE_TUNE_ADAM ? fe::kStepAdam : fe::kStepGD, 1e-3, 0.9, 0.999, 1e-8};
  int flip = 0;
  auto launch = [&]() -> int {
    if (kind == FE_TUNE_GRAD) return fe_energy_grad_async(c, u, work, nullptr);
    // one step on the copy (no mass shift: the same kernel, without the first
    // wave's sum of its predecessor's partials)
    void* src = flip ? c->d_pingpong : work;
    void* dst = flip ? work : c->d_pingpong;
    flip ^= 1;
    return sweep(c, c->stream, rule.mode, src, dst, nullptr, partials_buf(c, 0), rule, 0);
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    restore();
    return set_error(FE_EHIP, "hipEventCreate failed");
  }
  // settle the clocks: 50 ms of the workload in the current launch shape
  {
    const auto t0 = std::chrono::steady_clock::now();
    while (rc == FE_OK && std::chrono::steady_clock::now() - t0 < std::chrono::milliseconds(50)) {
      for (int i = 0; i < 4 && rc == FE_OK; ++i) rc = launch();
      if (hipStreamSynchronize(c->stream) != hipSuccess) rc = set_error(FE_EHIP, "hipStreamSynchronize failed");
    }
  }
  double best = 1e300;
  int best_v = keep_v, best_lz = keep_lz;
  for (int v = 0; v < (int)variants().size() && rc == FE_OK; ++v) {
    if (!variant_ok(v, c->grid.dtype)) continue;
    const Variant& x = variants()[v];
    if (x.tx > 2 * c->grid.nx || x.ty > 2 * c->grid.ny) continue;
    if ((c->use_cfield && !has_sp(v, c->grid.dtype)) || (c->use_box && !has_box(v, c->grid.dtype))) continue;
    // z chunks: powers of two from 4, the equal-chunk length with as many
    // chunks as each, and the automatic choice
    std::vector<int> lzs;
    const int nz = c->grid.nz;
    for (int p = 4; p <= 128 && p <= nz; p *= 2) {
      lzs.push_back(p);
      lzs.push_back(ceil_div(nz, ceil_div(nz, p)));
    }
    lzs.push_back(geometry(c, v, 0, kind == FE_TUNE_GRAD ? (int)fe::kGrad : rule.mode).lz);
    std::sort(lzs.begin(), lzs.end());
    lzs.erase(std::unique(lzs.begin(), lzs.end()), lzs.end());
    for (int lz : lzs) {
      c->variant = v;
      c->lz = lz;
      rc = launch();   // warm-up
      if (rc) break;
      if (hipEventRecord(e0, c->stream) != hipSuccess) { rc = set_error(FE_EHIP, "hipEventRecord failed"); break; }
      for (int i = 0; i < iters && rc == FE_OK; ++i) rc = launch();
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
  restore();
  c->variant = rc ? keep_v : best_v;
  c->lz = rc ? keep_lz : best_lz;
  if (rc) return rc;
  tune_store(key, TuneEntry{best_v, best_lz, best});
  if (best_us) *best_us = best;
  return FE_OK;
}

int fe_tune_cache_save(const char* path) {
  g_last_error.clear();
  if (!path) return set_error(FE_EINVAL, "path is NULL");
  std::lock_guard<std::mutex> lock(g_tune_mu);
  FILE* f = std::fopen(path, "w");
  if (!f) return set_error(FE_EINVAL, "cannot open %s for writing", path);
  for (const auto& kv : g_tune_cache)
    std::fprintf(f, "%s %d %d %.6f\n", kv.first.c_str(), kv.second.variant, kv.second.lz, kv.second.us);
  const bool ok = std::fclose(f) == 0;
  return ok ? FE_OK : set_error(FE_EINVAL, "writing %s failed", path);
}

int fe_tune_cache_load(const char* path) {
  g_last_error.clear();
  if (!path) return set_error(FE_EINVAL, "path is NULL");
  FILE* f = std::fopen(path, "r");
  if (!f) return set_error(FE_EINVAL, "cannot open %s", path);
  std::map<std::string, TuneEntry> got;
  char line[512];
  int lineno = 0;
  int rc = FE_OK;
  while (std::fgets(line, sizeof(line), f)) {
    ++lineno;
    char key[400];
    TuneEntry e;
    if (line[0] == '\n' || line[0] == '#') continue;
    if (std::sscanf(line, "%399s %d %d %lf", key, &e.variant, &e.lz, &e.us) != 4 || e.variant < 0 ||
        e.variant >= (int)variants().size() || e.lz < 0) {
      rc = set_error(FE_EINVAL, "%s:%d: not a tuning record", path, lineno);
      break;
    }
    got[key] = e;
  }
  std::fclose(f);
  if (rc) return rc;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  for (const auto& kv : got) g_tune_cache[kv.first] = kv.second;
  return FE_OK;
}

void fe_tune_cache_clear(void) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune_cache.clear();
}

void fe_destroy(fe_ctx* c) {
  if (!c) return;
  DeviceGuard dg(c->device);
  drop_graphs(c);
  if (c->d_prm) (void)hipFree(c->d_prm);
  if (c->d_prm_scaled) (void)hipFree(c->d_prm_scaled);
  if (c->d_partials) (void)hipFree(c->d_partials);
  if (c->d_energy) (void)hipFree(c->d_energy);
  if (c->d_mass) (void)hipFree(c->d_mass);
  if (c->d_shift) (void)hipFree(c->d_shift);
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
