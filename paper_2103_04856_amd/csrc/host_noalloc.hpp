// The allocation-free energy + gradient entry point (fe_energy_grad_noalloc):
// the per-instance table and the block partials of the sweep live in one
// file-scope device array instead of context memory, so the call needs no
// context and allocates nothing. Included once by fe_api.hip.
#pragma once

#include <mutex>

namespace {

constexpr int kNoAllocMaxBatch = 16;
constexpr size_t kScratchBytes = size_t(1) << 20;      // 1 MiB per device
constexpr size_t kScratchPrmBytes = 4096;               // the per-instance table
constexpr size_t kScratchPartials =                     // block partials (two doubles each)
    (kScratchBytes - kScratchPrmBytes) / (2 * sizeof(double));
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

static_assert(kNoAllocMaxBatch * sizeof(fe::InstParams<double>) <= kScratchPrmBytes, "table area too small");

// The table travels by value in the kernel arguments (4 KiB at most), so
// filling it needs no host staging buffer and no copy call.
template <typename T>
struct ParamPack {
  fe::InstParams<T> p[kNoAllocMaxBatch];
};
static_assert(sizeof(ParamPack<double>) <= 4096, "kernel argument limit");

template <typename T>
__global__ __launch_bounds__(64) void store_params(ParamPack<T> pack, int batch, fe::InstParams<T>* dst) {
  const int b = threadIdx.x;
  if (b < batch) dst[b] = pack.p[b];
}

struct ScratchSlot {
  void* ptr = nullptr;   // device address of `scratch` on this device
  int num_cu = 0;
};
ScratchSlot g_scratch[kMaxDevices];
std::mutex g_scratch_mu;

// The device address of `scratch` on the current device (once per device:
// each device holds its own copy of the array at its own address) and its
// compute-unit count.
int scratch_slot(ScratchSlot& out) {
  int dev = -1;
  FE_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return set_error(FE_EINVAL, "device ordinal %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  ScratchSlot& s = g_scratch[dev];
  if (!s.ptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(FE_EHIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1) ncu = 256;
    s.num_cu = ncu;
    s.ptr = p;
  }
  out = s;
  return FE_OK;
}

template <typename T>
int noalloc_sweep(const fe_grid& grid, const double* eps, const double* a, const void* u, void* g,
                  double* energy_dev, hipStream_t stream, const ScratchSlot& slot) {
  const int vi = default_variant(grid);
  ParamPack<T> pack{};
  const double theta0[3] = {0.0, 0.0, 0.0};
  for (int b = 0; b < grid.batch; ++b) pack.p[b] = inst_params<T>(grid.h, eps[b], a + 6 * b, 0.0, theta0);
  const Variant& v = variants()[vi];
  const Kernels<T>& k = kernels_of<T>(v, false);
  const SweepFn<T> fn = sweep_kernel<T>(k, fe::kGrad, batch_body(pack.p, grid.batch));
  // z chunks from the blocks per compute unit of the kernel launched, as in a context
  int slots = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&slots, (const void*)fn, v.nt, 0) != hipSuccess || slots < 1)
    slots = 1;
  const Geometry geo = g ? geometry_of(grid, slot.num_cu, vi, 0, slots) : energy_geometry(grid, slot.num_cu);
  const size_t nblocks = (size_t)geo.per_inst * grid.batch;
  if (nblocks > kScratchPartials)
    return set_error(FE_EINVAL, "grid needs %zu block partials; the static scratch holds %zu", nblocks,
                     kScratchPartials);
  auto* prm = reinterpret_cast<fe::InstParams<T>*>(slot.ptr);
  double* partials = reinterpret_cast<double*>(static_cast<char*>(slot.ptr) + kScratchPrmBytes);
  hipLaunchKernelGGL(store_params<T>, dim3(1), dim3(64), 0, stream, pack, grid.batch, prm);
  FE_HIP(hipGetLastError());

  fe::SweepArgs<T> sa{};
  sa.src = static_cast<const T*>(u);
  sa.dst = static_cast<T*>(g);
  sa.prm = prm;
  sa.prev_partials = nullptr;
  sa.partials = partials;
  sa.mass = nullptr;
  sa.inv_nvox = 1.0 / ((double)grid.nx * grid.ny * grid.nz);
  sa.k = grid_consts<T>(grid.h);
  sa.nx = grid.nx;
  sa.ny = grid.ny;
  sa.nz = grid.nz;
  sa.ntx = geo.ntx;
  sa.nty = geo.nty;
  sa.nzc = geo.nzc;
  sa.lz = geo.lz;
  sa.batch = grid.batch;
  if (g) {
    hipLaunchKernelGGL(fn, dim3((unsigned)nblocks), dim3((unsigned)v.nt), 0, stream, sa);
    FE_HIP(hipGetLastError());
  } else {
    const int rc = launch_energy_cols<T>(grid, geo, u, prm, partials, stream);
    if (rc) return rc;
  }
  if (energy_dev) {
    hipLaunchKernelGGL(fe::sweep_finish, dim3(grid.batch), dim3(64), 0, stream, (const double*)partials,
                       geo.per_inst, energy_dev, (const double*)nullptr, sa.inv_nvox, (double*)nullptr);
    FE_HIP(hipGetLastError());
  }
  return FE_OK;
}

}  // namespace

extern "C" {

int fe_energy_grad_noalloc(const fe_grid* grid, const double* eps, const double* p_coeffs, const void* u, void* g,
                           double* energy_dev, void* stream) {
  g_last_error.clear();
  int rc = check_grid(grid);
  if (rc) return rc;
  if (grid->batch > kNoAllocMaxBatch)
    return set_error(FE_EINVAL, "batch %d exceeds the allocation-free limit of %d", grid->batch, kNoAllocMaxBatch);
  if ((rc = check_params(grid->batch, eps, p_coeffs))) return rc;
  if (!u) return set_error(FE_EINVAL, "u is NULL");
  if (g == u) return set_error(FE_EINVAL, "g must not alias u");
  if (!g && !energy_dev) return set_error(FE_EINVAL, "nothing to compute: g and energy_dev are both NULL");
  {
    // a bound that needs no device: at least one z chunk per tile column
    const Variant& v = variants()[default_variant(*grid)];
    const size_t cols = g ? (size_t)ceil_div(grid->nx, v.tx) * ceil_div(grid->ny, v.ty) * grid->batch
                          : (size_t)ceil_div(grid->nx, 64) *
                                ceil_div(grid->ny, energy_rows(grid->dtype) * kEnergyWaves) * grid->batch;
    if (cols > kScratchPartials)
      return set_error(FE_EINVAL, "grid needs at least %zu block partials; the static scratch holds %zu", cols,
                       kScratchPartials);
  }
  ScratchSlot slot;
  if ((rc = scratch_slot(slot))) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  return grid->dtype == FE_F32 ? noalloc_sweep<float>(*grid, eps, p_coeffs, u, g, energy_dev, s, slot)
                               : noalloc_sweep<double>(*grid, eps, p_coeffs, u, g, energy_dev, s, slot);
}

}  // extern "C"
