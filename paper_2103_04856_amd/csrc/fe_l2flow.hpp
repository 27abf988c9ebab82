// Device pieces of Algorithm 2 (Sec. 4.2): the L2 flow of F_h(k * u) with
// replicate boundary conditions, driven by L-BFGS.
//
// The box field lives inside a padded array (pad width W on every side); the
// padding holds copies of the nearest box voxel (replicate padding) whenever a
// stencil or the blur reads it. The sweep then runs on the padded array as a
// periodic field with a box mask, and the derivatives that land on pad samples
// are added back onto the box voxels they copy (the transpose of the padding).
// Vectors of the optimiser use the same padded layout with zero padding.
#pragma once

#include <hip/hip_runtime.h>

#include "fe_kernels.hpp"

namespace fe {

struct PadBox {
  int nx, ny, nz;          // padded array
  int lo[3], hi[3];        // box [lo, hi) in x, y, z
};

__device__ __forceinline__ int clamp_to(int v, int lo, int hi) { return v < lo ? lo : (v >= hi ? hi - 1 : v); }

// Launch shape of the padding kernels: one thread per sample of a row of 256,
// grid (ceil(nx/256), ny, nz).
// Fill every pad sample with the nearest box voxel (reads box voxels only).
template <typename T>
__global__ __launch_bounds__(256) void pad_replicate(T* __restrict__ f, PadBox b) {
  const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
  if (x >= b.nx) return;
  const int cx = clamp_to(x, b.lo[0], b.hi[0]), cy = clamp_to(y, b.lo[1], b.hi[1]), cz = clamp_to(z, b.lo[2], b.hi[2]);
  if (cx != x || cy != y || cz != z)
    f[((size_t)z * b.ny + y) * b.nx + x] = f[((size_t)cz * b.ny + cy) * b.nx + cx];
}

// out = P^T g: every box voxel gathers the pad samples that copy it (on a box
// face, the whole run of pad samples beyond it along each clamped axis); pad
// samples of out are zero. g and out must differ.
template <typename T>
__global__ __launch_bounds__(256) void fold_pads(const T* __restrict__ g, T* __restrict__ out, PadBox b) {
  const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
  if (x >= b.nx) return;
  const size_t i = ((size_t)z * b.ny + y) * b.nx + x;
  const bool in = x >= b.lo[0] && x < b.hi[0] && y >= b.lo[1] && y < b.hi[1] && z >= b.lo[2] && z < b.hi[2];
  if (!in) {
    out[i] = T(0);
    return;
  }
  const int x0 = x == b.lo[0] ? 0 : x, x1 = x == b.hi[0] - 1 ? b.nx - 1 : x;
  const int y0 = y == b.lo[1] ? 0 : y, y1 = y == b.hi[1] - 1 ? b.ny - 1 : y;
  const int z0 = z == b.lo[2] ? 0 : z, z1 = z == b.hi[2] - 1 ? b.nz - 1 : z;
  if (x0 == x1 && y0 == y1 && z0 == z1) {
    out[i] = g[i];
    return;
  }
  T acc = T(0);
  for (int zz = z0; zz <= z1; ++zz)
    for (int yy = y0; yy <= y1; ++yy)
      for (int xx = x0; xx <= x1; ++xx) acc += g[((size_t)zz * b.ny + yy) * b.nx + xx];
  out[i] = acc;
}

// ---- vector operations of the optimiser (FP64 reductions, fixed order) ----

constexpr int kVecBlocks = 1024;

template <int OP>
__device__ __forceinline__ double vec_combine(double acc, double v) {
  return OP == 2 ? fmax(acc, v) : acc + v;
}

// partial[k] for block k: sum of a*b (OP 0), |a| (OP 1), or max |a| (OP 2).
// Each thread keeps four independent accumulators over four strided elements
// per round, so four loads are in flight; the fixed grid and fixed order keep
// the result deterministic.
template <typename T, int OP>
__global__ __launch_bounds__(256) void vec_reduce(const T* __restrict__ a, const T* __restrict__ b, size_t n,
                                                  double* __restrict__ partial) {
  __shared__ double s[256];
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const size_t j = i + k * stride;
      const double v = OP == 0 ? double(a[j]) * double(b[j]) : fabs(double(a[j]));
      acc[k] = vec_combine<OP>(acc[k], v);
    }
  }
  for (; i < n; i += stride) {
    const double v = OP == 0 ? double(a[i]) * double(b[i]) : fabs(double(a[i]));
    acc[0] = vec_combine<OP>(acc[0], v);
  }
  s[threadIdx.x] = vec_combine<OP>(vec_combine<OP>(acc[0], acc[1]), vec_combine<OP>(acc[2], acc[3]));
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) s[threadIdx.x] = OP == 2 ? fmax(s[threadIdx.x], s[threadIdx.x + w]) : s[threadIdx.x] + s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = s[0];
}

// out[0] = reduction of the nblk partials (one block, fixed order); the result may
// go to any slot of a device scalar array.
template <int OP>
__global__ __launch_bounds__(256) void vec_finish(const double* __restrict__ partial, int nblk, double* __restrict__ out) {
  __shared__ double s[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nblk; i += 256) acc = OP == 2 ? fmax(acc, partial[i]) : acc + partial[i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) s[threadIdx.x] = OP == 2 ? fmax(s[threadIdx.x], s[threadIdx.x + w]) : s[threadIdx.x] + s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = s[0];
}

// y = alpha x + beta y  (alpha and beta in the vector precision, as the vectors are)
template <typename T>
__global__ __launch_bounds__(256) void vec_axpby(T alpha, const T* __restrict__ x, T beta, T* __restrict__ y, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] = alpha * x[i] + beta * y[i];
}

// y = (ka sc[ia] + kb sc[ib]) x + y, the coefficient formed from device scalars
// (ib < 0: no second term), so that the two-loop recursion needs no host sync.
template <typename T>
__global__ __launch_bounds__(256) void vec_axpy_dev(const double* __restrict__ sc, int ia, double ka, int ib,
                                                    double kb, const T* __restrict__ x, T* __restrict__ y,
                                                    size_t n) {
  const T alpha = T(ka * sc[ia] + (ib >= 0 ? kb * sc[ib] : 0.0));
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] = alpha * x[i] + y[i];
}

// z = x - y
template <typename T>
__global__ __launch_bounds__(256) void vec_sub(const T* __restrict__ x, const T* __restrict__ y, T* __restrict__ z,
                                               size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    z[i] = x[i] - y[i];
}

// Copy between the box of a padded array and a dense box field [nz][ny][nx].
template <typename T>
__global__ __launch_bounds__(256) void box_copy(const T* __restrict__ src, T* __restrict__ dst, PadBox b,
                                                int to_padded) {
  const int bx = b.hi[0] - b.lo[0], by = b.hi[1] - b.lo[1], bz = b.hi[2] - b.lo[2];
  const size_t n = (size_t)bx * by * bz;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const int x = (int)(i % bx), y = (int)((i / bx) % by), z = (int)(i / ((size_t)bx * by));
    const size_t pi = ((size_t)(z + b.lo[2]) * b.ny + (y + b.lo[1])) * b.nx + (x + b.lo[0]);
    if (to_padded) dst[pi] = src[i];
    else dst[i] = src[pi];
  }
}

}  // namespace fe
