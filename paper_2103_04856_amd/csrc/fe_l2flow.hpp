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

// Fill every pad sample with the nearest box voxel (reads box voxels only).
// Threads enumerate the pad shell alone, in three regions: the planes below
// and above the box in z, then within the box's z range the rows below and
// above it in y, then within the box's y and z ranges the runs left and right
// of it in x. Grid: ceil(shell / 256) blocks of 256 (pad_shell_size).
__host__ __device__ __forceinline__ size_t pad_shell_size(const PadBox& b) {
  const size_t bx = b.hi[0] - b.lo[0], by = b.hi[1] - b.lo[1], bz = b.hi[2] - b.lo[2];
  const size_t px = b.nx - bx, py = b.ny - by, pz = b.nz - bz;
  return pz * b.ny * b.nx + bz * py * b.nx + bz * by * px;
}

template <typename T>
__global__ __launch_bounds__(256) void pad_replicate(T* __restrict__ f, PadBox b) {
  const size_t bx = b.hi[0] - b.lo[0], by = b.hi[1] - b.lo[1], bz = b.hi[2] - b.lo[2];
  const size_t px = b.nx - bx, py = b.ny - by, pz = b.nz - bz;
  const size_t nA = pz * b.ny * b.nx, nB = bz * py * b.nx, nC = bz * by * px;
  size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  int x, y, z;
  if (j < nA) {
    const size_t plane = (size_t)b.nx * b.ny;
    const int k = (int)(j / plane), r = (int)(j % plane);
    z = k < b.lo[2] ? k : b.hi[2] + (k - b.lo[2]);
    y = r / b.nx;
    x = r % b.nx;
  } else if ((j -= nA) < nB) {
    const size_t per = py * b.nx;
    const int k = (int)(j / per), r = (int)(j % per);
    const int ky = r / b.nx;
    z = b.lo[2] + k;
    y = ky < b.lo[1] ? ky : b.hi[1] + (ky - b.lo[1]);
    x = r % b.nx;
  } else if ((j -= nB) < nC) {
    const int row = (int)(j / px), kx = (int)(j % px);
    z = b.lo[2] + row / (int)by;
    y = b.lo[1] + row % (int)by;
    x = kx < b.lo[0] ? kx : b.hi[0] + (kx - b.lo[0]);
  } else {
    return;
  }
  const int cx = clamp_to(x, b.lo[0], b.hi[0]), cy = clamp_to(y, b.lo[1], b.hi[1]), cz = clamp_to(z, b.lo[2], b.hi[2]);
  f[((size_t)z * b.ny + y) * b.nx + x] = f[((size_t)cz * b.ny + cy) * b.nx + cx];
}

// out = P^T g: every box voxel gathers the pad samples that copy it (on a box
// face, the run of pad samples beyond it along each clamped axis, the voxel
// included); pad samples of out are zero; voxels off the box surface copy g.
// W > 0: every pad is W wide, so a run on one face is W + 1 samples at fixed
// offsets (unrolled, all loads in flight); W = 0: general runs. Edges and
// corners (two or three clamped axes) take the general loop. One thread per
// sample of a plane: grid (ceil(nx ny / 256), nz). g and out must differ.
template <typename T, int W>
__global__ __launch_bounds__(256) void fold_pads(const T* __restrict__ g, T* __restrict__ out, PadBox b) {
  const int ip = blockIdx.x * 256 + threadIdx.x, z = blockIdx.y;
  if (ip >= b.nx * b.ny) return;
  const int y = ip / b.nx, x = ip - y * b.nx;
  const size_t i = (size_t)z * b.nx * b.ny + ip;
  const bool in = x >= b.lo[0] && x < b.hi[0] && y >= b.lo[1] && y < b.hi[1] && z >= b.lo[2] && z < b.hi[2];
  if (!in) {
    out[i] = T(0);
    return;
  }
  const bool fx = x == b.lo[0] || x == b.hi[0] - 1, fy = y == b.lo[1] || y == b.hi[1] - 1,
             fz = z == b.lo[2] || z == b.hi[2] - 1;
  const int nf = int(fx) + int(fy) + int(fz);
  if (nf == 0) {
    out[i] = g[i];
    return;
  }
  if (W > 0 && nf == 1) {
    // the run from the voxel outwards along its one clamped axis
    const int lo = fx ? b.lo[0] : fy ? b.lo[1] : b.lo[2];
    const int c = fx ? x : fy ? y : z;
    const long step = fx ? 1 : fy ? (long)b.nx : (long)b.nx * b.ny;
    const long dir = c == lo ? -step : step;
    T v[W + 1];
#pragma unroll
    for (int k = 0; k <= W; ++k) v[k] = g[(long)i + k * dir];
    T acc = T(0);                // in increasing index order, as the general loop adds
    if (dir < 0) {
#pragma unroll
      for (int k = W; k >= 0; --k) acc += v[k];
    } else {
#pragma unroll
      for (int k = 0; k <= W; ++k) acc += v[k];
    }
    out[i] = acc;
    return;
  }
  const int x0 = x == b.lo[0] ? 0 : x, x1 = x == b.hi[0] - 1 ? b.nx - 1 : x;
  const int y0 = y == b.lo[1] ? 0 : y, y1 = y == b.hi[1] - 1 ? b.ny - 1 : y;
  const int z0 = z == b.lo[2] ? 0 : z, z1 = z == b.hi[2] - 1 ? b.nz - 1 : z;
  T acc = T(0);
  for (int zz = z0; zz <= z1; ++zz)
    for (int yy = y0; yy <= y1; ++yy)
      for (int xx = x0; xx <= x1; ++xx) acc += g[((size_t)zz * b.ny + yy) * b.nx + xx];
  out[i] = acc;
}

// ---- vector operations of the optimiser (FP64 reductions, fixed order) ----
//
// Every reduction runs on kVecBlocks blocks of kVecThreads threads and leaves
// one FP64 partial per block in a bank of its own. The value of a reduction is
// the combination of its bank in one fixed order (bank_value), formed where it
// is needed: by every block of a later vector pass that takes it as a
// coefficient, or by vec_finish for the host. No block waits for another and
// no pass needs a device-wide fence, which on this GPU costs more than the
// pass itself when every block issues one.

constexpr int kVecBlocks = 256;
constexpr int kVecThreads = 1024;

template <int OP>
__device__ __forceinline__ double vec_combine(double acc, double v) {
  return OP == 2 ? fmax(acc, v) : acc + v;
}

// The value of a bank of kVecBlocks partials: lane l of the block's first wave
// combines partials l, l + 64, l + 128, l + 192 in that order, then a butterfly
// over the wave (each step combines a lane with its partner, and the two orders
// of a commutative operation agree bit for bit, so all lanes finish equal).
// The result is broadcast to the whole block; call from every thread.
template <int OP>
__device__ __forceinline__ double bank_value(const double* __restrict__ bank) {
  static_assert(kVecBlocks == 4 * 64, "bank_value reads four partials per lane");
  __shared__ double s_val;
  if (threadIdx.x < 64) {
    double a = bank[threadIdx.x];
    a = vec_combine<OP>(a, bank[threadIdx.x + 64]);
    a = vec_combine<OP>(a, bank[threadIdx.x + 128]);
    a = vec_combine<OP>(a, bank[threadIdx.x + 192]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) a = vec_combine<OP>(a, __shfl_xor(a, off, 64));
    if (threadIdx.x == 0) s_val = a;
  }
  __syncthreads();
  const double v = s_val;
  __syncthreads();   // s_val may be reused by a later call
  return v;
}

// The block's combination of one value per thread into bank[blockIdx.x], in a
// fixed order (each wave's butterfly, then the waves in order).
template <int OP>
__device__ __forceinline__ void vec_block_partial(double acc, double* __restrict__ bank) {
  __shared__ double s_w[kVecThreads / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc = vec_combine<OP>(acc, __shfl_xor(acc, off, 64));
  if (threadIdx.x % 64 == 0) s_w[threadIdx.x / 64] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = s_w[0];
    for (int k = 1; k < kVecThreads / 64; ++k) a = vec_combine<OP>(a, s_w[k]);
    bank[blockIdx.x] = a;
  }
}

// Four consecutive vector elements, moved with 16-byte loads and stores (the
// vectors are whole device allocations, so element 4k is 16-byte aligned).
template <typename T>
struct alignas(16) Pack4 {
  T v[4];
};

// bank <- partials of sum a*b (OP 0), sum |a| (OP 1) or max |a| (OP 2),
// accumulated in FP64 with one accumulator per element of a pack. Grid-stride
// over packs of four, two packs of each vector in flight per thread; block 0
// takes the n % 4 tail.
template <typename T, int OP>
__global__ __launch_bounds__(kVecThreads) void vec_reduce(const T* __restrict__ a, const T* __restrict__ b, size_t n,
                                                          double* __restrict__ bank) {
  const size_t n4 = n / 4, stride = (size_t)gridDim.x * blockDim.x;
  const Pack4<T>* pa = reinterpret_cast<const Pack4<T>*>(a);
  const Pack4<T>* pb = reinterpret_cast<const Pack4<T>*>(b);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (size_t i0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i0 < n4; i0 += 2 * stride) {
    Pack4<T> va[2], vb[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const size_t i = i0 + u * stride;
      va[u] = Pack4<T>{};
      vb[u] = Pack4<T>{};
      if (i < n4) {
        va[u] = pa[i];
        if (OP == 0) vb[u] = pb[i];
      }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int k = 0; k < 4; ++k)
        acc[k] = vec_combine<OP>(acc[k], OP == 0 ? double(va[u].v[k]) * double(vb[u].v[k]) : fabs(double(va[u].v[k])));
  }
  if (blockIdx.x == 0 && threadIdx.x < n - 4 * n4) {
    const size_t j = 4 * n4 + threadIdx.x;
    acc[0] = vec_combine<OP>(acc[0], OP == 0 ? double(a[j]) * double(b[j]) : fabs(double(a[j])));
  }
  vec_block_partial<OP>(vec_combine<OP>(vec_combine<OP>(acc[0], acc[1]), vec_combine<OP>(acc[2], acc[3])), bank);
}

// Coefficient of a vector pass, ka v(bank_a) + kb v(bank_b) + kc in FP64, from
// the values of two dot-product banks (a null bank: that term is absent).
struct VecCoef {
  const double* bank_a;
  double ka;
  const double* bank_b;
  double kb;
  double kc;
};

// y = alpha x + y (ACC) or y = alpha x, alpha = the coefficient rounded once to
// the vector precision; then, when w is given, bank <- partials of w . y (the
// updated y). Each step of the L-BFGS two-loop recursion is one such pass: the
// update by one history entry and the dot product that the next entry needs,
// with no host synchronisation. Layout of the work as in vec_reduce.
template <typename T, bool ACC>
__global__ __launch_bounds__(kVecThreads) void vec_update_dot(VecCoef cf, const T* __restrict__ x, T* __restrict__ y,
                                                              const T* __restrict__ w, size_t n,
                                                              double* __restrict__ bank) {
  const double ca = cf.bank_a ? bank_value<0>(cf.bank_a) : 0.0;
  const double cb = cf.bank_b ? bank_value<0>(cf.bank_b) : 0.0;
  const T alpha = T(cf.ka * ca + cf.kb * cb + cf.kc);
  const size_t n4 = n / 4, stride = (size_t)gridDim.x * blockDim.x;
  const Pack4<T>* px = reinterpret_cast<const Pack4<T>*>(x);
  Pack4<T>* py = reinterpret_cast<Pack4<T>*>(y);
  const Pack4<T>* pw = reinterpret_cast<const Pack4<T>*>(w);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (size_t i0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i0 < n4; i0 += 2 * stride) {
    Pack4<T> vx[2], vy[2], vw[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const size_t i = i0 + u * stride;
      vx[u] = vy[u] = vw[u] = Pack4<T>{};
      if (i < n4) {
        vx[u] = px[i];
        if (ACC) vy[u] = py[i];
        if (w) vw[u] = pw[i];
      }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const size_t i = i0 + u * stride;
      Pack4<T> r;
#pragma unroll
      for (int k = 0; k < 4; ++k) r.v[k] = ACC ? alpha * vx[u].v[k] + vy[u].v[k] : alpha * vx[u].v[k];
      if (i < n4) {
        py[i] = r;
        if (w) {
#pragma unroll
          for (int k = 0; k < 4; ++k) acc[k] += double(vw[u].v[k]) * double(r.v[k]);
        }
      }
    }
  }
  if (blockIdx.x == 0 && threadIdx.x < n - 4 * n4) {
    const size_t j = 4 * n4 + threadIdx.x;
    const T v = ACC ? alpha * x[j] + y[j] : alpha * x[j];
    y[j] = v;
    if (w) acc[0] += double(w[j]) * double(v);
  }
  if (w) vec_block_partial<0>((acc[0] + acc[1]) + (acc[2] + acc[3]), bank);
}

// Values of up to four banks for the host: out[k] = bank_value<op[k]>(bank[k]).
struct BankList {
  const double* bank[4];
  double* out[4];
  int op[4];
  int count;
};

__global__ __launch_bounds__(64) void vec_finish(BankList l) {
  for (int k = 0; k < l.count; ++k) {
    const double v = l.op[k] == 2 ? bank_value<2>(l.bank[k]) : bank_value<0>(l.bank[k]);
    if (threadIdx.x == 0) *l.out[k] = v;
  }
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
