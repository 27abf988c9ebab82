// Kernels of the H^-1 flow of Algorithm 1 (Sec. 4.1): u = div A + m0, the
// periodic Gaussian blur, and Adam on the vector field A with
// dG/dA = -grad (k * dF/du). The energy and dF/du come from the fused sweep.
//
// Layout: scalar fields [batch][nz][ny][nx]; the vector field A and its Adam
// moments [batch][3][nz][ny][nx] (components x, y, z), x fastest. Central
// differences are the ones of the energy's stencils; their periodic transpose
// is minus themselves, which is where the minus sign of dG/dA comes from.
#pragma once

#include <hip/hip_runtime.h>

#include "fe_voxel.hpp"

namespace fe {

constexpr int kBlurMaxR = 16;   // at most 33 taps: blur widths up to 4 voxels

template <typename T>
struct BlurTaps {
  T w[2 * kBlurMaxR + 1];       // w[r + j], j = -r..r, even, summing to 1
  int r;
};

struct FieldDims {
  int nx, ny, nz, batch;
};

__device__ __forceinline__ int wrap_up(int v, int n) { return v >= n ? v - n : v; }
__device__ __forceinline__ int wrap_down(int v, int n) { return v < 0 ? v + n : v; }
__device__ __forceinline__ int wrap_any(int v, int n) {
  int r = v % n;
  return r < 0 ? r + n : r;
}

// u[b] = m0[b] + sum_a (A_a(i + e_a) - A_a(i - e_a)) / (2h).
// Grid: (ceil(nx/64), ceil(ny/4), nz * batch), block (64, 4).
template <typename T>
__global__ __launch_bounds__(256) void div_field(const T* __restrict__ A, T* __restrict__ u,
                                                 const double* __restrict__ m0, FieldDims d, T inv2h) {
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int y = blockIdx.y * 4 + threadIdx.y;
  const int z = blockIdx.z % d.nz, b = blockIdx.z / d.nz;
  if (x >= d.nx || y >= d.ny) return;
  const size_t plane = (size_t)d.nx * d.ny, vol = plane * d.nz;
  const T* Ax = A + (size_t)b * 3 * vol;
  const T* Ay = Ax + vol;
  const T* Az = Ay + vol;
  const size_t row = (size_t)z * plane + (size_t)y * d.nx;
  const int xp = wrap_up(x + 1, d.nx), xm = wrap_down(x - 1, d.nx);
  const size_t yp = (size_t)z * plane + (size_t)wrap_up(y + 1, d.ny) * d.nx;
  const size_t ym = (size_t)z * plane + (size_t)wrap_down(y - 1, d.ny) * d.nx;
  const size_t zp = (size_t)wrap_up(z + 1, d.nz) * plane + (size_t)y * d.nx;
  const size_t zm = (size_t)wrap_down(z - 1, d.nz) * plane + (size_t)y * d.nx;
  const T s = (Ax[row + xp] - Ax[row + xm]) + (Ay[yp + x] - Ay[ym + x]) + (Az[zp + x] - Az[zm + x]);
  u[(size_t)b * vol + row + x] = T(m0[b]) + s * inv2h;
}

// Blur along x: one block per (row, 256-wide chunk); the row segment and its
// periodic halo of r are staged in LDS. Grid: (ceil(nx/256), ny, nz * batch).
template <typename T>
__global__ __launch_bounds__(256) void blur_x(const T* __restrict__ in, T* __restrict__ out, FieldDims d,
                                              BlurTaps<T> k) {
  __shared__ T s[256 + 2 * kBlurMaxR];
  const int x0 = blockIdx.x * 256;
  const size_t row = ((size_t)blockIdx.z * d.ny + blockIdx.y) * d.nx;   // blockIdx.z = b * nz + z
  const T* src = in + row;
  for (int e = threadIdx.x; e < 256 + 2 * k.r; e += 256) s[e] = src[wrap_any(x0 - k.r + e, d.nx)];
  __syncthreads();
  const int x = x0 + threadIdx.x;
  if (x >= d.nx) return;
  T acc = T(0);
  for (int j = 0; j <= 2 * k.r; ++j) acc += k.w[j] * s[threadIdx.x + j];
  out[row + x] = acc;
}

// Blur along y (AXIS = 1) or z (AXIS = 2): a block covers 64 x-values and 64
// positions along the axis, with the halo of r staged in LDS.
// Grid: (ceil(nx/64), ceil(n_axis/64), n_other * batch), block (64, 4);
// the other axis is z for AXIS = 1 and y for AXIS = 2.
template <typename T, int AXIS>
__global__ __launch_bounds__(256) void blur_yz(const T* __restrict__ in, T* __restrict__ out, FieldDims d,
                                               BlurTaps<T> k) {
  __shared__ T s[64 + 2 * kBlurMaxR][64];
  const int n_axis = AXIS == 1 ? d.ny : d.nz;
  const int n_other = AXIS == 1 ? d.nz : d.ny;
  const size_t stride = AXIS == 1 ? (size_t)d.nx : (size_t)d.nx * d.ny;
  const int other = blockIdx.z % n_other, b = blockIdx.z / n_other;
  const size_t base = (size_t)b * d.nz * d.ny * d.nx +
                      (AXIS == 1 ? (size_t)other * d.nx * d.ny : (size_t)other * d.nx);
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int p0 = blockIdx.y * 64;
  const bool xin = x < d.nx;
  for (int q = threadIdx.y; q < 64 + 2 * k.r; q += 4)
    s[q][threadIdx.x] = xin ? in[base + (size_t)wrap_any(p0 - k.r + q, n_axis) * stride + x] : T(0);
  __syncthreads();
  if (!xin) return;
  for (int q = threadIdx.y; q < 64; q += 4) {
    const int p = p0 + q;
    if (p >= n_axis) break;
    T acc = T(0);
    for (int j = 0; j <= 2 * k.r; ++j) acc += k.w[j] * s[q + j][threadIdx.x];
    out[base + (size_t)p * stride + x] = acc;
  }
}

// Adam on A with dG/dA_a = -(g(i + e_a) - g(i - e_a)) / (2h), g = k * dF/du.
// Moments and A are updated in place; t >= 1 is read from device memory.
// Grid and block as div_field.
template <typename T>
__global__ __launch_bounds__(256) void adam_vector_field(const T* __restrict__ g, T* __restrict__ A,
                                                         T* __restrict__ m1, T* __restrict__ m2, FieldDims d,
                                                         T inv2h, T lr, T beta1, T beta2, T adam_eps,
                                                         const int* __restrict__ adam_t) {
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int y = blockIdx.y * 4 + threadIdx.y;
  const int z = blockIdx.z % d.nz, b = blockIdx.z / d.nz;
  if (x >= d.nx || y >= d.ny) return;
  const int t = *adam_t;
  const T bc1 = T(1.0 / (1.0 - ::pow(double(beta1), double(t))));
  const T bc2 = T(1.0 / (1.0 - ::pow(double(beta2), double(t))));
  const size_t plane = (size_t)d.nx * d.ny, vol = plane * d.nz;
  const T* gb = g + (size_t)b * vol;
  const size_t row = (size_t)z * plane + (size_t)y * d.nx;
  T grad[3];
  grad[0] = -(gb[row + wrap_up(x + 1, d.nx)] - gb[row + wrap_down(x - 1, d.nx)]) * inv2h;
  grad[1] = -(gb[(size_t)z * plane + (size_t)wrap_up(y + 1, d.ny) * d.nx + x] -
              gb[(size_t)z * plane + (size_t)wrap_down(y - 1, d.ny) * d.nx + x]) * inv2h;
  grad[2] = -(gb[(size_t)wrap_up(z + 1, d.nz) * plane + (size_t)y * d.nx + x] -
              gb[(size_t)wrap_down(z - 1, d.nz) * plane + (size_t)y * d.nx + x]) * inv2h;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const size_t i = ((size_t)b * 3 + a) * vol + row + x;
    const T mo = beta1 * m1[i] + (T(1) - beta1) * grad[a];
    const T vo = beta2 * m2[i] + (T(1) - beta2) * grad[a] * grad[a];
    m1[i] = mo;
    m2[i] = vo;
    A[i] -= lr * (mo * bc1) * rcp_t(sqrt_t(vo * bc2) + adam_eps);
  }
}

__global__ __launch_bounds__(64) void bump_counter(int* t) {
  if (threadIdx.x == 0) atomicAdd(t, 1);
}

}  // namespace fe
