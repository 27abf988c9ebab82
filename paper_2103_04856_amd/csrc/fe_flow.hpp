// Kernels of the H^-1 flow of Algorithm 1 (Sec. 4.1): u = div A + m0, the
// periodic Gaussian blur, and Adam on the vector field A with
// dG/dA = -grad (k * dF/du). The energy and dF/du come from the fused sweep.
//
// Layout: scalar fields [batch][nz][ny][nx]; the vector field A and its Adam
// moments [batch][3][nz][ny][nx] (components x, y, z), x fastest. Central
// differences are the ones of the energy's stencils; their periodic transpose
// is minus themselves, which is where the minus sign of dG/dA comes from.
//
// One iteration is: blur_x<DIV> (div A + m0, blurred along x), blur_axis<1>,
// blur_axis<2>, the sweep, blur_x of dF/du, blur_axis<1>, blur_axis<2>,
// adam_vector_field; for the radii 4 and 8 the blur of dF/du runs blur_xy
// (x and y in one pass) and adam_zblur (the z pass fused with Adam). Without blur (r = 0) only the first kernel, the sweep and the
// Adam kernel run. Every kernel is a 64-wide row of x per wave, so loads
// and stores are coalesced; the blur halos are staged in LDS.
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

// Adam step number of the flow and its bias corrections 1 / (1 - beta^t),
// advanced once per iteration by the iteration's first kernel.
struct FlowClock {
  int t;
  int pad;
  double bc1, bc2;
};

__device__ __forceinline__ int wrap_any(int v, int n) {
  int r = v % n;
  return r < 0 ? r + n : r;
}
__device__ __forceinline__ int wrap_up(int v, int n) { return v >= n ? v - n : v; }
__device__ __forceinline__ int wrap_down(int v, int n) { return v < 0 ? v + n : v; }

// The blur kernels take the radius as a template argument R for the common
// widths (sigma_k = 1 and 2 give r = 4 and 8), so their tap loops are fixed;
// R = -1 is the general form, whose loops run to the largest radius under a
// uniform guard. Either way the taps are read at fixed offsets (kernel
// arguments in scalar registers), never indexed at run time.
template <int R>
constexpr int radius_bound() { return R >= 0 ? R : kBlurMaxR; }

// sum_j w_j v[j * step], j = 0..2r
template <typename T, int R>
__device__ __forceinline__ T taps_dot(const BlurTaps<T>& k, const T* v, int step) {
  T acc = T(0);
#pragma unroll
  for (int j = 0; j <= 2 * radius_bound<R>(); ++j)
    if (R >= 0 || j <= 2 * k.r) acc += k.w[j] * v[j * step];
  return acc;
}

// Blur along x of row segments: a block is kBlurRows rows x 64 x-values
// (block (64, 4), each thread on kBlurRows / 4 rows; grid (ceil(nx/64),
// ceil(ny/kBlurRows), nz * batch)); each row's segment and its periodic halo
// of r go through LDS. With DIV the loaded value is div A + m0 (the field of
// Algorithm 1; m(x) from mfield instead of the instance's m0 when given, the
// space-dependent mass of Sec. 5.2) and block (0,0,0) advances the clock (when
// given); without, it is in[]. r = 0 is a plain copy (or div). All loads of a thread are issued
// before the first LDS write, so a block keeps many in flight.
constexpr int kBlurRows = 16;

template <typename T, bool DIV, int R = -1>
__global__ __launch_bounds__(256) void blur_x(const T* __restrict__ in, T* __restrict__ out,
                                              const double* __restrict__ m0, const T* __restrict__ mfield,
                                              FieldDims d, T inv2h, BlurTaps<T> k, FlowClock* __restrict__ clk,
                                              double beta1, double beta2) {
  constexpr int kW = 64 + 2 * kBlurMaxR;
  constexpr int kPer = (kW + 63) / 64;          // segment elements per thread and row
  constexpr int kR = kBlurRows / 4;             // rows per thread
  __shared__ T s[kBlurRows][kW];
  if (DIV && clk && blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && threadIdx.x == 0 &&
      threadIdx.y == 0) {
    const int t = clk->t + 1;
    clk->t = t;
    clk->bc1 = 1.0 / (1.0 - ::pow(beta1, (double)t));
    clk->bc2 = 1.0 / (1.0 - ::pow(beta2, (double)t));
  }
  const int z = blockIdx.z % d.nz, b = blockIdx.z / d.nz;
  const int x0 = blockIdx.x * 64;
  const size_t plane = (size_t)d.nx * d.ny, vol = plane * d.nz;
  const T* base = in + (size_t)b * (DIV ? 3 : 1) * vol;
  const int r = R >= 0 ? R : k.r;
  const int nseg = 64 + 2 * r;
  T v[kR][kPer][7];          // the non-DIV form uses [0] only; [6] holds m(x)
#pragma unroll
  for (int i = 0; i < kR; ++i) {
    const int y = blockIdx.y * kBlurRows + threadIdx.y + 4 * i;
    if (y >= d.ny) continue;
    const size_t row = (size_t)z * plane + (size_t)y * d.nx;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int e = threadIdx.x + 64 * j;
      if (e >= nseg) continue;
      const int x = wrap_any(x0 - r + e, d.nx);
      if (DIV) {
        v[i][j][0] = base[row + wrap_up(x + 1, d.nx)];
        v[i][j][1] = base[row + wrap_down(x - 1, d.nx)];
        const T* Ay = base + vol;
        const T* Az = base + 2 * vol;
        v[i][j][2] = Ay[(size_t)z * plane + (size_t)wrap_up(y + 1, d.ny) * d.nx + x];
        v[i][j][3] = Ay[(size_t)z * plane + (size_t)wrap_down(y - 1, d.ny) * d.nx + x];
        v[i][j][4] = Az[(size_t)wrap_up(z + 1, d.nz) * plane + (size_t)y * d.nx + x];
        v[i][j][5] = Az[(size_t)wrap_down(z - 1, d.nz) * plane + (size_t)y * d.nx + x];
        if (mfield) v[i][j][6] = mfield[(size_t)b * vol + row + x];
      } else {
        v[i][j][0] = base[row + x];
      }
    }
  }
  const T mass = (DIV && !mfield) ? T(m0[b]) : T(0);
#pragma unroll
  for (int i = 0; i < kR; ++i) {
    const int y = blockIdx.y * kBlurRows + threadIdx.y + 4 * i;
    if (y >= d.ny) continue;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int e = threadIdx.x + 64 * j;
      if (e >= nseg) continue;
      if (DIV)
        s[threadIdx.y + 4 * i][e] =
            (mfield ? v[i][j][6] : mass) +
            ((v[i][j][0] - v[i][j][1]) + (v[i][j][2] - v[i][j][3]) + (v[i][j][4] - v[i][j][5])) * inv2h;
      else
        s[threadIdx.y + 4 * i][e] = v[i][j][0];
    }
  }
  __syncthreads();
  const int x = x0 + threadIdx.x;
  if (x >= d.nx) return;
#pragma unroll
  for (int i = 0; i < kR; ++i) {
    const int y = blockIdx.y * kBlurRows + threadIdx.y + 4 * i;
    if (y >= d.ny) continue;
    out[(size_t)b * vol + (size_t)z * plane + (size_t)y * d.nx + x] =
        taps_dot<T, R>(k, &s[threadIdx.y + 4 * i][threadIdx.x], 1);
  }
}

// Blur along y (AXIS = 1) or z (AXIS = 2) with a register window: each thread
// owns kAxisChunk consecutive outputs of one column, loads that segment and
// its periodic halo of r once (coalesced across the 64 x-lanes of a wave) and
// forms every output from registers, so the pass needs no LDS. Block (64, 4),
// one column per thread; grid (ceil(nx/64), ceil(n_axis/kAxisChunk),
// ceil(n_other/4) * batch), the other axis being z for AXIS = 1 and y for
// AXIS = 2.
constexpr int kAxisChunk = 16;

template <typename T, int AXIS, int R = -1>
__global__ __launch_bounds__(256) void blur_axis(const T* __restrict__ in, T* __restrict__ out, FieldDims d,
                                                 BlurTaps<T> k) {
  constexpr int kWin = kAxisChunk + 2 * radius_bound<R>();
  const int r = R >= 0 ? R : k.r;
  const int n_axis = AXIS == 1 ? d.ny : d.nz;
  const int n_other = AXIS == 1 ? d.nz : d.ny;
  const int og = (n_other + 3) / 4;
  const int other = (blockIdx.z % og) * 4 + threadIdx.y, b = blockIdx.z / og;
  const int x = blockIdx.x * 64 + threadIdx.x;
  if (x >= d.nx || other >= n_other) return;
  const size_t stride = AXIS == 1 ? (size_t)d.nx : (size_t)d.nx * d.ny;
  const size_t base = (size_t)b * d.nz * d.ny * d.nx +
                      (AXIS == 1 ? (size_t)other * d.nx * d.ny : (size_t)other * d.nx) + x;
  const int p0 = blockIdx.y * kAxisChunk;
  T v[kWin];
#pragma unroll
  for (int i = 0; i < kWin; ++i)
    if (R >= 0 || i < kAxisChunk + 2 * r) v[i] = in[base + (size_t)wrap_any(p0 - r + i, n_axis) * stride];
#pragma unroll
  for (int o = 0; o < kAxisChunk; ++o) {
    if (p0 + o >= n_axis) break;
    T acc = T(0);
#pragma unroll
    for (int j = 0; j <= 2 * radius_bound<R>(); ++j)
      if (R >= 0 || j <= 2 * r) acc += k.w[j] * v[o + j];
    out[base + (size_t)(p0 + o) * stride] = acc;
  }
}

// Blur along x and then y in one pass, for the fixed radii R (> 0): a block
// owns 64 x-values by kXYRows y-values of one plane. The tile and its halo of
// R in x and y are staged in LDS, blurred along x into a second LDS array over
// all rows of the halo, then along y. Both blurs run from register windows: in
// the x pass a thread forms four consecutive outputs of a row from 4 + 2R
// staged values, in the y pass four consecutive outputs of a column. The
// result equals blur_x followed by blur_axis<1> (each output is formed by the
// same sums in the same order). Block (64, 8); grid (ceil(nx/64),
// ceil(ny/kXYRows), nz * batch).
constexpr int kXYRows = 32;

template <typename T, int R>
__global__ __launch_bounds__(512) void blur_xy(const T* __restrict__ in, T* __restrict__ out, FieldDims d,
                                               BlurTaps<T> k) {
  static_assert(R > 0 && 2 * R <= 64 && R % 2 == 0, "blur_xy needs a fixed even radius");
  constexpr int NT = 512;
  constexpr int W = 64 + 2 * R, H = kXYRows + 2 * R;
  constexpr int OUT = 4;                        // outputs per thread and pass
  static_assert(kXYRows == OUT * (NT / 64), "one y window per thread");
  __shared__ T s_in[H][W];
  __shared__ T s_mid[H][64];
  const int tid = threadIdx.y * 64 + threadIdx.x;
  const int z = blockIdx.z % d.nz, b = blockIdx.z / d.nz;
  const int x0 = blockIdx.x * 64, y0 = blockIdx.y * kXYRows;
  const size_t plane = (size_t)d.nx * d.ny, vol = plane * d.nz;
  const T* src = in + (size_t)b * vol + (size_t)z * plane;
  // Stage the tile with its halo: wave w takes the rows w, w + 8, ... (their y
  // is wave-uniform, so it lives in scalar registers), lane l the columns l
  // and, for l < 2R, 64 + l. All loads of a thread are issued before the
  // first LDS write.
  constexpr int RPW = (H + NT / 64 - 1) / (NT / 64);   // rows per wave
  const int wy = __builtin_amdgcn_readfirstlane(threadIdx.y);
  const int lane = threadIdx.x;
  const int xc0 = wrap_any(x0 - R + lane, d.nx), xc1 = wrap_any(x0 - R + 64 + lane, d.nx);
  T v[RPW][2];
#pragma unroll
  for (int i = 0; i < RPW; ++i) {
    const int rr = wy + (NT / 64) * i;
    if (rr >= H) continue;
    const T* row = src + (size_t)wrap_any(y0 - R + rr, d.ny) * d.nx;
    v[i][0] = row[xc0];
    if (lane < 2 * R) v[i][1] = row[xc1];
  }
#pragma unroll
  for (int i = 0; i < RPW; ++i) {
    const int rr = wy + (NT / 64) * i;
    if (rr >= H) continue;
    s_in[rr][lane] = v[i][0];
    if (lane < 2 * R) s_in[rr][64 + lane] = v[i][1];
  }
  __syncthreads();
  // x blur of every staged row: thread -> (row, quad of four x-values)
#pragma unroll
  for (int p = 0; p < (H * 16 + NT - 1) / NT; ++p) {
    const int q = tid % 16, rr = tid / 16 + p * (NT / 16);
    if (rr < H) {
      T w[OUT + 2 * R];
#pragma unroll
      for (int i = 0; i < OUT + 2 * R; ++i) w[i] = s_in[rr][4 * q + i];
#pragma unroll
      for (int o = 0; o < OUT; ++o) {
        T acc = T(0);
#pragma unroll
        for (int j = 0; j <= 2 * R; ++j) acc += k.w[j] * w[o + j];
        s_mid[rr][4 * q + o] = acc;
      }
    }
  }
  __syncthreads();
  // y blur from a register window of this thread's column
  const int x = x0 + threadIdx.x;
  if (x >= d.nx) return;
  T col[OUT + 2 * R];
#pragma unroll
  for (int i = 0; i < OUT + 2 * R; ++i) col[i] = s_mid[threadIdx.y * OUT + i][threadIdx.x];
#pragma unroll
  for (int o = 0; o < OUT; ++o) {
    const int y = y0 + threadIdx.y * OUT + o;
    if (y >= d.ny) break;
    T acc = T(0);
#pragma unroll
    for (int j = 0; j <= 2 * R; ++j) acc += k.w[j] * col[o + j];
    out[(size_t)b * vol + (size_t)z * plane + (size_t)y * d.nx + x] = acc;
  }
}

// Adam on A with dG/dA_a = -(g(i + e_a) - g(i - e_a)) / (2h), g = k * dF/du.
// Moments and A are updated in place; the bias corrections come from the
// clock, which this iteration's first kernel advanced.
// Block (64, 4); grid (ceil(nx/64), ceil(ny/4), nz * batch).
template <typename T>
__global__ __launch_bounds__(256) void adam_vector_field(const T* __restrict__ g, T* __restrict__ A,
                                                         T* __restrict__ m1, T* __restrict__ m2, FieldDims d,
                                                         T inv2h, T lr, T beta1, T beta2, T adam_eps,
                                                         const FlowClock* __restrict__ clk) {
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int y = blockIdx.y * 4 + threadIdx.y;
  const int z = blockIdx.z % d.nz, b = blockIdx.z / d.nz;
  if (x >= d.nx || y >= d.ny) return;
  const size_t plane = (size_t)d.nx * d.ny, vol = plane * d.nz;
  const T* gb = g + (size_t)b * vol;
  const size_t row = (size_t)z * plane + (size_t)y * d.nx;
  // every load of the voxel is issued before the first use, so one memory
  // round trip covers them
  const T gxp = gb[row + wrap_up(x + 1, d.nx)], gxm = gb[row + wrap_down(x - 1, d.nx)];
  const T gyp = gb[(size_t)z * plane + (size_t)wrap_up(y + 1, d.ny) * d.nx + x];
  const T gym = gb[(size_t)z * plane + (size_t)wrap_down(y - 1, d.ny) * d.nx + x];
  const T gzp = gb[(size_t)wrap_up(z + 1, d.nz) * plane + (size_t)y * d.nx + x];
  const T gzm = gb[(size_t)wrap_down(z - 1, d.nz) * plane + (size_t)y * d.nx + x];
  const size_t i0 = (size_t)b * 3 * vol + row + x;
  T av[3], m1v[3], m2v[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    av[a] = A[i0 + a * vol];
    m1v[a] = m1[i0 + a * vol];
    m2v[a] = m2[i0 + a * vol];
  }
  const T bc1 = T(clk->bc1), bc2 = T(clk->bc2);
  const T grad[3] = {-(gxp - gxm) * inv2h, -(gyp - gym) * inv2h, -(gzp - gzm) * inv2h};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const T mo = beta1 * m1v[a] + (T(1) - beta1) * grad[a];
    const T vo = beta2 * m2v[a] + (T(1) - beta2) * grad[a] * grad[a];
    m1[i0 + a * vol] = mo;
    m2[i0 + a * vol] = vo;
    A[i0 + a * vol] = av[a] - lr * (mo * bc1) * rcp_t(sqrt_t(vo * bc2) + adam_eps);
  }
}

// The z blur of w and Adam on A in one pass, for the fixed radii R: g = blur_z(w)
// never goes to memory. A block owns 64 x 4 columns and kAdamZ consecutive
// planes. Phase 1: every column of the tile and its one-column ring (66 x 6)
// is blurred along z over the planes z0 - 1 .. z0 + kAdamZ from a register
// window of kAdamZ + 2 + 2R samples (each thread one or two columns), into LDS.
// Phase 2: each thread updates its column's voxels plane by plane, with the
// neighbours of the central differences from LDS. Sums and update are formed
// in the same order as blur_axis<2> followed by adam_vector_field.
// Block (64, 4); grid (ceil(nx/64), ceil(ny/4), ceil(nz/kAdamZ) * batch).
constexpr int kAdamZ = 16;

template <typename T, int R>
__global__ __launch_bounds__(256) void adam_zblur(const T* __restrict__ w, T* __restrict__ A, T* __restrict__ m1,
                                                  T* __restrict__ m2, FieldDims d, BlurTaps<T> k, T inv2h, T lr,
                                                  T beta1, T beta2, T adam_eps, const FlowClock* __restrict__ clk) {
  static_assert(R > 0 && R <= kBlurMaxR, "adam_zblur needs a fixed radius");
  constexpr int CX = 66, CY = 6, NC = CX * CY;  // tile columns with their ring
  constexpr int NP = kAdamZ + 2;                // blurred planes z0 - 1 .. z0 + kAdamZ
  constexpr int NWIN = NP + 2 * R;              // samples per column
  __shared__ T sg[NP][NC];
  const int tid = threadIdx.y * 64 + threadIdx.x;
  const int nzc = (d.nz + kAdamZ - 1) / kAdamZ;
  const int z0 = (blockIdx.z % nzc) * kAdamZ, b = blockIdx.z / nzc;
  const int x0 = blockIdx.x * 64, y0 = blockIdx.y * 4;
  const size_t plane = (size_t)d.nx * d.ny, vol = plane * d.nz;
  const T* wb = w + (size_t)b * vol;
  // phase 1: the z blur of the columns of the tile and its ring
#pragma unroll
  for (int cc = 0; cc < 2; ++cc) {
    const int c = tid + 256 * cc;
    if (c >= NC) continue;
    const int gx = wrap_any(x0 - 1 + c % CX, d.nx), gy = wrap_any(y0 - 1 + c / CX, d.ny);
    const T* col = wb + (size_t)gy * d.nx + gx;
    T v[NWIN];
#pragma unroll
    for (int i = 0; i < NWIN; ++i) v[i] = col[(size_t)wrap_any(z0 - 1 - R + i, d.nz) * plane];
#pragma unroll
    for (int o = 0; o < NP; ++o) {
      T acc = T(0);
#pragma unroll
      for (int j = 0; j <= 2 * R; ++j) acc += k.w[j] * v[o + j];
      sg[o][c] = acc;
    }
  }
  __syncthreads();
  // phase 2: Adam on the tile's voxels, plane by plane
  const int x = x0 + threadIdx.x, y = y0 + threadIdx.y;
  if (x >= d.nx || y >= d.ny) return;
  const int cc = (threadIdx.y + 1) * CX + threadIdx.x + 1;
  const T bc1 = T(clk->bc1), bc2 = T(clk->bc2);
  for (int o = 0; o < kAdamZ; ++o) {
    const int z = z0 + o;
    if (z >= d.nz) break;
    const size_t i0 = (size_t)b * 3 * vol + (size_t)z * plane + (size_t)y * d.nx + x;
    T av[3], m1v[3], m2v[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      av[a] = A[i0 + a * vol];
      m1v[a] = m1[i0 + a * vol];
      m2v[a] = m2[i0 + a * vol];
    }
    const T gxp = sg[o + 1][cc + 1], gxm = sg[o + 1][cc - 1];
    const T gyp = sg[o + 1][cc + CX], gym = sg[o + 1][cc - CX];
    const T gzp = sg[o + 2][cc], gzm = sg[o][cc];
    const T grad[3] = {-(gxp - gxm) * inv2h, -(gyp - gym) * inv2h, -(gzp - gzm) * inv2h};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const T mo = beta1 * m1v[a] + (T(1) - beta1) * grad[a];
      const T vo = beta2 * m2v[a] + (T(1) - beta2) * grad[a] * grad[a];
      m1[i0 + a * vol] = mo;
      m2[i0 + a * vol] = vo;
      A[i0 + a * vol] = av[a] - lr * (mo * bc1) * rcp_t(sqrt_t(vo * bc2) + adam_eps);
    }
  }
}

// Zero the moments (n elements each) and restart the clock at t = 0.
template <typename T>
__global__ __launch_bounds__(256) void flow_reset(T* m1, T* m2, size_t n, FlowClock* clk) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    m1[i] = T(0);
    m2[i] = T(0);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    clk->t = 0;
    clk->pad = 0;
    clk->bc1 = 1.0;
    clk->bc2 = 1.0;
  }
}

}  // namespace fe
