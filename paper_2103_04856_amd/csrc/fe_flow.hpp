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
// adam_vector_field; for the radii 4 and 8 the x and y blurs of dF/du are one
// pass (blur_xy). Without blur (r = 0) only the first kernel, the sweep and
// the Adam kernel run. Every wave reads and writes consecutive voxels of a row
// (blur_x, blur_xy: 64-wide row tiles with their halos in LDS) or of a plane
// (blur_axis, adam_vector_field: flat runs of 256 voxels), so every access is
// coalesced; tiles are placed on the XCDs by xcd_tile (blur_xy excepted).
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

// base[i] for a wave-uniform base and an element offset below 2^32 bytes (the
// flow entry points reject planes of 4 GiB or more): the load then takes the
// scalar base and a 32-bit vector offset, and a lane spends no 64-bit address
// arithmetic on it.
template <typename T>
__device__ __forceinline__ T load_u32(const T* base, unsigned i) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + i * (unsigned)sizeof(T));
}

template <typename T>
__device__ __forceinline__ void store_u32(T* base, unsigned i, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + i * (unsigned)sizeof(T)) = v;
}

// Workgroups go to the chip's 8 XCDs in turn (workgroup i of the x-fastest
// order to XCD i mod 8), and each XCD has an L2 of its own, so tiles with
// consecutive numbers never share an L2. The flow kernels' tiles read each
// other's halos (the ring and window rows and planes, and the cache lines that
// straddle two tiles of a row), so they take their tile from xcd_tile: the
// workgroups are renumbered so that every XCD runs one contiguous range of
// tiles in x-fastest order, and neighbouring tiles meet in one L2 at about the
// same time. The last (count mod 8) workgroups keep their numbers. A grid of
// at most about four workgroups per CU (kXcdRenumberFrom) keeps the hardware's
// order: all of it is resident at once, so tiles that share halos run together
// anyway, and gathering them on one XCD only queues their identical requests
// there (100^3, the y and z blur passes with 280 workgroups: 5.6 and 8.3 us in
// the hardware's order, 8.9 and 10.5 us renumbered). Only the placement
// changes: every tile computes the same sums.
struct Tile3 {
  int x, y, z;
};

constexpr unsigned kXcdRenumberFrom = 1024;

__device__ __forceinline__ Tile3 xcd_tile() {
  constexpr unsigned kXcds = 8;
  const unsigned gx = gridDim.x, gy = gridDim.y;
  const unsigned n = gx * gy * gridDim.z, per = n / kXcds;
  unsigned b = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  if (n >= kXcdRenumberFrom && b < per * kXcds) b = (b % kXcds) * per + b / kXcds;
  Tile3 t;
  t.x = (int)(b % gx);
  b /= gx;
  t.y = (int)(b % gy);
  t.z = (int)(b / gy);
  return t;
}

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
// ROWS: rows with nx + 2r <= 128 are staged whole (x0 = 0, one x tile, grid
// (1, ceil(ny/kBlurRows), nz * batch)): a row of 100 then stages 116 samples
// instead of two 64-wide tiles' 2 x (64 + 2r), and 100 of 128 lanes form outputs.
constexpr int kBlurRows = 16;
constexpr int kRowsMax = 128;   // ROWS: the longest staged row, nx + 2r

template <typename T, bool DIV, int R = -1, bool ROWS = false>
__global__ __launch_bounds__(256) void blur_x(const T* __restrict__ in, T* __restrict__ out,
                                              const double* __restrict__ m0, const T* __restrict__ mfield,
                                              FieldDims d, T inv2h, BlurTaps<T> k, FlowClock* __restrict__ clk,
                                              double beta1, double beta2) {
  constexpr int kW = ROWS ? kRowsMax : 64 + 2 * kBlurMaxR;
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
  const Tile3 t = xcd_tile();
  const int z = t.z % d.nz, b = t.z / d.nz;
  const int x0 = ROWS ? 0 : t.x * 64;
  const size_t plane = (size_t)d.nx * d.ny, vol = plane * d.nz;
  const T* base = in + (size_t)b * (DIV ? 3 : 1) * vol;
  const int r = R >= 0 ? R : k.r;
  const int nseg = (ROWS ? d.nx : 64) + 2 * r;
  // A wave's rows are uniform (threadIdx.y is the wave), so the row pointers
  // live in scalar registers and every load takes a 32-bit lane offset: the
  // segment's x positions and their periodic x neighbours, formed once.
  const int wy = __builtin_amdgcn_readfirstlane(threadIdx.y);
  int xs[kPer], xp[kPer], xm[kPer];
#pragma unroll
  for (int j = 0; j < kPer; ++j) {
    const int x = wrap_any(x0 - r + (int)threadIdx.x + 64 * j, d.nx);
    xs[j] = x;
    xp[j] = wrap_up(x + 1, d.nx);
    xm[j] = wrap_down(x - 1, d.nx);
  }
  T v[kR][kPer][7];          // the non-DIV form uses [0] only; [6] holds m(x)
#pragma unroll
  for (int i = 0; i < kR; ++i) {
    const int y = t.y * kBlurRows + wy + 4 * i;
    if (y >= d.ny) continue;
    const T* row = base + (size_t)z * plane + (size_t)y * d.nx;
    // the A_y rows y +- 1 and the A_z rows of the planes z +- 1 (DIV only)
    const T* rowyp = DIV ? base + vol + (size_t)z * plane + (size_t)wrap_up(y + 1, d.ny) * d.nx : row;
    const T* rowym = DIV ? base + vol + (size_t)z * plane + (size_t)wrap_down(y - 1, d.ny) * d.nx : row;
    const T* rowzp = DIV ? base + 2 * vol + (size_t)wrap_up(z + 1, d.nz) * plane + (size_t)y * d.nx : row;
    const T* rowzm = DIV ? base + 2 * vol + (size_t)wrap_down(z - 1, d.nz) * plane + (size_t)y * d.nx : row;
    const T* rowm = (DIV && mfield) ? mfield + (size_t)b * vol + (size_t)z * plane + (size_t)y * d.nx : row;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int e = threadIdx.x + 64 * j;
      if (e >= nseg) continue;
      if (DIV) {
        v[i][j][0] = load_u32(row, xp[j]);
        v[i][j][1] = load_u32(row, xm[j]);
        v[i][j][2] = load_u32(rowyp, xs[j]);
        v[i][j][3] = load_u32(rowym, xs[j]);
        v[i][j][4] = load_u32(rowzp, xs[j]);
        v[i][j][5] = load_u32(rowzm, xs[j]);
        if (mfield) v[i][j][6] = load_u32(rowm, xs[j]);
      } else {
        v[i][j][0] = load_u32(row, xs[j]);
      }
    }
  }
  const T mass = (DIV && !mfield) ? T(m0[b]) : T(0);
#pragma unroll
  for (int i = 0; i < kR; ++i) {
    const int y = t.y * kBlurRows + wy + 4 * i;
    if (y >= d.ny) continue;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      const int e = threadIdx.x + 64 * j;
      if (e >= nseg) continue;
      if (DIV)
        s[wy + 4 * i][e] =
            (mfield ? v[i][j][6] : mass) +
            ((v[i][j][0] - v[i][j][1]) + (v[i][j][2] - v[i][j][3]) + (v[i][j][4] - v[i][j][5])) * inv2h;
      else
        s[wy + 4 * i][e] = v[i][j][0];
    }
  }
  __syncthreads();
#pragma unroll
  for (int jo = 0; jo < (ROWS ? kPer : 1); ++jo) {
    const int xo = threadIdx.x + 64 * jo;       // output position in the tile
    const int x = x0 + xo;
    if (x >= d.nx) break;
#pragma unroll
    for (int i = 0; i < kR; ++i) {
      const int y = t.y * kBlurRows + wy + 4 * i;
      if (y >= d.ny) continue;
      T* orow = out + (size_t)b * vol + (size_t)z * plane + (size_t)y * d.nx;
      orow[x] = taps_dot<T, R>(k, &s[wy + 4 * i][xo], 1);
    }
  }
}

// Blur along y (AXIS = 1) or z (AXIS = 2) with a register window: each thread
// owns kAxisChunk consecutive outputs of one column, loads that segment and
// its periodic halo of r once and forms every output from registers, so the
// pass needs no LDS. The columns are numbered flat over the two other axes
// (for z, the voxels of a plane in memory order; for y, the x values of every
// plane in turn), so a block is 256 consecutive columns and no lane idles on a
// row that is not a multiple of 64 wide. Block 256; grid (ceil(columns / 256),
// ceil(n_axis / kAxisChunk), batch).
constexpr int kAxisChunk = 16;

template <typename T, int AXIS, int R = -1>
__global__ __launch_bounds__(256) void blur_axis(const T* __restrict__ in, T* __restrict__ out, FieldDims d,
                                                 BlurTaps<T> k) {
  constexpr int kWin = kAxisChunk + 2 * radius_bound<R>();
  const int r = R >= 0 ? R : k.r;
  const Tile3 t = xcd_tile();
  const int n_axis = AXIS == 1 ? d.ny : d.nz;
  const size_t plane = (size_t)d.nx * d.ny, vol = plane * d.nz;
  const unsigned nflat = AXIS == 2 ? (unsigned)plane : (unsigned)d.nz * (unsigned)d.nx;
  const unsigned q = (unsigned)t.x * 256u + threadIdx.x;
  if (q >= nflat) return;
  const int p0 = t.y * kAxisChunk;
  const T* inb = in + (size_t)t.z * vol;
  T* outb = out + (size_t)t.z * vol;
  T v[kWin];
  if (AXIS == 2) {
#pragma unroll
    for (int i = 0; i < kWin; ++i)
      if (R >= 0 || i < kAxisChunk + 2 * r) v[i] = load_u32(inb + (size_t)wrap_any(p0 - r + i, n_axis) * plane, q);
#pragma unroll
    for (int o = 0; o < kAxisChunk; ++o) {
      if (p0 + o >= n_axis) break;
      T acc = T(0);
#pragma unroll
      for (int j = 0; j <= 2 * radius_bound<R>(); ++j)
        if (R >= 0 || j <= 2 * r) acc += k.w[j] * v[o + j];
      store_u32(outb + (size_t)(p0 + o) * plane, q, acc);
    }
  } else {
    const unsigned zq = q / (unsigned)d.nx, x = q - zq * (unsigned)d.nx;
    const size_t lane = (size_t)zq * plane + x;
#pragma unroll
    for (int i = 0; i < kWin; ++i)
      if (R >= 0 || i < kAxisChunk + 2 * r) v[i] = inb[lane + (size_t)wrap_any(p0 - r + i, n_axis) * d.nx];
#pragma unroll
    for (int o = 0; o < kAxisChunk; ++o) {
      if (p0 + o >= n_axis) break;
      T acc = T(0);
#pragma unroll
      for (int j = 0; j <= 2 * radius_bound<R>(); ++j)
        if (R >= 0 || j <= 2 * r) acc += k.w[j] * v[o + j];
      outb[lane + (size_t)(p0 + o) * d.nx] = acc;
    }
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
// ROWS: rows with nx + 2R <= 128 are staged whole with their periodic halo
// (grid (1, ceil(ny/kXYRows), nz * batch)); the x pass then deals out quads
// 32 to a row, the y pass two columns per thread (x and x + 64). A row of 100
// stages 116 samples instead of 2 x (64 + 2R) and takes 25 quads per row
// where two 64-wide tiles take 32.
constexpr int kXYRows = 32;

template <typename T, int R, bool ROWS = false>
__global__ __launch_bounds__(512) void blur_xy(const T* __restrict__ in, T* __restrict__ out, FieldDims d,
                                               BlurTaps<T> k) {
  static_assert(R > 0 && 2 * R <= 64 && R % 2 == 0, "blur_xy needs a fixed even radius");
  constexpr int NT = 512;
  constexpr int OUT = 4;                        // outputs per thread and pass
  // staged row width; ROWS: up to 128 staged, plus the 3 a ragged last quad reads past them
  constexpr int W = ROWS ? kRowsMax + OUT : 64 + 2 * R, H = kXYRows + 2 * R;
  constexpr int WM = ROWS ? kRowsMax : 64;      // x-blurred row width
  static_assert(kXYRows == OUT * (NT / 64), "one y window per thread");
  __shared__ T s_in[H][W];
  __shared__ T s_mid[H][WM];
  const int tid = threadIdx.y * 64 + threadIdx.x;
  // Tiles in the hardware's order: this pass is bound by its LDS and VALU
  // work, not by its halo fetches (those hit MALL), and xcd_tile's placement
  // measured slower for it (16 x 100^3: 656 against 648 us per iteration).
  const int z = blockIdx.z % d.nz, b = blockIdx.z / d.nz;
  const int x0 = ROWS ? 0 : blockIdx.x * 64, y0 = blockIdx.y * kXYRows;
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
  const bool second = ROWS ? 64 + lane < d.nx + 2 * R : lane < 2 * R;
  T v[RPW][2];
#pragma unroll
  for (int i = 0; i < RPW; ++i) {
    const int rr = wy + (NT / 64) * i;
    if (rr >= H) continue;
    const T* row = src + (size_t)wrap_any(y0 - R + rr, d.ny) * d.nx;
    v[i][0] = row[xc0];
    if (second) v[i][1] = row[xc1];
  }
#pragma unroll
  for (int i = 0; i < RPW; ++i) {
    const int rr = wy + (NT / 64) * i;
    if (rr >= H) continue;
    s_in[rr][lane] = v[i][0];
    if (second) s_in[rr][64 + lane] = v[i][1];
  }
  __syncthreads();
  // x blur of every staged row: thread -> (row, quad of four x-values); QPR
  // quads per row (ROWS: the row's ceil(nx/4) of 32 slots)
  constexpr int QPR = ROWS ? 32 : 16;
  const int nquad = ROWS ? (d.nx + OUT - 1) / OUT : 16;
#pragma unroll
  for (int p = 0; p < (H * QPR + NT - 1) / NT; ++p) {
    const int q = tid % QPR, rr = tid / QPR + p * (NT / QPR);
    if (rr < H && q < nquad) {
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
  // y blur from a register window of this thread's column (ROWS: x and x + 64)
#pragma unroll
  for (int jx = 0; jx < (ROWS ? 2 : 1); ++jx) {
    const int xo = threadIdx.x + 64 * jx;
    const int x = x0 + xo;
    if (x >= d.nx) break;
    T col[OUT + 2 * R];
#pragma unroll
    for (int i = 0; i < OUT + 2 * R; ++i) col[i] = s_mid[threadIdx.y * OUT + i][xo];
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
}

// Adam on A with dG/dA_a = -(g(i + e_a) - g(i - e_a)) / (2h), g = k * dF/du.
// Moments and A are updated in place; the bias corrections come from the
// clock, which this iteration's first kernel advanced. A block is 256
// consecutive voxels of one plane in memory order (the x and y neighbours of a
// voxel from its row and plane, periodic), so every lane has a voxel whatever
// the row width. Block 256; grid (ceil(nx ny / 256), 1, nz * batch).
template <typename T>
__global__ __launch_bounds__(256) void adam_vector_field(const T* __restrict__ g, T* __restrict__ A,
                                                         T* __restrict__ m1, T* __restrict__ m2, FieldDims d,
                                                         T inv2h, T lr, T beta1, T beta2, T adam_eps,
                                                         const FlowClock* __restrict__ clk) {
  const Tile3 t = xcd_tile();
  const unsigned np = (unsigned)d.nx * (unsigned)d.ny;
  const unsigned q = (unsigned)t.x * 256u + threadIdx.x;
  if (q >= np) return;
  const int z = t.z % d.nz, b = t.z / d.nz;
  const int y = (int)(q / (unsigned)d.nx), x = (int)q - y * d.nx;
  const size_t plane = np, vol = plane * d.nz;
  const T* gp = g + (size_t)b * vol + (size_t)z * plane;     // uniform
  const unsigned rowq = q - (unsigned)x;
  const T gxp = load_u32(gp, rowq + (unsigned)wrap_up(x + 1, d.nx));
  const T gxm = load_u32(gp, rowq + (unsigned)wrap_down(x - 1, d.nx));
  const T gyp = load_u32(gp, (unsigned)(wrap_up(y + 1, d.ny) * d.nx + x));
  const T gym = load_u32(gp, (unsigned)(wrap_down(y - 1, d.ny) * d.nx + x));
  const T gzp = load_u32(g + (size_t)b * vol + (size_t)wrap_up(z + 1, d.nz) * plane, q);
  const T gzm = load_u32(g + (size_t)b * vol + (size_t)wrap_down(z - 1, d.nz) * plane, q);
  const size_t p0 = (size_t)b * 3 * vol + (size_t)z * plane;
  T av[3], m1v[3], m2v[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    av[a] = load_u32(A + p0 + a * vol, q);
    m1v[a] = load_u32(m1 + p0 + a * vol, q);
    m2v[a] = load_u32(m2 + p0 + a * vol, q);
  }
  const T bc1 = T(clk->bc1), bc2 = T(clk->bc2);
  const T grad[3] = {-(gxp - gxm) * inv2h, -(gyp - gym) * inv2h, -(gzp - gzm) * inv2h};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const T mo = beta1 * m1v[a] + (T(1) - beta1) * grad[a];
    const T vo = beta2 * m2v[a] + (T(1) - beta2) * grad[a] * grad[a];
    store_u32(m1 + p0 + a * vol, q, mo);
    store_u32(m2 + p0 + a * vol, q, vo);
    store_u32(A + p0 + a * vol, q, av[a] - lr * (mo * bc1) * rcp_t(sqrt_t(vo * bc2) + adam_eps));
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
