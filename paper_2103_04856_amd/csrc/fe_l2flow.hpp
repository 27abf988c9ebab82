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
// W > 0: every pad is W wide and the box is at least 2 voxels along every
// axis, so a run on one face is W + 1 samples at fixed offsets and an edge or a
// corner gathers (W+1)^2 or (W+1)^3 of them (unrolled, loads in flight);
// W = 0: general runs, for any box (a box 1 voxel thick has runs on both of
// its sides). One thread per sample of a plane: grid (ceil(nx ny / 256), nz).
// g and out must differ.
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
  if (W > 0) {
    // An edge or a corner: the (W+1)^2 block spanned by the runs along two
    // clamped axes, every load in flight. On an edge the third axis is fixed;
    // on a corner the block is in (y, x) and z runs over its W + 1 planes.
    // Blocks are summed in increasing index order, as the general loop adds.
    const long sx = 1, sy = b.nx, sz = (long)b.nx * b.ny;
    long sp = sy, sq = sx, so = sz;
    int no = fz ? W + 1 : 1;
    if (nf == 2 && fz) {
      no = 1;
      if (!fy) {
        sp = sz;
        sq = sx;
        so = sy;
      } else {
        sp = sz;
        sq = sy;
        so = sx;
      }
    }
    const T* p0 = g + ((size_t)z0 * b.ny + y0) * b.nx + x0;
    T acc = T(0);
    for (int ko = 0; ko < no; ++ko) {
      T v[(W + 1) * (W + 1)];
#pragma unroll
      for (int kp = 0; kp <= W; ++kp)
#pragma unroll
        for (int kq = 0; kq <= W; ++kq) v[kp * (W + 1) + kq] = p0[ko * so + kp * sp + kq * sq];
#pragma unroll
      for (int k = 0; k < (W + 1) * (W + 1); ++k) acc += v[k];
    }
    out[i] = acc;
    return;
  }
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

// ---- the L-BFGS direction through Gram matrices ----
//
// The two-loop recursion only ever combines the history vectors s_i, y_i and
// the gradient g linearly, and its scalars are inner products of those
// vectors. So the host runs the recursion on the inner products (FP64, kept
// up to date as pairs enter and leave the history) and the device makes two
// passes per iteration: vec_gram forms the new pair and every inner product
// the recursion needs, vec_lincomb forms the direction from the coefficients.

// Threads per vec_gram block: a full block for FP32; a quarter for FP64, whose
// accumulators and packs need twice the registers.
template <typename T>
constexpr int gram_threads() { return sizeof(T) == 4 ? kVecThreads : kVecThreads / 4; }
constexpr int kDotVecs = 24;    // history vectors per vec_gram pass (all of them up to history 12)
constexpr int kCombVecs = 24;   // vectors per vec_lincomb pass (all 2m + 1 of them up to history 11)

template <typename T>
struct DotList {
  const T* v[kDotVecs];
  int count;
};

template <typename T>
struct CombList {
  const T* v[kCombVecs];
  double c[kCombVecs];
  int count;
};

// The partials of NV values per block, each in a fixed order (the wave's
// butterfly, then the waves in order), into bank k * kVecBlocks + blockIdx.x.
template <int NV, int NT>
__device__ __forceinline__ void vec_block_partials(double (&acc)[NV], int nv, double* __restrict__ banks) {
  __shared__ double s_w[NV][NT / 64];
  // every value takes the butterfly (fixed trip counts keep acc in registers)
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double a = acc[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
    if (threadIdx.x % 64 == 0) s_w[k][threadIdx.x / 64] = a;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < nv; k += NT) {
    double a = s_w[k][0];
    for (int wv = 1; wv < NT / 64; ++wv) a += s_w[k][wv];
    banks[(size_t)k * kVecBlocks + blockIdx.x] = a;
  }
}

// One pass of the Gram update. FORM: first y = g - prev_g and s = t d, stored,
// and the banks 0..4 get y.y, y.s, y.g, g.g, g.s (NB = 5; otherwise NB = 0).
// The first NL list vectors V_k then give g.V_k in bank NB + k. The products
// of y with the history need no pass of their own: y.V = g.V - prev_g.V, and
// the host kept prev_g.V from the previous pass. All NL list entries are read
// (the host points unused ones at g, and only the first `count` reach the
// banks), so the loops have fixed trip counts and every value stays in
// registers. FP64 accumulation, packs of four, block 0 takes the n % 4 tail.
// Grid: kVecBlocks blocks of gram_threads<T>().
template <typename T, bool FORM, int NL>
__global__ __launch_bounds__(gram_threads<T>()) void vec_gram(const T* __restrict__ g, const T* __restrict__ prev_g,
                                                              const T* __restrict__ d, double t, T* __restrict__ y,
                                                              T* __restrict__ s, DotList<T> L, size_t n,
                                                              double* __restrict__ banks) {
  static_assert(NL >= 0 && NL <= kDotVecs && (FORM || NL > 0), "vec_gram list width");
  constexpr int NB = FORM ? 5 : 0;
  constexpr int NV = NB + NL;
  const T tt = T(t);
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  const size_t n4 = n / 4, stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
    const Pack4<T> pg = reinterpret_cast<const Pack4<T>*>(g)[i];
    if constexpr (FORM) {
      const Pack4<T> pp = reinterpret_cast<const Pack4<T>*>(prev_g)[i];
      const Pack4<T> pd = reinterpret_cast<const Pack4<T>*>(d)[i];
      Pack4<T> py, ps;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        py.v[e] = pg.v[e] - pp.v[e];
        ps.v[e] = tt * pd.v[e];
      }
      reinterpret_cast<Pack4<T>*>(y)[i] = py;
      reinterpret_cast<Pack4<T>*>(s)[i] = ps;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const double ye = py.v[e], ge = pg.v[e], se = ps.v[e];
        acc[0] += ye * ye;
        acc[1] += ye * se;
        acc[2] += ye * ge;
        acc[3] += ge * ge;
        acc[4] += ge * se;
      }
    }
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      const Pack4<T> pv = reinterpret_cast<const Pack4<T>*>(L.v[k])[i];
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[NB + k] += double(pg.v[e]) * double(pv.v[e]);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x < n - 4 * n4) {
    const size_t j = 4 * n4 + threadIdx.x;
    const double ge = g[j];
    if constexpr (FORM) {
      const T yt = g[j] - prev_g[j], st = tt * d[j];
      y[j] = yt;
      s[j] = st;
      const double ye = yt, se = st;
      acc[0] += ye * ye;
      acc[1] += ye * se;
      acc[2] += ye * ge;
      acc[3] += ge * ge;
      acc[4] += ge * se;
    }
#pragma unroll
    for (int k = 0; k < NL; ++k) acc[NB + k] += ge * double(L.v[k][j]);
  }
  vec_block_partials<NV, gram_threads<T>()>(acc, NB + L.count, banks);
}

// out = sum_k c_k V_k (+ out when acc), accumulated in FP64 and rounded once;
// when dmax is given, its bank gets the partials of max |out|; when x is
// given, x += t out (FP64, rounded once) with the rounded out, which is the
// optimiser's step folded into the pass that forms its direction. All W list
// entries are read (the host pads a short list with zero coefficients on a
// listed vector), so the loop has a fixed trip count. Layout of the work as in
// vec_reduce.
template <typename T, int W>
__global__ __launch_bounds__(kVecThreads) void vec_lincomb(CombList<T> L, T* __restrict__ out, int acc, size_t n,
                                                           double* __restrict__ dmax, T* __restrict__ x, double t) {
  static_assert(W >= 1 && W <= kCombVecs, "vec_lincomb width");
  const size_t n4 = n / 4, stride = (size_t)gridDim.x * blockDim.x;
  double mx = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    if (acc) {
      const Pack4<T> po = reinterpret_cast<const Pack4<T>*>(out)[i];
#pragma unroll
      for (int e = 0; e < 4; ++e) a[e] = double(po.v[e]);
    }
#pragma unroll
    for (int k = 0; k < W; ++k) {
      const Pack4<T> pv = reinterpret_cast<const Pack4<T>*>(L.v[k])[i];
#pragma unroll
      for (int e = 0; e < 4; ++e) a[e] += L.c[k] * double(pv.v[e]);
    }
    Pack4<T> r;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      r.v[e] = T(a[e]);
      mx = fmax(mx, fabs(double(r.v[e])));
    }
    reinterpret_cast<Pack4<T>*>(out)[i] = r;
    if (x) {
      Pack4<T> px = reinterpret_cast<const Pack4<T>*>(x)[i];
#pragma unroll
      for (int e = 0; e < 4; ++e) px.v[e] = T(double(px.v[e]) + t * double(r.v[e]));
      reinterpret_cast<Pack4<T>*>(x)[i] = px;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x < n - 4 * n4) {
    const size_t j = 4 * n4 + threadIdx.x;
    double a = acc ? double(out[j]) : 0.0;
#pragma unroll
    for (int k = 0; k < W; ++k) a += L.c[k] * double(L.v[k][j]);
    const T r = T(a);
    out[j] = r;
    mx = fmax(mx, fabs(double(r)));
    if (x) x[j] = T(double(x[j]) + t * double(r));
  }
  if (dmax) vec_block_partial<2>(mx, dmax);
}

// Values of `count` consecutive sum banks: out[k] = bank_value<0>(bank k).
// Grid: count blocks of 64.
__global__ __launch_bounds__(64) void vec_finish_sums(const double* __restrict__ banks, double* __restrict__ out) {
  const double v = bank_value<0>(banks + (size_t)blockIdx.x * kVecBlocks);
  if (threadIdx.x == 0) out[blockIdx.x] = v;
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
