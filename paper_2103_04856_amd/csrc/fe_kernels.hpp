// HIP kernels for gfx950: the fused energy + gradient sweep, the energy-only
// sweep, the deterministic per-instance finalisation and the step helpers.
//
// Data layout: fields are [batch][nz][ny][nx], x fastest. A block owns an
// interior tile of TX x TY columns and a chunk of lz consecutive z planes of
// one instance, and streams through the planes (2.5-D blocking):
//
//   * u is staged in LDS as a rolling window of three planes, each with a
//     periodic halo of 2 in x and y (the gather needs the adjoint on a ring
//     of one voxel, and the adjoint at a voxel needs the 19-point stencil);
//   * for every plane the block computes forward + adjoint on the interior
//     plus a one-voxel ring (the Hessian is recomputed, never stored) and
//     parks the ten scaled adjoint values in LDS;
//   * the transposed stencils are applied as adds: in-plane terms from LDS,
//     terms from the planes above and below through a three-plane register
//     pipeline, so each output voxel is written exactly once;
//   * sums (energy, mass of the stepped field) are accumulated per thread in
//     FP64, reduced with wavefront shuffles and one LDS pass, and written as
//     one partial per block. Whoever needs an instance's totals adds its
//     partials in one fixed order (deterministic): the next step's blocks,
//     for the shift that projects the stepped field back onto its target
//     mean, or sweep_finish for the energy. No block waits for another, and
//     a step is one launch with no device-wide fence.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "fe_voxel.hpp"

namespace fe {

constexpr int kWave = 64;

// A lane's byte offset into a plane, made opaque to the optimiser where a loop
// over planes uses it: the access then stays a block-uniform plane address
// (scalar registers, advanced by the scalar unit) plus this 32-bit offset,
// instead of a 64-bit per-lane pointer advanced with vector arithmetic every
// plane. The empty statement emits no instruction.
__device__ __forceinline__ unsigned lane_offset(unsigned o) {
  __asm__("" : "+v"(o));
  return o;
}

// A raw buffer over `bytes` bytes from `base` (stride 0; the third-dword format
// of a 32-bit raw buffer on gfx9-family chips). The hardware drops a store whose
// offset is at or past `bytes`, so a store that must not land can still be
// issued, at kDropOffset: the memory operations issued are then the same on
// every path. Planes are at most 4 GiB - 64 KiB (checked on the host), so
// kDropOffset is never in range.
constexpr unsigned kDropOffset = 0xFFFFFFF0u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ void buffer_store(float v, __amdgpu_buffer_rsrc_t r, unsigned off) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)off, 0, 0);
}

__device__ __forceinline__ void buffer_store(double v, __amdgpu_buffer_rsrc_t r, unsigned off) {
  typedef unsigned u32x2 __attribute__((__vector_size__(2 * sizeof(unsigned))));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)off, 0, 0);
}

// Loads and stores through such a buffer take the 32-bit lane offset as an
// operand of the instruction, so the compiler neither widens it to a 64-bit
// lane address nor needs it kept opaque, and the plane address stays in
// scalar registers.
__device__ __forceinline__ float buffer_load(__amdgpu_buffer_rsrc_t r, unsigned off, float) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}

__device__ __forceinline__ double buffer_load(__amdgpu_buffer_rsrc_t r, unsigned off, double) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}

// Issue priority of a sweep's waves at plane `it` of the n planes of its z
// chunk. The blocks of a sweep share compute units (two or three each) and
// start together, and a compute unit issues the older block's waves first: left
// alone, the first block finished long before the others, which then ran with
// the unit half idle (256^3 step: 142 k against 186 k shader cycles per block).
// The priority falls as a block advances (3 from the start, 2 from half way, 1
// from three quarters, 0 for the last tenth), so a block that lags takes the
// issue slots until it has caught up. The first level is set before the loop
// (start_priority), so that the loop keeps a single body: a branch on the first
// iteration made the compiler peel it, and the copies contracted some products
// into FMAs differently, which broke the bitwise agreement between launch shapes.
__device__ __forceinline__ void start_priority() { __builtin_amdgcn_s_setprio(3); }

__device__ __forceinline__ void progress_priority(int it, int n) {
  if (it == n / 2) __builtin_amdgcn_s_setprio(2);
  if (it == (3 * n) / 4) __builtin_amdgcn_s_setprio(1);
  if (it == (9 * n) / 10) __builtin_amdgcn_s_setprio(0);
}

__device__ __forceinline__ int wrap_index(int v, int n) {
  int r = v % n;
  return r < 0 ? r + n : r;
}

// Block-wide sum of two doubles; result valid in thread 0. Fixed reduction
// order, so repeated runs give identical bits.
template <int NT>
__device__ __forceinline__ void block_sum2(double& a, double& b, double (*sred)[2]) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    a += __shfl_xor(a, off, kWave);
    b += __shfl_xor(b, off, kWave);
  }
  const int lane = threadIdx.x % kWave;
  const int wv = threadIdx.x / kWave;
  if (lane == 0) {
    sred[wv][0] = a;
    sred[wv][1] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0.0, sb = 0.0;
#pragma unroll
    for (int i = 0; i < NT / kWave; ++i) {
      sa += sred[i][0];
      sb += sred[i][1];
    }
    a = sa;
    b = sb;
  }
}

// Linear block id -> logical tile, so that the blocks dispatched to one XCD
// (hardware round-robins consecutive ids over the 8 XCDs) form a contiguous
// range of neighbouring tiles that share halo lines in that XCD's L2.
__device__ __forceinline__ int xcd_logical_block(int linear, int total) {
  constexpr int kXcd = 8;
  if (total % kXcd != 0) return linear;
  return (linear % kXcd) * (total / kXcd) + linear / kXcd;
}

// Which per-voxel bodies a sweep kernel holds (see grad_sweep).
enum SweepBody { kBodyAny = 0, kBodyNoS = 1, kBodyFull = 2 };

// What the fused sweep writes.
enum SweepMode {
  kGrad = 0,      // dst = dF_h/du (h^3 included); partial[1] = sum of src
  kStepGD = 1,    // dst = u - tau dF_h/du, u = src + shift of src; partial[1] = sum of dst
  kStepAdam = 2,  // dst = u - lr mhat / (sqrt(vhat) + adam_eps), moments updated in place
};

template <typename T>
struct SweepArgs {
  const T* src;                 // [batch][nz][ny][nx]
  T* dst;                       // gradient or stepped field; unused by the energy sweep
  const InstParams<T>* prm;     // [batch]
  const double* prev_partials;  // steps: the partials of the step that wrote src; the instance's shift
                                // mass - mean(src) formed from them is added to src (null: no shift)
  double* partials;             // out: [batch][blocks_per_instance][2] per-block sums of the energy
                                // density and of the field (steps: the stepped field, else src)
  const double* mass;           // steps: [batch] target means
  double inv_nvox;
  T* m1;                        // Adam: first moment, same layout as src
  T* m2;                        // Adam: second moment
  const int* adam_t;            // Adam: base step number t0 (device, advanced by adam_tick)
  int t_add;                    // Adam: this step's number is t0 + t_add
  const T* cfield;              // space-dependent coefficients: [batch][nz][ny][nx] records of the six
                                // scaled C1..C6 (VoxelCoeffs), read by the SP instantiations only
  int box_lo[3], box_hi[3];     // BOX instantiations: the voxels (x, y, z) whose density is summed;
                                // the others only supply samples (a padded field)
  GridConsts<T> k;
  T tau;                        // GD step size, or Adam learning rate
  T beta1, beta2, adam_eps;     // Adam
  int nx, ny, nz;
  int ntx, nty, nzc, lz;        // tiles in x and y, z chunks, planes per chunk
  int batch;
};

// The six scaled coefficients of one voxel from the coefficient field (Sec. 5.2:
// a(x) acts at the voxel where the density is evaluated). The context keeps the
// field as one record per voxel, so a voxel's six values are one contiguous
// 24-byte (FP64: 48-byte) record, read with two or three wide loads instead of
// six loads from six planes a field apart.
template <typename T>
struct alignas(2 * sizeof(T)) VoxelCoeffs {
  T c[6];
};

template <typename T>
__device__ __forceinline__ const VoxelCoeffs<T>* coeff_records(const T* cfield) {
  return reinterpret_cast<const VoxelCoeffs<T>*>(cfield);
}

template <typename T>
__device__ __forceinline__ InstParams<T> with_coeffs(InstParams<T> p, const VoxelCoeffs<T>& v) {
  p.C1 = v.c[0];
  p.C2 = v.c[1];
  p.C3 = v.c[2];
  p.C4 = v.c[3];
  p.C5 = v.c[4];
  p.C6 = v.c[5];
  return p;
}

// End of a sweep block: the block's two sums go to its partial. They are
// combined per instance by instance_sums, in one fixed order, wherever they
// are needed (the next step's shift, sweep_finish), so no block waits for
// another and a launch needs no device-wide fence.
template <int NT, typename T>
__device__ __forceinline__ void write_partials(const SweepArgs<T>& a, int logical, double acc_f, double acc_m,
                                               double (*sred)[2]) {
  block_sum2<NT>(acc_f, acc_m, sred);
  if (threadIdx.x == 0) {
    double* out = a.partials + (size_t)logical * 2;
    out[0] = acc_f;
    out[1] = acc_m;
  }
}

// Per-instance sums of the block partials of a sweep: lane l of the calling
// wave adds the partials of blocks l, l + 64, l + 128, ... in that order, then
// a butterfly over the wave combines the lanes. Each butterfly step adds a lane
// and its partner, and the two orders of an addition agree bit for bit, so
// every lane of every wave that calls this gets the same bits. Call from all
// 64 lanes of a wave.
__device__ __forceinline__ void instance_sums(const double* __restrict__ partials, int inst, int per_inst,
                                              double& sf, double& sm) {
  const int lane = threadIdx.x % kWave;
  const double* pp = partials + (size_t)inst * per_inst * 2;
  double f = 0.0, m = 0.0;
  for (int k = lane; k < per_inst; k += kWave) {
    f += pp[2 * k];
    m += pp[2 * k + 1];
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    f += __shfl_xor(f, off, kWave);
    m += __shfl_xor(m, off, kWave);
  }
  sf = f;
  sm = m;
}

// The 19 stencil samples of a voxel from the LDS planes p (bc), p-1 (bm) and
// p+1 (bp) of a window UX values wide. Each pointer is the byte address of
// the sample at (x-1, y-1) in its plane, so every sample sits at a
// non-negative constant offset of at most 2 UX + 2 values from it, which the
// LDS read instructions (paired reads included) take as their immediate:
// three address additions per voxel, one per plane.
template <typename T, int UX>
__device__ __forceinline__ Stencil19<T> load_stencil(const char* bc, const char* bm, const char* bp) {
  auto at = [](const char* b, int i) { return *reinterpret_cast<const T*>(b + i * (int)sizeof(T)); };
  constexpr int C = UX + 1;                    // the centre
  Stencil19<T> s;
  s.c = at(bc, C);
  s.xm = at(bc, C - 1); s.xp = at(bc, C + 1); s.ym = at(bc, C - UX); s.yp = at(bc, C + UX);
  s.zm = at(bm, C); s.zp = at(bp, C);
  s.xpyp = at(bc, C + UX + 1); s.xpym = at(bc, C + 1 - UX); s.xmyp = at(bc, C + UX - 1); s.xmym = at(bc, 0);
  s.xpzp = at(bp, C + 1); s.xpzm = at(bm, C + 1); s.xmzp = at(bp, C - 1); s.xmzm = at(bm, C - 1);
  s.ypzp = at(bp, C + UX); s.ypzm = at(bm, C + UX); s.ymzp = at(bp, C - UX); s.ymzm = at(bm, C - UX);
  return s;
}

// Byte offset in an LDS window plane of the sample at (x-1, y-1) of the voxel
// whose centre is value index c, kept opaque so that the compiler addresses
// the stencil from it rather than from the centre (negative offsets, which the
// LDS instructions do not take, would cost extra additions).
template <typename T, int UX>
__device__ __forceinline__ unsigned stencil_base(int c) {
  return lane_offset((unsigned)(c - UX - 1) * (unsigned)sizeof(T));
}

// An LDS address held in a register the compiler may not re-form: reads through
// it take their distance from it as the instruction's immediate offset, so a
// base formed once before a loop costs no address addition inside it.
template <typename T>
using lds_cptr = __attribute__((address_space(3))) const T*;

// Two adjoint values that the gather reads at the same neighbours, kept
// together so that one LDS instruction moves both.
template <typename T>
struct alignas(2 * sizeof(T)) FieldPair {
  T a, b;
};

template <typename T>
__device__ __forceinline__ lds_cptr<T> opaque_lds(const T* p) {
  lds_cptr<T> q = (lds_cptr<T>)p;
  __asm__("" : "+v"(q));
  return q;
}

// Block -> (instance, tile x, tile y, z chunk).
struct BlockTile {
  int inst, logical, per_inst, x0, y0, k0, kend;
};

template <typename T, int TX, int TY>
__device__ __forceinline__ BlockTile block_tile(const SweepArgs<T>& a) {
  BlockTile b;
  b.per_inst = a.ntx * a.nty * a.nzc;
  b.logical = xcd_logical_block(blockIdx.x, b.per_inst * a.batch);
  b.inst = b.logical / b.per_inst;
  int rem = b.logical - b.inst * b.per_inst;
  const int tx = rem % a.ntx;
  rem /= a.ntx;
  const int ty = rem % a.nty;
  const int chunk = rem / a.nty;
  b.x0 = tx * TX;
  b.y0 = ty * TY;
  b.k0 = chunk * a.lz;
  b.kend = min(b.k0 + a.lz, a.nz);
  return b;
}

// Fused forward + adjoint + transposed-stencil gather, then the write of MODE.
// partial[0] = sum of the energy density over the block's output voxels.
//
// Per plane p of the chunk (p = k0-1 .. kend): the u plane p+1, prefetched into
// registers one plane earlier, goes to LDS; barrier; forward + adjoint on the
// (TX+2) x (TY+2) ring-extended plane p; barrier; the gather finishes output
// plane p-1. Each thread evaluates the interior voxels it later gathers, so
// their centre-only adjoints (du, da_z, db_aa) stay in registers and only the
// seven values the neighbours read go through LDS; the one-voxel border of
// the ring is shared out afterwards. The gather takes u at its output voxels
// from registers (read from the slot of plane p-1 before the second barrier),
// so no u slot is read after the second barrier: three rotating u slots and
// two barriers per plane suffice.
//
// BODY: which per-voxel body the kernel holds. kBodyAny picks it per instance
// (a batch that mixes p symmetric in k1, k2 with others); kBodyNoS and
// kBodyFull hold one body only, for batches whose instances all take it: a
// single body needs fewer registers (FP32 32 x 32 tiles: step without S~ terms
// 81 VGPRs against 116 with both bodies; Adam 96 and 123 against 130, where
// both bodies leave one block per CU).
// SP: the coefficients C1..C6 come per voxel from a.cfield (loaded for every
// ring voxel of a plane right after the plane is staged, so their latency
// overlaps the barrier) instead of from the instance's parameters.
// BOX: only voxels inside [box_lo, box_hi) carry a density; the others (the
// padding of a non-periodic field) have zero adjoints, and the gradient is
// written at every voxel, padding included, for the caller to fold back.
template <typename T, int TX, int TY, int NT, int MODE, bool SP = false, bool BOX = false, int BODY = kBodyAny>
__global__ __launch_bounds__(NT) void grad_sweep(SweepArgs<T> a) {
  constexpr int UX = TX + 4, UY = TY + 4;      // u window: interior + halo 2
  constexpr int RX = TX + 2, RY = TY + 2;      // adjoint ring: interior + 1
  constexpr int NU = (UX * UY + NT - 1) / NT;  // u elements staged per thread per plane
  constexpr int NI = TX * TY;                  // interior (output) voxels
  constexpr int NO = (NI + NT - 1) / NT;       // interior voxels per thread
  constexpr int NB = 2 * RX + 2 * TY;          // border voxels of the ring
  constexpr int NW = (NI + NB + NT - 1) / NT;  // ring voxels per thread (interior first)
  // The gather reads a_x's and b_xx's adjoints at the same two neighbours
  // (x +- 1), and a_y's and b_yy's at y +- 1: without a coefficient field each
  // such pair is one 8-byte record (XP, YP: two field rows of sx seen as
  // RY * RX records), written with one instruction and read with one paired
  // instruction per neighbour pair; with one (whose kernels have no registers
  // to spare for the wider reads) the four are rows of their own, in the same
  // storage. BXY, BXZ and BYZ are single fields.
  enum { XP = 0, YP = 2, BXY = 4, BXZ, BYZ, NFIELD };
  constexpr bool kPairs = !SP;
  constexpr bool STEP = MODE != kGrad;

  __shared__ T su[3][UY * UX];
  __shared__ alignas(4 * sizeof(T)) T sx[NFIELD][RY * RX];
  FieldPair<T>* const xrec = reinterpret_cast<FieldPair<T>*>(&sx[XP][0]);   // (a_x / 2, b_xx) adjoints
  FieldPair<T>* const yrec = reinterpret_cast<FieldPair<T>*>(&sx[YP][0]);   // (a_y / 2, b_yy) adjoints
  auto put_xy = [&](int v, T gx, T bxx, T gy, T byy) {
    if constexpr (kPairs) {
      xrec[v] = FieldPair<T>{gx, bxx};
      yrec[v] = FieldPair<T>{gy, byy};
    } else {
      sx[XP][v] = gx; sx[XP + 1][v] = bxx;
      sx[YP][v] = gy; sx[YP + 1][v] = byy;
    }
  };
  __shared__ double sred[NT / kWave][2];

  const int tid = threadIdx.x;
  const BlockTile bt = block_tile<T, TX, TY>(a);
  const int x0 = bt.x0, y0 = bt.y0, k0 = bt.k0, kend = bt.kend;
  const size_t plane = (size_t)a.nx * a.ny;
  const size_t inst_off = (size_t)bt.inst * a.nz * plane;
  const T* srcb = a.src + inst_off;
  T* dstb = a.dst + inst_off;
  const InstParams<T> prm = a.prm[bt.inst];
  // Adam bias corrections 1/(1 - beta^t)
  T bc1 = T(1), bc2 = T(1);
  if (MODE == kStepAdam) {
    const int t = *a.adam_t + a.t_add;
    bc1 = T(1.0 / (1.0 - ::pow(double(a.beta1), double(t))));
    bc2 = T(1.0 / (1.0 - ::pow(double(a.beta2), double(t))));
  }

  // In-plane byte offsets of the u window (periodic wrap in x, y) and of this
  // thread's output voxels, computed once. A plane is under 4 GiB (checked on the
  // host), so every load and store is a block-uniform plane address plus a 32-bit
  // lane offset, with no 64-bit address arithmetic per access.
  unsigned uoff[NU];
#pragma unroll
  for (int j = 0; j < NU; ++j) {
    const int e = tid + j * NT;
    const int ex = e % UX, ey = e / UX;
    uoff[j] = (e < UX * UY)
                  ? (unsigned)(wrap_index(y0 - 2 + ey, a.ny) * a.nx + wrap_index(x0 - 2 + ex, a.nx)) * sizeof(T)
                  : 0u;
  }
  unsigned ooff[NO];
  bool oin[NO];                                // an output voxel inside the grid
#pragma unroll
  for (int j = 0; j < NO; ++j) {
    const int w = tid + j * NT;
    const int gx = x0 + w % TX, gy = y0 + w / TX;
    oin[j] = w < TX * TY && gx < a.nx && gy < a.ny;
    ooff[j] = oin[j] ? (unsigned)(gy * a.nx + gx) * sizeof(T) : 0u;
  }
  T pre[NU];
  T shift = T(0);                              // steps: the uniform shift of src, set below
  const unsigned pbytes = (unsigned)(plane * sizeof(T));
  auto fetch_wrapped = [&](int pw) {          // pw: a plane index already in [0, nz)
    const auto r = plane_rsrc(srcb + (size_t)pw * plane, pbytes);
#pragma unroll
    for (int j = 0; j < NU; ++j)
      if (tid + j * NT < UX * UY) pre[j] = buffer_load(r, uoff[j], T());
  };
  auto fetch = [&](int p) { fetch_wrapped(wrap_index(p, a.nz)); };
  auto stage = [&](int slot) {
#pragma unroll
    for (int j = 0; j < NU; ++j) {
      const int e = tid + j * NT;
      if (e < UX * UY) su[slot][e] = pre[j] + shift;
    }
  };
  // ring position of border voxel b (top row, bottom row, then the two side columns)
  auto border_pos = [](int b) {
    if (b < RX) return b;
    if (b < 2 * RX) return (RY - 1) * RX + (b - RX);
    const int k = b - 2 * RX;
    return (1 + (k >> 1)) * RX + ((k & 1) ? RX - 1 : 0);
  };
  // ring position of this thread's ring item j (interior first, then the border)
  auto ring_pos = [&](int j) {
    const int item = tid + j * NT;
    return item < NI ? (item / TX + 1) * RX + item % TX + 1 : border_pos(item - NI);
  };
  // LDS byte offset of each ring item's stencil base (its (x-1, y-1) sample) in a
  // u window plane, the same in every plane
  unsigned slo[NW];
#pragma unroll
  for (int j = 0; j < NW; ++j) {
    const int v = ring_pos(j);
    slo[j] = stencil_base<T, UX>((v / RX + 1) * UX + v % RX + 1);
  }
  // SP: in-plane offsets of this thread's ring voxels and their coefficients
  const size_t vol = plane * a.nz;
  const VoxelCoeffs<T>* cfb = SP ? coeff_records(a.cfield) + (size_t)bt.inst * vol : nullptr;
  unsigned coff[SP ? NW : 1];                  // byte offsets within a plane of records
  VoxelCoeffs<T> cv[SP ? NW : 1];
  if (SP) {
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      const int item = tid + j * NT;
      int v = 0;
      if (item < NI) v = (item / TX + 1) * RX + item % TX + 1;
      else if (item < NI + NB) v = border_pos(item - NI);
      coff[j] = (unsigned)(wrap_index(y0 - 1 + v / RX, a.ny) * a.nx + wrap_index(x0 - 1 + v % RX, a.nx)) *
                (unsigned)sizeof(VoxelCoeffs<T>);
    }
  }

  double acc_f = 0.0, acc_m = 0.0;
  // The gather reads seven fields around each output voxel, 4.6 KB apart in LDS
  // (beyond the reach of a paired read's immediates), so every field needs an
  // address of its own: with FP32 these are formed once here instead of at
  // every plane (14 registers, which the FP32 kernels without a coefficient
  // field have to spare at two blocks per compute unit).
  constexpr bool kGatherBases = sizeof(T) == 4 && !SP;
  constexpr int NSINGLE = NFIELD - BXY;
  lds_cptr<T> gbase[kGatherBases ? NO : 1][NSINGLE];
  lds_cptr<FieldPair<T>> gxr[kGatherBases ? NO : 1], gyr[kGatherBases ? NO : 1];
  if constexpr (kGatherBases) {
#pragma unroll
    for (int j = 0; j < NO; ++j) {
      const int w = tid + j * NT;
      const int v = w < NI ? (w / TX + 1) * RX + w % TX + 1 : RX + 1;
#pragma unroll
      for (int f = 0; f < NSINGLE; ++f) gbase[j][f] = opaque_lds(&sx[BXY + f][v - RX - 1]);
      gxr[j] = opaque_lds(&xrec[v - RX - 1]);
      gyr[j] = opaque_lds(&yrec[v - RX - 1]);
    }
  }
  // single field f (BXY, BXZ or BYZ) of the ring at index v + d, and the x and
  // y records there, for this thread's output voxel j at v
  auto sxat = [&](int j, int v, int f, int d) -> T {
    if constexpr (kGatherBases) return gbase[j][f - BXY][d + RX + 1];
    else return sx[f][v + d];
  };
  auto xat = [&](int j, int v, int d) -> FieldPair<T> {
    if constexpr (kGatherBases) return FieldPair<T>{gxr[j][d + RX + 1].a, gxr[j][d + RX + 1].b};
    else if constexpr (kPairs) return xrec[v + d];
    else return FieldPair<T>{sx[XP][v + d], sx[XP + 1][v + d]};
  };
  auto yat = [&](int j, int v, int d) -> FieldPair<T> {
    if constexpr (kGatherBases) return FieldPair<T>{gyr[j][d + RX + 1].a, gyr[j][d + RX + 1].b};
    else if constexpr (kPairs) return yrec[v + d];
    else return FieldPair<T>{sx[YP][v + d], sx[YP + 1][v + d]};
  };
  T c_prev[NO], l_prev[NO], l_pp[NO];
  T u_out[NO];                                 // u at this thread's output voxels of plane p-1
  T m1c[NO], m2c[NO], m1n[NO], m2n[NO];        // Adam moments: current and next output plane
#pragma unroll
  for (int j = 0; j < NO; ++j) c_prev[j] = l_prev[j] = l_pp[j] = u_out[j] = m1n[j] = m2n[j] = T(0);

  // plane q lives in slot (q - k0 + 2) mod 3; the three slots rotate
  fetch(k0 - 2);
  // the shift of src, formed by the first wave while the first plane loads
  __shared__ double s_shift;
  if (STEP && tid < kWave) {
    double sf = 0.0, sm = 0.0;
    if (a.prev_partials) instance_sums(a.prev_partials, bt.inst, bt.per_inst, sf, sm);
    if (tid == 0) s_shift = a.prev_partials ? a.mass[bt.inst] - sm * a.inv_nvox : 0.0;
  }
  __syncthreads();
  if (STEP) shift = T(s_shift);
  stage(0);
  fetch(k0 - 1);
  stage(1);
  fetch(k0);

  const int nit = (kend - k0) + 2;             // forward planes k0-1 .. kend
  int sm = 0, sc = 1, sp = 2;                  // slots of p-1, p, p+1
  int pf = wrap_index(k0 + 1, a.nz);           // plane p + 2, wrapped (advanced by one per plane)
  start_priority();
  for (int it = 0; it < nit; ++it) {
    const int p = k0 - 1 + it;
    progress_priority(it, nit);
    stage(sp);
    if (it + 1 < nit) fetch_wrapped(pf);       // plane p + 2, in flight during this plane's compute
    pf = pf + 1 == a.nz ? 0 : pf + 1;
    // Adam moments of output plane p (written in the next iteration), loaded a
    // whole plane ahead: the wait for them then leaves this plane's stores in
    // flight (loads and stores share one in-order counter)
    if (MODE == kStepAdam) {
#pragma unroll
      for (int j = 0; j < NO; ++j) {
        m1c[j] = m1n[j];
        m2c[j] = m2n[j];
      }
      if (it + 1 < nit && p >= k0) {
        const size_t po = inst_off + (size_t)p * plane;
        const auto r1 = plane_rsrc(a.m1 + po, pbytes), r2 = plane_rsrc(a.m2 + po, pbytes);
#pragma unroll
        for (int j = 0; j < NO; ++j) {
          m1n[j] = oin[j] ? buffer_load(r1, ooff[j], T()) : T(0);
          m2n[j] = oin[j] ? buffer_load(r2, ooff[j], T()) : T(0);
        }
      }
    }
    if (SP) {
      const size_t zoff = (size_t)wrap_index(p, a.nz) * plane;
#pragma unroll
      for (int j = 0; j < NW; ++j)
        if (tid + j * NT < NI + NB) {
          // the coefficient records of plane p: a uniform plane address, one lane offset
          const char* cp = reinterpret_cast<const char*>(cfb + zoff);
          cv[j] = *reinterpret_cast<const VoxelCoeffs<T>*>(cp + lane_offset(coff[j]));
        }
    }
    __syncthreads();

    // ---- forward + adjoint on the ring-extended plane p ----
    const bool out_plane = (p >= k0) && (p < kend);
    const int pz = BOX ? wrap_index(p, a.nz) : 0;
    const bool zin = !BOX || (pz >= a.box_lo[2] && pz < a.box_hi[2]);
    auto eval = [&](int v, unsigned lo, VoxelAdjoint<T>& ad, const InstParams<T>& pv) {
      if (BOX) {
        const int gx = wrap_index(x0 - 1 + v % RX, a.nx), gy = wrap_index(y0 - 1 + v / RX, a.ny);
        if (!zin || gx < a.box_lo[0] || gx >= a.box_hi[0] || gy < a.box_lo[1] || gy >= a.box_hi[1]) {
          ad = VoxelAdjoint<T>{};
          put_xy(v, T(0), T(0), T(0), T(0));
          sx[BXY][v] = T(0); sx[BXZ][v] = T(0); sx[BYZ][v] = T(0);
          return T(0);
        }
      }
      const char* pc = reinterpret_cast<const char*>(su[sc]) + lo;
      const char* pm = reinterpret_cast<const char*>(su[sm]) + lo;
      const char* pp = reinterpret_cast<const char*>(su[sp]) + lo;
      // with both bodies, the one without S~ terms where the instance has none,
      // so an instance takes the same arithmetic in every batch it is part of
      // (a coefficient field varies per voxel: always the full body)
      auto st = [&]() { return load_stencil<T, UX>(pc, pm, pp); };
      T f;
      if constexpr (BODY == kBodyNoS)
        f = voxel_density_adjoint_body<true>(st(), st, pv, a.k, ad);
      else if constexpr (BODY == kBodyFull)
        f = voxel_density_adjoint_body<false>(st(), st, pv, a.k, ad);
      else
        f = voxel_density_adjoint<SP>(st(), st, pv, a.k, ad);
      put_xy(v, ad.hgx, ad.nbxx, ad.hgy, ad.nbyy);
      sx[BXY][v] = ad.dbxy; sx[BXZ][v] = ad.dbxz; sx[BYZ][v] = ad.dbyz;
      return f;
    };
    // Interior and border voxels are dealt out from one index space, so the
    // per-thread counts differ by at most one (the border goes to the threads
    // whose interior share is shorter).
    // the centre-only adjoint terms of this thread's output voxels: ub + 2 (b_zz +
    // b_xx + b_yy), a_z and b_zz (the last two also reach the planes above and below)
    T own_c0[NO], own_gz[NO], own_bzz[NO];
    T fpl = T(0);                              // this thread's energy of plane p (one FP64 add per plane)
#pragma unroll
    for (int j = 0; j < NW; ++j) {
      const int item = tid + j * NT;
      if (item < NI + NB) {
        const bool inner = item < NI;
        const int ix = item % TX, iy = item / TX;
        VoxelAdjoint<T> ad;
        const T f = eval(ring_pos(j), slo[j], ad, SP ? with_coeffs(prm, cv[j]) : prm);
        if (j < NO && inner) {
          own_c0[j] = ad.ub + T(2) * ((ad.nbzz + ad.nbxx) + ad.nbyy);
          own_gz[j] = ad.gz;
          own_bzz[j] = ad.nbzz;
          // u of output plane p-1 at this voxel (the stencil's centre in plane
          // p-1), read before the second barrier (its slot takes plane p+2 in
          // the next iteration)
          u_out[j] = *reinterpret_cast<const T*>(reinterpret_cast<const char*>(su[sm]) + slo[j] +
                                                 (UX + 1) * sizeof(T));
          if (out_plane && x0 + ix < a.nx && y0 + iy < a.ny) fpl += f;
        }
      }
    }
    acc_f += double(fpl);
    __syncthreads();

    // ---- transposed stencils on the interior ----
    // The b adjoints are held negated (nb = -df/db), which flips their signs
    // here; the records' first values hold half the a_x, a_y derivatives and BXY, BXZ, BYZ twice
    // the (negated) b_ab ones, hence the factors 2 and 1/2.
    T mpl = T(0);                              // this thread's sum of the field written for plane p - 1
    const size_t po = (size_t)(it >= 2 ? p - 1 : 0) * plane;   // output plane p - 1 (written from it = 2)
    const auto rd = plane_rsrc(dstb + po, pbytes);
    const auto rm1 = plane_rsrc(MODE == kStepAdam ? a.m1 + inst_off + po : dstb, pbytes);
    const auto rm2 = plane_rsrc(MODE == kStepAdam ? a.m2 + inst_off + po : dstb, pbytes);
#pragma unroll
    for (int j = 0; j < NO; ++j) {
      const int w = tid + j * NT;
      if (w < TX * TY) {
        const int ix = w % TX, iy = w / TX;
        const int v = (iy + 1) * RX + ix + 1;
        const T d = T(0.5) * ((sxat(j, v, BXZ, 1) - sxat(j, v, BXZ, -1)) +
                              (sxat(j, v, BYZ, RX) - sxat(j, v, BYZ, -RX)));
        const T bzz = own_bzz[j], gz = own_gz[j];
        const T gd = gz + d;
        const T upn = gd + bzz;        // minus what plane p adds to output plane p-1
        const T lo = gd - bzz;         // what plane p adds to output plane p+1
        if (it >= 2 && oin[j]) {
          const T g = (c_prev[j] - upn) + l_pp[j];
          const unsigned o = ooff[j];
          const T uc = u_out[j];
          if (MODE == kStepGD) {
            const T un = uc - a.tau * g;
            buffer_store(un, rd, o);
            mpl += un;
          } else if (MODE == kStepAdam) {
            const T mo = a.beta1 * m1c[j] + (T(1) - a.beta1) * g;
            const T vo = a.beta2 * m2c[j] + (T(1) - a.beta2) * g * g;
            buffer_store(mo, rm1, o);
            buffer_store(vo, rm2, o);
            const T un = uc - a.tau * (mo * bc1) * rcp_t(sqrt_t(vo * bc2) + a.adam_eps);
            buffer_store(un, rd, o);
            mpl += un;
          } else {
            buffer_store(g, rd, o);
            mpl += uc;
          }
        }
        const FieldPair<T> xp1 = xat(j, v, 1), xm1 = xat(j, v, -1);
        const FieldPair<T> yp1 = yat(j, v, RX), ym1 = yat(j, v, -RX);
        const T cin = own_c0[j]
                      - T(2) * ((xp1.a - xm1.a) + (yp1.a - ym1.a))
                      - ((xp1.b + xm1.b) + (yp1.b + ym1.b))
                      - T(0.5) * ((sxat(j, v, BXY, RX + 1) - sxat(j, v, BXY, -RX + 1)) -
                                  (sxat(j, v, BXY, RX - 1) - sxat(j, v, BXY, -RX - 1)));
        l_pp[j] = l_prev[j];
        l_prev[j] = lo;
        c_prev[j] = cin;

      }
    }
    acc_m += double(mpl);
    // plane p+2 goes where p-1 was: its last reader has passed the second barrier
    const int t = sm;
    sm = sc;
    sc = sp;
    sp = t;
  }

  write_partials<NT>(a, bt.logical, acc_f, acc_m, sred);
}

// Forward only: per-block sums of the energy density and of u. SP: per-voxel
// coefficients from a.cfield.
template <typename T, int TX, int TY, int NT, bool SP = false>
__global__ __launch_bounds__(NT) void energy_sweep(SweepArgs<T> a) {
  constexpr int UX = TX + 2, UY = TY + 2;      // halo 1 suffices for the forward stencil
  constexpr int NU = (UX * UY + NT - 1) / NT;
  constexpr int NO = (TX * TY + NT - 1) / NT;

  __shared__ T su[3][UY * UX];
  __shared__ double sred[NT / kWave][2];

  const int tid = threadIdx.x;
  const BlockTile bt = block_tile<T, TX, TY>(a);
  const int x0 = bt.x0, y0 = bt.y0, k0 = bt.k0, kend = bt.kend;
  const size_t plane = (size_t)a.nx * a.ny;
  const T* srcb = a.src + (size_t)bt.inst * a.nz * plane;
  const InstParams<T> prm = a.prm[bt.inst];

  int uoff[NU];
#pragma unroll
  for (int j = 0; j < NU; ++j) {
    const int e = tid + j * NT;
    const int ex = e % UX, ey = e / UX;
    uoff[j] = (e < UX * UY) ? wrap_index(y0 - 1 + ey, a.ny) * a.nx + wrap_index(x0 - 1 + ex, a.nx) : 0;
  }
  auto load_plane = [&](int p, int slot) {
    const T* sp = srcb + (size_t)wrap_index(p, a.nz) * plane;
#pragma unroll
    for (int j = 0; j < NU; ++j) {
      const int e = tid + j * NT;
      if (e < UX * UY) su[slot][e] = sp[uoff[j]];
    }
  };

  const size_t vol = plane * a.nz;
  const VoxelCoeffs<T>* cfb = SP ? coeff_records(a.cfield) + (size_t)bt.inst * vol : nullptr;
  VoxelCoeffs<T> cv[SP ? NO : 1];

  double acc_f = 0.0, acc_m = 0.0;
  load_plane(k0 - 1, 0);
  load_plane(k0, 1);
  for (int it = 0; it < kend - k0; ++it) {
    const int p = k0 + it;
    const int sm = it % 3, sc = (it + 1) % 3, sp = (it + 2) % 3;
    load_plane(p + 1, sp);
    if (SP) {
#pragma unroll
      for (int j = 0; j < NO; ++j) {
        const int w = tid + j * NT;
        const int gx = x0 + w % TX, gy = y0 + w / TX;
        if (w < TX * TY && gx < a.nx && gy < a.ny)
          cv[j] = cfb[(size_t)p * plane + (size_t)gy * a.nx + gx];
        else
          cv[j] = VoxelCoeffs<T>{};
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NO; ++j) {
      const int w = tid + j * NT;
      if (w >= TX * TY) continue;
      const int ix = w % TX, iy = w / TX;
      const int c = (iy + 1) * UX + ix + 1;
      const unsigned lo = stencil_base<T, UX>(c);
      const char* pc = reinterpret_cast<const char*>(su[sc]) + lo;
      const char* pm = reinterpret_cast<const char*>(su[sm]) + lo;
      const char* pp = reinterpret_cast<const char*>(su[sp]) + lo;
      const Stencil19<T> st = load_stencil<T, UX>(pc, pm, pp);
      const T f = voxel_density<SP>(st, [&]() { return load_stencil<T, UX>(pc, pm, pp); },
                                    SP ? with_coeffs(prm, cv[j]) : prm, a.k);
      if (x0 + ix < a.nx && y0 + iy < a.ny) {
        acc_f += double(f);
        acc_m += double(st.c);
      }
    }
    __syncthreads();
  }

  write_partials<NT>(a, bt.logical, acc_f, acc_m, sred);
}

// Energy only, one x column per lane: a block owns a 64 x (V NWV) tile of
// columns and a chunk of lz planes of one instance; wave w owns rows
// [w V, w V + V) of the tile and lane l the column x0 + l. Per plane the u
// plane (prefetched into registers one plane earlier) is staged in LDS with a
// periodic halo of 1, and after the plane's one barrier every thread copies the
// 3 x (V + 2) window around its V voxels into registers. The windows of three
// consecutive planes hold all 19 stencil samples of the V voxels, so each
// staged value is read from LDS once per thread that needs it (6 reads per
// voxel at V = 2 instead of 19), and the three window roles rotate through an
// unrolled loop instead of moving registers. Two LDS slots suffice: a plane's
// slot is rewritten two planes later, after every thread has passed the
// barrier that follows its last read. Partial [0] is the block's energy.
template <typename T, int V, int NWV>
__global__ __launch_bounds__(64 * NWV) void energy_sweep_cols(SweepArgs<T> a) {
  constexpr int TX = 64, TY = V * NWV, NT = 64 * NWV;
  constexpr int UX = TX + 2, UY = TY + 2;
  constexpr int NU = (UX * UY + NT - 1) / NT;
  constexpr int WR = V + 2;

  __shared__ T su[2][UY * UX];
  __shared__ double sred[NWV][2];

  const int tid = threadIdx.x;
  const int lane = tid % kWave, wv = tid / kWave;
  const BlockTile bt = block_tile<T, TX, TY>(a);
  const int x0 = bt.x0, y0 = bt.y0, k0 = bt.k0, kend = bt.kend;
  const size_t plane = (size_t)a.nx * a.ny;
  const T* srcb = a.src + (size_t)bt.inst * a.nz * plane;
  const InstParams<T> prm = a.prm[bt.inst];

  // byte offsets within a plane (under 4 GiB), as in grad_sweep
  unsigned uoff[NU];
#pragma unroll
  for (int j = 0; j < NU; ++j) {
    const int e = tid + j * NT;
    const int ex = e % UX, ey = e / UX;
    uoff[j] = (e < UX * UY)
                  ? (unsigned)(wrap_index(y0 - 1 + ey, a.ny) * a.nx + wrap_index(x0 - 1 + ex, a.nx)) * sizeof(T)
                  : 0u;
  }
  T pre[NU];
  auto fetch_wrapped = [&](int pw) {          // pw: a plane index already in [0, nz)
    const auto r = plane_rsrc(srcb + (size_t)pw * plane, (unsigned)(plane * sizeof(T)));
#pragma unroll
    for (int j = 0; j < NU; ++j)
      if (tid + j * NT < UX * UY) pre[j] = buffer_load(r, uoff[j], T());
  };
  auto fetch = [&](int p) { fetch_wrapped(wrap_index(p, a.nz)); };
  auto stage = [&](int slot) {
#pragma unroll
    for (int j = 0; j < NU; ++j) {
      const int e = tid + j * NT;
      if (e < UX * UY) su[slot][e] = pre[j];
    }
  };
  // window row r of this thread is tile row wv V + r - 1; column c is x0 + lane + c - 1
  auto read_window = [&](int slot, T (&w)[WR][3]) {
    const T* b = su[slot] + (wv * V) * UX + lane;
#pragma unroll
    for (int r = 0; r < WR; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) w[r][c] = b[r * UX + c];
  };
  const bool xin = x0 + lane < a.nx;
  double acc_f = 0.0;
  T w0[WR][3], w1[WR][3], w2[WR][3];
  // prologue: planes k0 - 1 and k0 into the windows, plane k0 + 1 in flight
  fetch(k0 - 1);
  stage(0);
  fetch(k0);
  __syncthreads();
  read_window(0, w0);
  stage(1);
  fetch(k0 + 1);
  __syncthreads();
  read_window(1, w1);
  // the body without S~ terms where the instance has none (one uniform branch)
  auto run = [&](auto nos_tag) {
    constexpr bool NOS = decltype(nos_tag)::value;
    auto compute = [&](const T (&m)[WR][3], const T (&c)[WR][3], const T (&pl)[WR][3]) {
      T fs = T(0);
#pragma unroll
      for (int r = 0; r < V; ++r) {
        auto st = [&]() {
          Stencil19<T> s;
          s.c = c[r + 1][1];
          s.xm = c[r + 1][0]; s.xp = c[r + 1][2]; s.ym = c[r][1]; s.yp = c[r + 2][1];
          s.zm = m[r + 1][1]; s.zp = pl[r + 1][1];
          s.xpyp = c[r + 2][2]; s.xpym = c[r][2]; s.xmyp = c[r + 2][0]; s.xmym = c[r][0];
          s.xpzp = pl[r + 1][2]; s.xpzm = m[r + 1][2]; s.xmzp = pl[r + 1][0]; s.xmzm = m[r + 1][0];
          s.ypzp = pl[r + 2][1]; s.ypzm = m[r + 2][1]; s.ymzp = pl[r][1]; s.ymzm = m[r][1];
          return s;
        };
        const T f = voxel_density_body<NOS>(st(), st, prm, a.k);
        if (xin && y0 + wv * V + r < a.ny) fs += f;
      }
      acc_f += double(fs);
    };
    // plane p: stage p + 1 (into the slot of p - 1), prefetch p + 2, barrier,
    // window of p + 1, then the V voxels of plane p
    int pf = wrap_index(k0 + 2, a.nz);         // plane p + 2, wrapped (advanced by one per plane)
    auto plane_step = [&](int p, const T (&m)[WR][3], const T (&c)[WR][3], T (&pl)[WR][3]) {
      progress_priority(p - k0, kend - k0);
      const int slot = (p - k0 + 2) & 1;
      stage(slot);
      if (p + 2 <= kend) fetch_wrapped(pf);
      pf = pf + 1 == a.nz ? 0 : pf + 1;
      __syncthreads();
      read_window(slot, pl);
      compute(m, c, pl);
    };
    start_priority();
    for (int p = k0; p < kend; p += 3) {
      plane_step(p, w0, w1, w2);
      if (p + 1 >= kend) break;
      plane_step(p + 1, w1, w2, w0);
      if (p + 2 >= kend) break;
      plane_step(p + 2, w2, w0, w1);
    }
  };
  if (has_s_terms(prm))
    run(std::false_type{});
  else
    run(std::true_type{});
  write_partials<NT>(a, bt.logical, acc_f, 0.0, sred);
}

// Per-instance results of a sweep from its block partials, one wave per
// instance (grid: batch blocks of 64): energy[b] (when given), and, when shift
// is given, shift[b] = mass[b] - mean of the field the sweep summed.
__global__ __launch_bounds__(64) void sweep_finish(const double* __restrict__ partials, int per_inst,
                                                   double* __restrict__ energy, const double* __restrict__ mass,
                                                   double inv_nvox, double* __restrict__ shift) {
  const int b = blockIdx.x;
  double sf, sm;
  instance_sums(partials, b, per_inst, sf, sm);
  if (threadIdx.x == 0) {
    if (energy) energy[b] = sf;
    if (shift) shift[b] = mass[b] - sm * inv_nvox;
  }
}

// Advance the Adam step number by n (one thread; the only writer).
__global__ __launch_bounds__(64) void adam_tick(int* t, int n) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *t += n;
}

// dst[b][i] = src[b][i] + shift[b] (src may equal dst). Grid: x over the
// instance's voxels, y over instances. VEC: 16-byte groups (the host checks
// alignment and that an instance is a whole number of groups), each thread
// issuing its four loads before its four stores.
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  using type = float4;
  static __device__ __forceinline__ float4 add(float4 v, float s) { return make_float4(v.x + s, v.y + s, v.z + s, v.w + s); }
};
template <>
struct Vec16<double> {
  using type = double2;
  static __device__ __forceinline__ double2 add(double2 v, double s) { return make_double2(v.x + s, v.y + s); }
};

template <typename T, bool VEC>
__global__ __launch_bounds__(256) void add_shift(const T* src, T* dst, const double* __restrict__ shift,
                                                 size_t per_inst) {
  const T s = T(shift[blockIdx.y]);
  const T* sb = src + (size_t)blockIdx.y * per_inst;
  T* db = dst + (size_t)blockIdx.y * per_inst;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t i0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if constexpr (VEC) {
    using V = typename Vec16<T>::type;
    constexpr int U = 4;
    const size_t ng = per_inst / (16 / sizeof(T));
    const V* sv = reinterpret_cast<const V*>(sb);
    V* dv = reinterpret_cast<V*>(db);
    for (size_t i = i0; i < ng; i += U * stride) {
      V r[U];
#pragma unroll
      for (int k = 0; k < U; ++k)
        if (i + k * stride < ng) r[k] = sv[i + k * stride];
#pragma unroll
      for (int k = 0; k < U; ++k)
        if (i + k * stride < ng) dv[i + k * stride] = Vec16<T>::add(r[k], s);
    }
  } else {
    for (size_t i = i0; i < per_inst; i += stride) db[i] = sb[i] + s;
  }
}

// The per-instance table with every coefficient of the density of instance b
// (C1..C6 and the orientation term's Co) multiplied by s[b]: the density is
// linear in them, so a gradient sweep with this table gives s_b dF_h/du_b.
// One wave; the geometric constants are copied unchanged.
template <typename T>
__global__ __launch_bounds__(64) void scale_params(const InstParams<T>* __restrict__ src,
                                                   InstParams<T>* __restrict__ dst, const double* __restrict__ s,
                                                   int batch) {
  for (int b = threadIdx.x; b < batch; b += blockDim.x) {
    InstParams<T> q = src[b];
    const double f = s[b];
    q.C1 = T(double(q.C1) * f);
    q.C2 = T(double(q.C2) * f);
    q.C3 = T(double(q.C3) * f);
    q.C4 = T(double(q.C4) * f);
    q.C5 = T(double(q.C5) * f);
    q.C6 = T(double(q.C6) * f);
    q.Co = T(double(q.Co) * f);
    dst[b] = q;
  }
}

// g[b][i] *= s[b] (grid: x over the instance's voxels, y over instances).
template <typename T>
__global__ __launch_bounds__(256) void scale_per_instance(T* g, size_t per_inst, const double* __restrict__ s) {
  const T f = T(s[blockIdx.y]);
  T* gb = g + (size_t)blockIdx.y * per_inst;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < per_inst; i += (size_t)gridDim.x * blockDim.x)
    gb[i] *= f;
}

// Scaled coefficient field from a(x) = (a20, a11, a02, a10, a01, a00)(x)
// ([batch][6][vol] in, [batch][vol] records of six out), the per-voxel form of the
// per-instance C1..C6 (see fe_voxel.hpp): with kq = h^3 s^2 / (2 eps),
// kl = h^3 s / (4h), k0 = h^3 eps / (4h^2) of instance b (k[3b..3b+2]),
// C1 = kq (a20 + a02 - a11), C2 = kq a11, C3 = kq (a20 - a02),
// C4 = kl (a10 + a01), C5 = kl (a10 - a01), C6 = k0 a00.
template <typename T>
__global__ __launch_bounds__(256) void scale_coeff_field(const T* __restrict__ a, T* __restrict__ c, size_t vol,
                                                         int batch, const double* __restrict__ k) {
  const size_t n = vol * (size_t)batch;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const size_t b = i / vol, j = i - b * vol;
    const T* ab = a + b * 6 * vol + j;
    const double a20 = ab[0], a11 = ab[vol], a02 = ab[2 * vol], a10 = ab[3 * vol], a01 = ab[4 * vol],
                 a00 = ab[5 * vol];
    const double kq = k[3 * b], kl = k[3 * b + 1], k0 = k[3 * b + 2];
    VoxelCoeffs<T> r;
    r.c[0] = T(kq * (a20 + a02 - a11));
    r.c[1] = T(kq * a11);
    r.c[2] = T(kq * (a20 - a02));
    r.c[3] = T(kl * (a10 + a01));
    r.c[4] = T(kl * (a10 - a01));
    r.c[5] = T(k0 * a00);
    reinterpret_cast<VoxelCoeffs<T>*>(c)[i] = r;
  }
}

__global__ __launch_bounds__(64) void fill_f64(double* p, int n, double v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Zero both Adam moments and set the step number to 1.
template <typename T>
__global__ __launch_bounds__(256) void adam_reset(T* m1, T* m2, size_t n, int* t) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    m1[i] = T(0);
    m2[i] = T(0);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *t = 1;
}

}  // namespace fe
