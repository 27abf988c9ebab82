// Texture diagnostics from the energy's own stencils, in one sweep:
//   - the diffuse mean and Gaussian curvatures and the diffuse principal
//     curvatures of eqs. (Heps), (Keps), (kepsa), (kepsb) (Sec. 3.1), with
//     |grad u| regularised as rho = sqrt(|g|^2 + xi^2) as in the energy;
//   - the energy F_h (with the coefficient field when one is set), the
//     Cahn-Hilliard area A_eps of eq. (CH_eps) and the
//     normalised discrepancy of Sec. 4.5, with min u and max u (the paper's
//     viability test);
//   - a histogram of (kappa1, kappa2) weighted by h^3 eps |grad u|^2, the
//     density that concentrates on the diffuse interface: a mesh-free stand-in
//     for the curvature diagram of Sec. 4.1.
//
// In the raw stencil units of fe_voxel.hpp (T~, N~, X~, R = |a|^2 + 4h^2 xi^2):
//   H = 2 T~ / (h sqrt R),  K = 2 (T~^2 - N~) / (h^2 R),
//   kappa1,2 = (T~ +- sqrt(max(X~, 0))) / (h sqrt R),
//   eps/2 |g|^2 h^3 = (eps h / 8) Q,  W(u)/eps h^3 = h^3 (1 - u^2)^2 / (4 eps),
//   weight h^3 eps |g|^2 = (eps h / 4) Q.
#pragma once

#include <hip/hip_runtime.h>

#include "fe_kernels.hpp"

namespace fe {

constexpr int kDiagMaxBins = 64;      // per-block histogram in LDS: 64 x 64 FP64 = 32 KiB
constexpr int kDiagStats = 5;         // F_h, A_eps, |discrepancy| sum, min u, max u

struct DiagInst {
  double ca, cb, cw;                  // eps h / 8, h^3 / (4 eps), eps h / 4
};

template <typename T>
struct DiagArgs {
  const DiagInst* inst;               // [batch]
  T* curv;                            // [batch][4][nz][ny][nx] (H, K, kappa1, kappa2) or null
  double* hist;                       // [batch][nbins][nbins] or null
  double* partials;                   // [batch][blocks per instance][kDiagStats]
  int nbins;
  T kmax, bin_scale;                  // bin_scale = nbins / (2 kmax)
  T inv_h, inv_h2;
};

template <typename T>
__device__ __forceinline__ int diag_bin(T k, T kmax, T scale, int nbins) {
  const T kc = k < -kmax ? -kmax : (k > kmax ? kmax : k);
  const int i = (int)__builtin_floor((kc + kmax) * scale);
  return i < nbins - 1 ? i : nbins - 1;
}

// Block = a TX x TY column tile and lz planes (as the energy sweep, halo 1).
// Each block writes its kDiagStats partials; diag_finish reduces them.
template <typename T, int TX, int TY, int NT>
__global__ __launch_bounds__(NT) void diag_sweep(SweepArgs<T> a, DiagArgs<T> d) {
  constexpr int UX = TX + 2, UY = TY + 2;
  constexpr int NU = (UX * UY + NT - 1) / NT;
  constexpr int NO = (TX * TY + NT - 1) / NT;
  static_assert(NO == 1, "the curvatures held for one plane are one voxel per thread");
  __shared__ T su[4][UY * UX];                 // four plane slots: one barrier per plane
  __shared__ double shist[kDiagMaxBins * kDiagMaxBins];
  __shared__ double sred[NT / kWave][kDiagStats];

  const int tid = threadIdx.x;
  const BlockTile bt = block_tile<T, TX, TY>(a);
  const int x0 = bt.x0, y0 = bt.y0, k0 = bt.k0, kend = bt.kend;
  const size_t plane = (size_t)a.nx * a.ny;
  const size_t vol = plane * a.nz;
  const T* srcb = a.src + (size_t)bt.inst * vol;
  const InstParams<T> prm = a.prm[bt.inst];
  const DiagInst di = d.inst[bt.inst];
  const int nb2 = d.hist ? d.nbins * d.nbins : 0;
  for (int i = tid; i < nb2; i += NT) shist[i] = 0.0;

  // byte offsets within a plane (at most 4 GiB - 64 KiB): the u window, and this thread's
  // output voxels for the curvature fields
  unsigned uoff[NU];
#pragma unroll
  for (int j = 0; j < NU; ++j) {
    const int e = tid + j * NT;
    const int ex = e % UX, ey = e / UX;
    uoff[j] = (e < UX * UY)
                  ? (unsigned)(wrap_index(y0 - 1 + ey, a.ny) * a.nx + wrap_index(x0 - 1 + ex, a.nx)) * sizeof(T)
                  : 0u;
  }
  unsigned ooff[NO];
#pragma unroll
  for (int j = 0; j < NO; ++j) {
    const int w = tid + j * NT;
    ooff[j] = (unsigned)((y0 + w / TX) * a.nx + x0 + w % TX) * sizeof(T);
  }
  // the next plane is loaded into registers while the current one is computed
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

  double acc_f = 0.0, acc_area = 0.0, acc_disc = 0.0;
  T umin = T(INFINITY), umax = T(-INFINITY);
  // histogram weight pending for one bin: consecutive voxels of a thread's
  // column often share a bin (smooth fields, and the clamped corner bins), so
  // runs are summed in a register and reach LDS with one atomic
  int run_bin = -1;
  double run_w = 0.0;
  // The curvatures of plane p are stored at the top of the next plane's
  // iteration, before the wait for the plane fetched ahead: loads and stores
  // share one in-order counter, so stores issued after that fetch (at the end of
  // the iteration) would make the wait cover them too. Every iteration issues
  // the four stores (the first to an empty buffer), so the wait is the same on
  // entry and round the loop.
  T held[4] = {T(0), T(0), T(0), T(0)};        // H, K, kappa1, kappa2 of plane p - 1
  unsigned held_off = kDropOffset;
  const unsigned fbytes = d.curv ? (unsigned)(plane * sizeof(T)) : 0u;
  const size_t fstep = d.curv ? vol : 0;       // elements from one curvature field to the next
  auto store_held = [&](int q, bool any) {     // plane q's held curvatures (none unless any)
    const T* cb = d.curv ? d.curv + (size_t)bt.inst * 4 * vol + (size_t)q * plane : a.src;
    const unsigned nb = any ? fbytes : 0u;
#pragma unroll
    for (int f = 0; f < 4; ++f) buffer_store(held[f], plane_rsrc(cb + f * fstep, nb), held_off);
  };
  fetch(k0 - 1);
  stage(0);
  fetch(k0);
  stage(1);
  fetch(k0 + 1);
  int pf = wrap_index(k0 + 2, a.nz);           // plane p + 2, wrapped (advanced by one per plane)
  start_priority();
  for (int it = 0; it < kend - k0; ++it) {
    const int p = k0 + it;
    // planes p - 1, p, p + 1 in slots it, it + 1, it + 2 (mod 4): the slot staged
    // here was last read two planes ago, before the previous plane's barrier
    const int sm = it & 3, sc = (it + 1) & 3, sp = (it + 2) & 3;
    progress_priority(it, kend - k0);
    store_held(it > 0 ? p - 1 : p, it > 0);   // plane p - 1
    stage(sp);                                 // plane p + 1
    if (it + 1 < kend - k0) fetch_wrapped(pf); // plane p + 2, in flight during this plane's compute
    pf = pf + 1 == a.nz ? 0 : pf + 1;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NO; ++j) {
      const int w = tid + j * NT;
      const int ix = w % TX, iy = w / TX;
      const bool valid = w < TX * TY && x0 + ix < a.nx && y0 + iy < a.ny;
      T cH = T(0), cK = T(0), k1 = T(0), k2 = T(0);
      if (valid) {
        const int c = (iy + 1) * UX + ix + 1;
        const unsigned lo = stencil_base<T, UX>(c);
        const char* pc = reinterpret_cast<const char*>(su[sc]) + lo;
        const char* pm = reinterpret_cast<const char*>(su[sm]) + lo;
        const char* pp = reinterpret_cast<const char*>(su[sp]) + lo;
        const Forward<T> fw = forward_chain(load_stencil<T, UX>(pc, pm, pp),
                                            [&]() { return load_stencil<T, UX>(pc, pm, pp); }, prm, a.k);
        const size_t gi = (size_t)p * plane + (size_t)(y0 + iy) * a.nx + (x0 + ix);
        acc_f += double(density_of(
            fw, a.cfield ? with_coeffs(prm, coeff_records(a.cfield)[(size_t)bt.inst * vol + gi]) : prm));
        const T grad_part = T(di.ca) * fw.Q;
        const T w2 = T(1) - fw.c * fw.c;
        const T well_part = T(di.cb) * w2 * w2;
        acc_area += double(grad_part + well_part);
        acc_disc += double(grad_part > well_part ? grad_part - well_part : well_part - grad_part);
        umin = fw.c < umin ? fw.c : umin;
        umax = fw.c > umax ? fw.c : umax;
        if (d.curv || d.hist) {
          const T rs = fw.rs * d.inv_h;                    // 1 / (h sqrt R)
          const T sq = fw.X > T(0) ? sqrt_t(fw.X) : T(0);
          k1 = (fw.tr + sq) * rs;
          k2 = (fw.tr - sq) * rs;
          cH = T(2) * fw.tr * rs;
          cK = T(2) * (fw.tr * fw.tr - fw.n2) * (d.inv_h2 * rcp_t(fw.R));
          if (d.hist) {
            const double wgt = di.cw * double(fw.Q);
            if (wgt != 0.0) {
              const int bin = diag_bin(k1, d.kmax, d.bin_scale, d.nbins) * d.nbins +
                              diag_bin(k2, d.kmax, d.bin_scale, d.nbins);
              if (bin != run_bin) {
                if (run_bin >= 0) unsafeAtomicAdd(&shist[run_bin], run_w);
                run_bin = bin;
                run_w = 0.0;
              }
              run_w += wgt;
            }
          }
        }
      }
      held[0] = cH;
      held[1] = cK;
      held[2] = k1;
      held[3] = k2;
      held_off = valid ? ooff[j] : kDropOffset;
    }
  }
  if (kend > k0) store_held(kend - 1, true);
  if (run_bin >= 0) unsafeAtomicAdd(&shist[run_bin], run_w);

  // block reduction of the five statistics
  double v[kDiagStats] = {acc_f, acc_area, acc_disc, double(umin), double(umax)};
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    v[0] += __shfl_xor(v[0], off, kWave);
    v[1] += __shfl_xor(v[1], off, kWave);
    v[2] += __shfl_xor(v[2], off, kWave);
    v[3] = fmin(v[3], __shfl_xor(v[3], off, kWave));
    v[4] = fmax(v[4], __shfl_xor(v[4], off, kWave));
  }
  const int lane = tid % kWave, wv = tid / kWave;
  if (lane == 0)
    for (int i = 0; i < kDiagStats; ++i) sred[wv][i] = v[i];
  __syncthreads();
  if (tid == 0) {
    double r[kDiagStats] = {0.0, 0.0, 0.0, INFINITY, -INFINITY};
    for (int i = 0; i < NT / kWave; ++i) {
      r[0] += sred[i][0];
      r[1] += sred[i][1];
      r[2] += sred[i][2];
      r[3] = fmin(r[3], sred[i][3]);
      r[4] = fmax(r[4], sred[i][4]);
    }
    double* out = d.partials + (size_t)bt.logical * kDiagStats;
    for (int i = 0; i < kDiagStats; ++i) out[i] = r[i];
  }
  if (d.hist) {
    __syncthreads();
    double* gh = d.hist + (size_t)bt.inst * nb2;
    for (int i = tid; i < nb2; i += NT)
      if (shist[i] != 0.0) unsafeAtomicAdd(&gh[i], shist[i]);
  }
}

// One block per instance: the partials of its blocks summed in a fixed order.
// stats[b] = (F_h, A_eps, discrepancy / A_eps, min u, max u).
__global__ __launch_bounds__(256) void diag_finish(const double* __restrict__ partials, int per_inst,
                                                   double* __restrict__ stats) {
  __shared__ double s[256][kDiagStats];
  const int b = blockIdx.x, t = threadIdx.x;
  const double* pp = partials + (size_t)b * per_inst * kDiagStats;
  double r[kDiagStats] = {0.0, 0.0, 0.0, INFINITY, -INFINITY};
  for (int i = t; i < per_inst; i += 256) {
    r[0] += pp[i * kDiagStats + 0];
    r[1] += pp[i * kDiagStats + 1];
    r[2] += pp[i * kDiagStats + 2];
    r[3] = fmin(r[3], pp[i * kDiagStats + 3]);
    r[4] = fmax(r[4], pp[i * kDiagStats + 4]);
  }
  for (int i = 0; i < kDiagStats; ++i) s[t][i] = r[i];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      s[t][0] += s[t + w][0];
      s[t][1] += s[t + w][1];
      s[t][2] += s[t + w][2];
      s[t][3] = fmin(s[t][3], s[t + w][3]);
      s[t][4] = fmax(s[t][4], s[t + w][4]);
    }
    __syncthreads();
  }
  if (t == 0) {
    double* o = stats + (size_t)b * kDiagStats;
    o[0] = s[0][0];
    o[1] = s[0][1];
    o[2] = s[0][1] > 0.0 ? s[0][2] / s[0][1] : 0.0;
    o[3] = s[0][3];
    o[4] = s[0][4];
  }
}

}  // namespace fe
