// Per-voxel arithmetic of the discrete energy F_h and of its adjoint.
//
// The forward chain follows eq. (Meps) and eq. (Feps) (Sec. 3.2) with the
// regularisations of Sec. 4.1: rho = sqrt(|g|^2 + xi^2) replaces |grad u|,
// n (x) n = g g^T / (|g|^2 + xi^2), and the positive part is the softplus
// xi log(1 + exp(x / xi)). The adjoint is the reverse-mode derivative of that
// chain with respect to the stencil values (u, g_a, H_ab) of one voxel.
//
// Precision: X = 2||M||^2 - (Tr M)^2 is a difference of two nearly equal terms
// wherever two eigenvalues of M nearly coincide (umbilic points, e.g. every
// point of a sphere), and dS/dX = 1/(2S) there, so an X with an FP32 rounding
// error of ~1e-7 ||M||^2 would leave the gradient at such voxels undetermined.
// The FP32 path therefore evaluates the chain from the stencil differences to
// X in FP32 and, where |X| < 2^-12 (2||M||^2 + (Tr M)^2) and that scale is not
// negligible next to xi, evaluates it again in FP64 (differences of FP32
// samples are exact in FP64). In noise fields this re-evaluation touches
// under 0.1% of the voxels. Everything after X (the positive part, the
// density, the adjoint and the gather) runs in the storage precision T.
#pragma once

#include <hip/hip_runtime.h>

namespace fe {

// Per-instance constants. The adjoint outputs are pre-multiplied by the
// factors the transposed stencils need, so that the gather is adds only:
//   ubar' = h^3 ubar,  gamma' = h^3/(2h) gamma,
//   theta'_aa = h^3/h^2 theta_aa,  theta'_ab = h^3/(4h^2) theta_ab,
// with theta = -eps Mbar folded into the scale.
template <typename T>
struct InstParams {
  double eps_d, inv_eps_d;     // FP64 forward chain
  T eps, inv_eps;
  T c1, c2, c3, c4, c5, c6e;   // c6e = c6 * eps
  T sc_u;                      // h^3
  T sc_gamma;                  // h^3 / (2h)
  T sc_tdiag;                  // -eps h^3 / h^2
  T sc_toff;                   // -eps h^3 / (4 h^2)
};

// Grid constants shared by all instances.
template <typename T>
struct StencilConsts {
  double inv2h;    // 1 / (2h)
  double invh2;    // 1 / h^2
  double inv4h2;   // 1 / (4 h^2)
  double xi2;      // xi^2
  T inv2h_t, invh2_t, inv4h2_t, xi2_t;   // the same in the storage precision
  T xi;            // 1e-6
  T inv_xi;        // 1 / xi
};

// ---- precision-specific helpers -----------------------------------------

__device__ __forceinline__ float rsqrt_t(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_t(double x) { return 1.0 / __builtin_sqrt(x); }
__device__ __forceinline__ float rcp_t(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_t(double x) { return 1.0 / x; }
__device__ __forceinline__ float exp_t(float x) { return __expf(x); }
__device__ __forceinline__ double exp_t(double x) { return ::exp(x); }
__device__ __forceinline__ float log1p_t(float x) { return ::log1pf(x); }
__device__ __forceinline__ double log1p_t(double x) { return ::log1p(x); }

// 1/x in FP64 to full precision: hardware estimate and two Newton steps.
__device__ __forceinline__ double rcp_f64(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, y, 1.0);
  y = __builtin_fma(y, e, y);
  e = __builtin_fma(-x, y, 1.0);
  return __builtin_fma(y, e, y);
}

// The 19 samples of the compact stencil around one voxel.
template <typename T>
struct Stencil19 {
  T c;                          // u(i)
  T xm, xp, ym, yp, zm, zp;     // face neighbours
  T xpyp, xpym, xmyp, xmym;     // xy edges
  T xpzp, xpzm, xmzp, xmzm;     // xz edges
  T ypzp, ypzm, ymzp, ymzm;     // yz edges
};

// What the forward chain hands on, in the storage precision.
template <typename T>
struct Forward {
  T c;                          // u(i)
  T gx, gy, gz;                 // central differences
  T mxx, myy, mzz, mxy, mxz, myz;
  T dxx, dyy, dzz;              // 2 M_aa - Tr M
  T tr, n2, X;                  // Tr M, ||M||^2, 2||M||^2 - (Tr M)^2
  T q;                          // |g|^2
  T sw;                         // W'(u) / (eps (q + xi^2))
  T r;                          // q + xi^2
  T rinv;                       // 1 / r
};

// Adjoint of one voxel, already scaled for the transposed-stencil gather.
template <typename T>
struct VoxelAdjoint {
  T ub;                 // h^3 df/du (through W')
  T gx, gy, gz;         // h^3/(2h) df/dg_a
  T txx, tyy, tzz;      // h^3/h^2 df/dH_aa
  T txy, txz, tyz;      // h^3/(4h^2) df/dH_ab
};

// Stencils, M and its invariants in FP64.
template <typename T>
__device__ __forceinline__ Forward<T> forward_fp64(const Stencil19<T>& s, const InstParams<T>& p,
                                                   const StencilConsts<T>& k) {
  const double c = s.c;
  const double gx = (double(s.xp) - double(s.xm)) * k.inv2h;
  const double gy = (double(s.yp) - double(s.ym)) * k.inv2h;
  const double gz = (double(s.zp) - double(s.zm)) * k.inv2h;
  const double c2u = c + c;
  const double hxx = (double(s.xp) + double(s.xm) - c2u) * k.invh2;
  const double hyy = (double(s.yp) + double(s.ym) - c2u) * k.invh2;
  const double hzz = (double(s.zp) + double(s.zm) - c2u) * k.invh2;
  const double hxy = ((double(s.xpyp) - double(s.xpym)) - (double(s.xmyp) - double(s.xmym))) * k.inv4h2;
  const double hxz = ((double(s.xpzp) - double(s.xpzm)) - (double(s.xmzp) - double(s.xmzm))) * k.inv4h2;
  const double hyz = ((double(s.ypzp) - double(s.ypzm)) - (double(s.ymzp) - double(s.ymzm))) * k.inv4h2;

  const double gxx = gx * gx, gyy = gy * gy, gzz = gz * gz;
  const double q = gxx + gyy + gzz;
  const double r = q + k.xi2;
  const double rinv = rcp_f64(r);
  const double w = c * (c * c - 1.0);                 // W'(u)
  const double sw = w * p.inv_eps_d * rinv;           // W'(u) / (eps (q + xi^2))
  const double e = p.eps_d;

  const double mxx = sw * gxx - e * hxx;
  const double myy = sw * gyy - e * hyy;
  const double mzz = sw * gzz - e * hzz;
  const double mxy = sw * (gx * gy) - e * hxy;
  const double mxz = sw * (gx * gz) - e * hxz;
  const double myz = sw * (gy * gz) - e * hyz;

  const double tr = mxx + myy + mzz;
  const double n2 = mxx * mxx + myy * myy + mzz * mzz + 2.0 * (mxy * mxy + mxz * mxz + myz * myz);

  Forward<T> o;
  o.c = s.c;
  o.gx = T(gx); o.gy = T(gy); o.gz = T(gz);
  o.mxx = T(mxx); o.myy = T(myy); o.mzz = T(mzz);
  o.mxy = T(mxy); o.mxz = T(mxz); o.myz = T(myz);
  o.dxx = T(2.0 * mxx - tr);
  o.dyy = T(2.0 * myy - tr);
  o.dzz = T(2.0 * mzz - tr);
  o.tr = T(tr);
  o.n2 = T(n2);
  o.X = T(2.0 * n2 - tr * tr);
  o.q = T(q);
  o.sw = T(sw);
  o.r = T(r);
  o.rinv = T(rinv);
  return o;
}

// Stencils, M and its invariants in FP32, and whether X is too ill-conditioned
// for that precision (see the header comment).
__device__ __forceinline__ Forward<float> forward_fp32(const Stencil19<float>& s, const InstParams<float>& p,
                                                       const StencilConsts<float>& k, bool& redo) {
  const float c = s.c;
  const float gx = (s.xp - s.xm) * k.inv2h_t;
  const float gy = (s.yp - s.ym) * k.inv2h_t;
  const float gz = (s.zp - s.zm) * k.inv2h_t;
  const float c2u = c + c;
  const float hxx = (s.xp + s.xm - c2u) * k.invh2_t;
  const float hyy = (s.yp + s.ym - c2u) * k.invh2_t;
  const float hzz = (s.zp + s.zm - c2u) * k.invh2_t;
  const float hxy = ((s.xpyp - s.xpym) - (s.xmyp - s.xmym)) * k.inv4h2_t;
  const float hxz = ((s.xpzp - s.xpzm) - (s.xmzp - s.xmzm)) * k.inv4h2_t;
  const float hyz = ((s.ypzp - s.ypzm) - (s.ymzp - s.ymzm)) * k.inv4h2_t;

  const float gxx = gx * gx, gyy = gy * gy, gzz = gz * gz;
  const float q = gxx + gyy + gzz;
  const float r = q + k.xi2_t;
  const float rinv = rcp_t(r);
  const float w = c * (c * c - 1.0f);
  const float sw = w * p.inv_eps * rinv;
  const float e = p.eps;

  Forward<float> o;
  o.mxx = sw * gxx - e * hxx;
  o.myy = sw * gyy - e * hyy;
  o.mzz = sw * gzz - e * hzz;
  o.mxy = sw * (gx * gy) - e * hxy;
  o.mxz = sw * (gx * gz) - e * hxz;
  o.myz = sw * (gy * gz) - e * hyz;
  const float tr = o.mxx + o.myy + o.mzz;
  const float d = o.mxx * o.mxx + o.myy * o.myy + o.mzz * o.mzz;
  const float od = o.mxy * o.mxy + o.mxz * o.mxz + o.myz * o.myz;
  const float n2 = d + 2.0f * od;
  const float tr2 = tr * tr;
  o.X = 2.0f * n2 - tr2;
  const float scale = 2.0f * n2 + tr2;
  redo = (scale > 4096.0f * k.xi) && (fabsf(o.X) < scale * (1.0f / 4096.0f));
  o.c = c;
  o.gx = gx; o.gy = gy; o.gz = gz;
  o.dxx = o.mxx + o.mxx - tr;
  o.dyy = o.myy + o.myy - tr;
  o.dzz = o.mzz + o.mzz - tr;
  o.tr = tr;
  o.n2 = n2;
  o.q = q;
  o.sw = sw;
  o.r = r;
  o.rinv = rinv;
  return o;
}

// The forward chain in the storage precision; reload() returns the stencil
// again for the (rare) FP64 re-evaluation.
template <typename Reload>
__device__ __forceinline__ Forward<double> forward_chain(const Stencil19<double>& s, Reload,
                                                         const InstParams<double>& p,
                                                         const StencilConsts<double>& k) {
  return forward_fp64(s, p, k);
}

template <typename Reload>
__device__ __forceinline__ Forward<float> forward_chain(const Stencil19<float>& s, Reload reload,
                                                        const InstParams<float>& p,
                                                        const StencilConsts<float>& k) {
  bool redo;
  Forward<float> o = forward_fp32(s, p, k, redo);
  if (redo) o = forward_fp64(reload(), p, k);
  return o;
}

// Smoothed positive part P = xi log(1 + exp(X/xi)) and its derivative
// sig = logistic(X/xi). Beyond |X| = 40 xi, exp(-|X|/xi) < 5e-18 is below the
// rounding unit of either precision, so P = max(X, 0) and sig = [X > 0] exactly.
template <typename T>
__device__ __forceinline__ void softplus_xi(T X, const StencilConsts<T>& k, T& P, T& sig) {
  const T ax = X < T(0) ? -X : X;
  if (ax < T(40) * k.xi) {
    const T e = exp_t(-ax * k.inv_xi);
    const T mx = X > T(0) ? X : T(0);
    P = mx + k.xi * log1p_t(e);
    const T inv = rcp_t(T(1) + e);
    sig = X >= T(0) ? inv : e * inv;
  } else {
    P = X > T(0) ? X : T(0);
    sig = X > T(0) ? T(1) : T(0);
  }
}

// Forward only: the energy density f at one voxel.
template <typename T, typename Reload>
__device__ __forceinline__ T voxel_density(const Stencil19<T>& s, Reload reload, const InstParams<T>& p,
                                           const StencilConsts<T>& k) {
  const Forward<T> fw = forward_chain(s, reload, p, k);
  T P, sig;
  softplus_xi(fw.X, k, P, sig);
  const T S = P > T(0) ? P * rsqrt_t(P) : T(0);
  const T rho = fw.r * rsqrt_t(fw.r);
  return p.c1 * fw.n2 + fw.tr * (p.c2 * fw.tr + p.c3 * S + p.c4 * rho) + p.c5 * rho * S + p.c6e * fw.q;
}

// Forward and adjoint at one voxel. Returns the density f; writes the scaled
// partial derivatives of f with respect to u(i), g_a(i) and H_ab(i).
template <typename T, typename Reload>
__device__ __forceinline__ T voxel_density_adjoint(const Stencil19<T>& s, Reload reload, const InstParams<T>& p,
                                                   const StencilConsts<T>& k, VoxelAdjoint<T>& a) {
  const Forward<T> fw = forward_chain(s, reload, p, k);
  const T tr = fw.tr;
  T P, sig;
  softplus_xi(fw.X, k, P, sig);
  const bool pos = P > T(0);
  const T rsP = pos ? rsqrt_t(P) : T(0);
  const T S = P * rsP;
  const T rs = rsqrt_t(fw.r);
  const T rho = fw.r * rs;

  const T f = p.c1 * fw.n2 + tr * (p.c2 * tr + p.c3 * S + p.c4 * rho) + p.c5 * rho * S + p.c6e * fw.q;

  // ---- reverse sweep ----
  const T Sb = p.c3 * tr + p.c5 * rho;               // df/dS
  const T rhob = p.c4 * tr + p.c5 * S;               // df/drho
  const T kap = Sb * sig * (T(0.5) * rsP);           // df/dX  (dS/dX = sig / (2S); 0 where S = 0)
  // df/dM through N2 (c1 + 2 kap), Tr M (trb0 - 2 Tr M kap) and X; the X part
  // of the diagonal is written 2 kap (2 M_aa - Tr M), with the difference formed
  // by the forward chain, so that no two kap-sized terms cancel.
  const T trb0 = T(2) * p.c2 * tr + p.c3 * S + p.c4 * rho;
  const T c1x2 = p.c1 + p.c1;
  const T kap2 = kap + kap;
  const T bxx = c1x2 * fw.mxx + trb0 + kap2 * fw.dxx;   // df/dM_aa
  const T byy = c1x2 * fw.myy + trb0 + kap2 * fw.dyy;
  const T bzz = c1x2 * fw.mzz + trb0 + kap2 * fw.dzz;
  const T n2b4 = T(4) * (p.c1 + kap2);
  const T bxy = n2b4 * fw.mxy;                       // df/dM_ab (both symmetric entries)
  const T bxz = n2b4 * fw.mxz;
  const T byz = n2b4 * fw.myz;

  // M_ab = -eps H_ab + sw g_a g_b
  a.txx = p.sc_tdiag * bxx;
  a.tyy = p.sc_tdiag * byy;
  a.tzz = p.sc_tdiag * bzz;
  a.txy = p.sc_toff * bxy;
  a.txz = p.sc_toff * bxz;
  a.tyz = p.sc_toff * byz;

  const T gx = fw.gx, gy = fw.gy, gz = fw.gz, sw = fw.sw;
  const T swb = bxx * gx * gx + byy * gy * gy + bzz * gz * gz + bxy * gx * gy + bxz * gx * gz + byz * gy * gz;
  // sw = W'(u) / (eps r), r = q + xi^2, rho = sqrt(r)
  const T qb = p.c6e + T(0.5) * rhob * rs - swb * sw * fw.rinv;                       // df/dq
  const T c = fw.c;
  a.ub = p.sc_u * swb * (T(3) * c * c - T(1)) * p.inv_eps * fw.rinv;
  const T qb2 = qb + qb;
  const T bxx2 = bxx + bxx, byy2 = byy + byy, bzz2 = bzz + bzz;
  a.gx = p.sc_gamma * (sw * (bxx2 * gx + bxy * gy + bxz * gz) + qb2 * gx);
  a.gy = p.sc_gamma * (sw * (byy2 * gy + bxy * gx + byz * gz) + qb2 * gy);
  a.gz = p.sc_gamma * (sw * (bzz2 * gz + bxz * gx + byz * gy) + qb2 * gz);
  return f;
}

}  // namespace fe
