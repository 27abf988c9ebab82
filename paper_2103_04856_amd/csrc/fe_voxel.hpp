// Per-voxel arithmetic of the discrete energy F_h and of its adjoint.
//
// The forward chain follows eq. (Meps) and eq. (Feps) (Sec. 3.2) with the
// regularisations of Sec. 4.1: rho = sqrt(|g|^2 + xi^2) replaces |grad u|,
// n (x) n = g g^T / (|g|^2 + xi^2), and the positive part is the softplus
// xi log(1 + exp(x / xi)). The adjoint is the reverse-mode derivative of that
// chain with respect to the stencil values of one voxel.
//
// Units. Everything is written in raw stencil differences of u, which are O(1)
// for any field with |u| <~ 1:
//   a_a  = u(i+e_a) - u(i-e_a)                       = 2h g_a
//   b_aa = u(i+e_a) + u(i-e_a) - 2u(i)               = h^2 H_aa
//   b_ab = u(++) - u(+-) - u(-+) + u(--)             = 4h^2 H_ab
// With s = eps/h^2, lam = h^2/eps^2, Q = |a|^2, R = Q + 4h^2 xi^2:
//   M_aa = s (lam W'(u) a_a^2 / R - b_aa) = s m_aa
//   M_ab = s (4 lam W'(u) a_a a_b / R - b_ab) / 4 = s o_ab / 4
//   Tr M = s T~, ||M||^2 = s^2 N~ with N~ = sum m_aa^2 + sum o_ab^2 / 8,
//   2||M||^2 - (Tr M)^2 = s^2 X~, S = s S~ with S~ = sqrt(softplus_{xi/s^2}(X~)),
//   rho = sqrt(R) / (2h), eps |g|^2 = eps Q / (4h^2).
// The factors s, 1/(2h), h^3 and eps/(4h^2) are folded into six per-instance
// coefficients C1..C6, so that the per-voxel density f~ = h^3 f and F_h is the
// plain sum of f~; its derivatives with respect to a, b and u are then the
// values the transposed stencils spread, with no further scaling.
//
// Precision: X~ is a difference of two nearly equal terms wherever two
// eigenvalues of M nearly coincide (umbilic points, e.g. every point of a
// sphere), and dS/dX = 1/(2S) there, so an X~ with an FP32 rounding error of
// ~1e-7 N~ would leave the gradient at such voxels undetermined. The FP32 path
// therefore evaluates the chain up to X~ in FP32 and, where
// |X~| < 2^-12 (2N~ + T~^2) and that scale is not negligible next to the
// softplus width, evaluates it again in FP64 (differences of FP32 samples are
// exact in FP64). In noise fields this re-evaluation touches under 0.1% of the
// voxels. Everything after X~ (the positive part, the density, the adjoint)
// runs in the storage precision T.
#pragma once

#include <hip/hip_runtime.h>

namespace fe {

// Per-instance constants (see the unit conventions above).
template <typename T>
struct InstParams {
  double lam_d;                // h^2 / eps^2, for the FP64 chain
  T lam;                       // h^2 / eps^2
  T C1, C2, C3, C4, C5, C6;    // h^3 c1 s^2, h^3 c2 s^2, h^3 c3 s^2, h^3 c4 s/(2h), h^3 c5 s/(2h), h^3 c6 eps/(4h^2)
  T xi, inv_xi;                // softplus width in X~ units: xi h^4 / eps^2, and its inverse
  T Co;                        // orientation term of Sec. 5.2: h^3 eps mu / (4h^2) (0: off)
  T thx, thy, thz;             // its direction theta
};

// Grid constants shared by all instances.
template <typename T>
struct GridConsts {
  double reg_d;                // 4 h^2 xi^2 (the xi offset in R), FP64
  T reg;                       // same in T
};

// ---- precision-specific helpers -----------------------------------------

__device__ __forceinline__ float rsqrt_t(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_t(double x) { return 1.0 / __builtin_sqrt(x); }
__device__ __forceinline__ float rcp_t(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float sqrt_t(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double sqrt_t(double x) { return __builtin_sqrt(x); }
__device__ __forceinline__ double rcp_t(double x) { return 1.0 / x; }
__device__ __forceinline__ float exp_t(float x) { return __expf(x); }
__device__ __forceinline__ double exp_t(double x) { return ::exp(x); }
// log(1 + e) for 0 <= e <= 1: log of the rounded sum, corrected by the
// rounding error of that sum to first order (a few ulp, also when 1 + e
// rounds to 1).
__device__ __forceinline__ float log1p_t(float e) {
  const float s = 1.0f + e;
  return __logf(s) - ((s - 1.0f) - e) * __builtin_amdgcn_rcpf(s);
}
__device__ __forceinline__ double log1p_t(double e) { return ::log1p(e); }

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
  T ax, ay, az;                 // raw central differences
  T mxx, myy, mzz;              // m_aa
  T oxy, oxz, oyz;              // o_ab
  T dxx, dyy, dzz;              // 2 m_aa - T~
  T tr, n2, X;                  // T~, N~, X~
  T Q, sw, R, Rinv, rs;         // |a|^2, lam W'(u) / R, R, 1/R, 1/sqrt(R)
};

// Adjoint of one voxel: derivatives of f~ with respect to the raw stencil
// values, which the transposed stencils spread to the neighbours. The b
// entries are returned negated (nb = -df~/db), which the gather absorbs, and
// the in-plane ones in the scale that needs no multiply here (powers of two,
// exact; the gather applies them once per output voxel instead).
template <typename T>
struct VoxelAdjoint {
  T ub;                 // df~/du(i) through W'
  T hgx, hgy;           // df~/da_x / 2, df~/da_y / 2
  T gz;                 // df~/da_z
  T nbxx, nbyy, nbzz;   // -df~/db_aa
  T dbxy, dbxz, dbyz;   // -2 df~/db_ab
};

// The chain up to X~ in FP64 (see the header comment).
template <typename T>
__device__ __forceinline__ Forward<T> forward_fp64(const Stencil19<T>& s, const InstParams<T>& p,
                                                   const GridConsts<T>& k) {
  const double c = s.c;
  const double ax = double(s.xp) - double(s.xm);
  const double ay = double(s.yp) - double(s.ym);
  const double az = double(s.zp) - double(s.zm);
  const double c2u = c + c;
  const double bxx = double(s.xp) + double(s.xm) - c2u;
  const double byy = double(s.yp) + double(s.ym) - c2u;
  const double bzz = double(s.zp) + double(s.zm) - c2u;
  const double bxy = (double(s.xpyp) - double(s.xpym)) - (double(s.xmyp) - double(s.xmym));
  const double bxz = (double(s.xpzp) - double(s.xpzm)) - (double(s.xmzp) - double(s.xmzm));
  const double byz = (double(s.ypzp) - double(s.ypzm)) - (double(s.ymzp) - double(s.ymzm));

  const double axx = ax * ax, ayy = ay * ay, azz = az * az;
  const double Q = axx + ayy + azz;
  const double R = Q + k.reg_d;
  const double Rinv = rcp_f64(R);
  const double sw = p.lam_d * c * (c * c - 1.0) * Rinv;
  const double sw4 = 4.0 * sw;
  const double mxx = sw * axx - bxx;
  const double myy = sw * ayy - byy;
  const double mzz = sw * azz - bzz;
  const double oxy = sw4 * (ax * ay) - bxy;
  const double oxz = sw4 * (ax * az) - bxz;
  const double oyz = sw4 * (ay * az) - byz;
  const double tr = mxx + myy + mzz;
  const double n2 = (mxx * mxx + myy * myy + mzz * mzz) + 0.125 * (oxy * oxy + oxz * oxz + oyz * oyz);

  Forward<T> o;
  o.c = s.c;
  o.ax = T(ax); o.ay = T(ay); o.az = T(az);
  o.mxx = T(mxx); o.myy = T(myy); o.mzz = T(mzz);
  o.oxy = T(oxy); o.oxz = T(oxz); o.oyz = T(oyz);
  o.dxx = T(2.0 * mxx - tr);
  o.dyy = T(2.0 * myy - tr);
  o.dzz = T(2.0 * mzz - tr);
  o.tr = T(tr);
  o.n2 = T(n2);
  o.X = T(2.0 * n2 - tr * tr);
  o.Q = T(Q);
  o.sw = T(sw);
  o.R = T(R);
  o.Rinv = T(Rinv);
  o.rs = T(1.0 / __builtin_sqrt(R));
  return o;
}

// The FP32 chain's re-evaluation where X~ is ill-conditioned: the differences,
// the matrix entries and the invariants again in FP64 from the same samples,
// overwriting only what the cancellation in X~ spoils (m, o, 2m - T~, T~, N~,
// X~). |a|^2, R, 1/R, 1/sqrt(R) and the a themselves carry no cancellation
// (sums of squares; a single difference of two samples is off by at most one
// FP32 rounding), so the FP32 values stand; lam W'(u) / R is formed in FP64
// here because the m_aa subtract it times a_a^2 from b_aa.
__device__ __forceinline__ void redo_fp64(const Stencil19<float>& s, const InstParams<float>& p,
                                          const GridConsts<float>& k, Forward<float>& o) {
  const double c = s.c;
  const double ax = double(s.xp) - double(s.xm);
  const double ay = double(s.yp) - double(s.ym);
  const double az = double(s.zp) - double(s.zm);
  const double c2u = c + c;
  const double bxx = double(s.xp) + double(s.xm) - c2u;
  const double byy = double(s.yp) + double(s.ym) - c2u;
  const double bzz = double(s.zp) + double(s.zm) - c2u;
  const double bxy = (double(s.xpyp) - double(s.xpym)) - (double(s.xmyp) - double(s.xmym));
  const double bxz = (double(s.xpzp) - double(s.xpzm)) - (double(s.xmzp) - double(s.xmzm));
  const double byz = (double(s.ypzp) - double(s.ypzm)) - (double(s.ymzp) - double(s.ymzm));
  const double axx = ax * ax, ayy = ay * ay, azz = az * az;
  const double R = (axx + ayy + azz) + k.reg_d;
  const double sw = p.lam_d * c * (c * c - 1.0) * rcp_f64(R);
  const double sw4 = 4.0 * sw;
  const double mxx = sw * axx - bxx;
  const double myy = sw * ayy - byy;
  const double mzz = sw * azz - bzz;
  const double oxy = sw4 * (ax * ay) - bxy;
  const double oxz = sw4 * (ax * az) - bxz;
  const double oyz = sw4 * (ay * az) - byz;
  const double tr = mxx + myy + mzz;
  const double n2 = (mxx * mxx + myy * myy + mzz * mzz) + 0.125 * (oxy * oxy + oxz * oxz + oyz * oyz);
  o.mxx = float(mxx); o.myy = float(myy); o.mzz = float(mzz);
  o.oxy = float(oxy); o.oxz = float(oxz); o.oyz = float(oyz);
  o.dxx = float(2.0 * mxx - tr);
  o.dyy = float(2.0 * myy - tr);
  o.dzz = float(2.0 * mzz - tr);
  o.tr = float(tr);
  o.n2 = float(n2);
  o.X = float(2.0 * n2 - tr * tr);
}

// Whether the density has the S~ terms: C3 (a20 - a02) and C5 (a10 - a01)
// vanish for every p symmetric in kappa1 and kappa2 (Willmore, Helfrich), and
// then S~, its softplus and dS~/dX~ meet only zero coefficients: f~ and its
// derivatives do without them. The per-voxel functions below take NOS (no S~
// terms) as a template argument; the sweeps pick the body once per call from
// the instance's coefficients, so an instance takes the same arithmetic in
// every batch it is part of.
template <typename T>
__device__ __forceinline__ bool has_s_terms(const InstParams<T>& p) {
  return p.C3 != T(0) || p.C5 != T(0);
}

// The chain up to X~ in FP32, and whether X~ is too ill-conditioned for it.
// With NOS, X~ is left 0 and never redone: the FP64 chain exists for X~, whose
// derivative grows as 1/S~ near umbilic voxels.
template <bool NOS = false>
__device__ __forceinline__ Forward<float> forward_fp32(const Stencil19<float>& s, const InstParams<float>& p,
                                                       const GridConsts<float>& k, bool& redo) {
  Forward<float> o;
  const float c = s.c;
  o.c = c;
  o.ax = s.xp - s.xm;
  o.ay = s.yp - s.ym;
  o.az = s.zp - s.zm;
  const float c2u = c + c;
  const float bxx = (s.xp + s.xm) - c2u;
  const float byy = (s.yp + s.ym) - c2u;
  const float bzz = (s.zp + s.zm) - c2u;
  const float bxy = (s.xpyp - s.xpym) - (s.xmyp - s.xmym);
  const float bxz = (s.xpzp - s.xpzm) - (s.xmzp - s.xmzm);
  const float byz = (s.ypzp - s.ypzm) - (s.ymzp - s.ymzm);

  const float axx = o.ax * o.ax, ayy = o.ay * o.ay, azz = o.az * o.az;
  o.Q = axx + ayy + azz;
  o.R = o.Q + k.reg;
  o.rs = rsqrt_t(o.R);           // one reciprocal square root serves 1/R and rho
  o.Rinv = o.rs * o.rs;
  o.sw = c * (p.lam * (c * c) - p.lam) * o.Rinv;
  const float sw4 = 4.0f * o.sw;
  o.mxx = o.sw * axx - bxx;
  o.myy = o.sw * ayy - byy;
  o.mzz = o.sw * azz - bzz;
  o.oxy = sw4 * (o.ax * o.ay) - bxy;
  o.oxz = sw4 * (o.ax * o.az) - bxz;
  o.oyz = sw4 * (o.ay * o.az) - byz;
  o.tr = o.mxx + o.myy + o.mzz;
  const float d = o.mxx * o.mxx + o.myy * o.myy + o.mzz * o.mzz;
  const float od = o.oxy * o.oxy + o.oxz * o.oxz + o.oyz * o.oyz;
  o.n2 = od * 0.125f + d;
  if constexpr (NOS) {
    o.X = 0.0f;
    redo = false;
  } else {
    const float n2x2 = o.n2 + o.n2;
    o.X = n2x2 - o.tr * o.tr;
    const float scale = n2x2 + o.tr * o.tr;
    redo = (scale > 4096.0f * p.xi) && (fabsf(o.X) < scale * (1.0f / 4096.0f));
  }
  o.dxx = 2.0f * o.mxx - o.tr;
  o.dyy = 2.0f * o.myy - o.tr;
  o.dzz = 2.0f * o.mzz - o.tr;
  return o;
}

// The forward chain in the storage precision; reload() returns the stencil
// again for the (rare) FP64 re-evaluation.
template <bool NOS = false, typename Reload>
__device__ __forceinline__ Forward<double> forward_chain(const Stencil19<double>& s, Reload,
                                                         const InstParams<double>& p,
                                                         const GridConsts<double>& k) {
  return forward_fp64(s, p, k);
}

template <bool NOS = false, typename Reload>
__device__ __forceinline__ Forward<float> forward_chain(const Stencil19<float>& s, Reload reload,
                                                        const InstParams<float>& p,
                                                        const GridConsts<float>& k) {
  bool redo;
  Forward<float> o = forward_fp32<NOS>(s, p, k, redo);
  if (redo) redo_fp64(reload(), p, k, o);
  return o;
}

// Smoothed positive part P = xi log(1 + exp(X/xi)) and its derivative
// sig = logistic(X/xi), in X~ units. Beyond |X| = 40 xi, exp(-|X|/xi) < 5e-18
// is below the rounding unit of either precision, so P = max(X, 0) and
// sig = [X > 0] exactly.
template <typename T>
__device__ __forceinline__ void softplus_xi(T X, const InstParams<T>& p, T& P, T& sig) {
  const T ax = X < T(0) ? -X : X;
  const T mx = X > T(0) ? X : T(0);
  if (ax < T(40) * p.xi) {
    const T e = exp_t(-ax * p.inv_xi);
    P = mx + p.xi * log1p_t(e);
    const T inv = rcp_t(T(1) + e);
    sig = X >= T(0) ? inv : e * inv;
  } else {
    P = mx;
    sig = X > T(0) ? T(1) : T(0);
  }
}

// Forward only: the scaled energy density f~ = h^3 f at one voxel.
// f~ from the forward chain's values.
template <bool NOS = false, typename T>
__device__ __forceinline__ T density_of(const Forward<T>& fw, const InstParams<T>& p) {
  const T rho = fw.R * fw.rs;
  T f;
  if constexpr (NOS) {
    f = p.C1 * fw.n2 + fw.tr * (p.C2 * fw.tr + p.C4 * rho) + p.C6 * fw.Q;
  } else {
    T P, sig;
    softplus_xi(fw.X, p, P, sig);
    const T S = P > T(0) ? P * rsqrt_t(P) : T(0);
    f = p.C1 * fw.n2 + fw.tr * (p.C2 * fw.tr + p.C3 * S + p.C4 * rho) + p.C5 * rho * S + p.C6 * fw.Q;
  }
  if (p.Co != T(0)) {                              // eps mu (theta . g)^2 = Co (theta . a)^2 / h^3
    const T ta = p.thx * fw.ax + p.thy * fw.ay + p.thz * fw.az;
    f += p.Co * ta * ta;
  }
  return f;
}

template <bool NOS, typename T, typename Reload>
__device__ __forceinline__ T voxel_density_body(const Stencil19<T>& s, Reload reload, const InstParams<T>& p,
                                                const GridConsts<T>& k) {
  return density_of<NOS>(forward_chain<NOS>(s, reload, p, k), p);
}

// FULL: the instance may have S~ terms at any voxel (a coefficient field), so
// the full body runs without looking.
template <bool FULL = false, typename T, typename Reload>
__device__ __forceinline__ T voxel_density(const Stencil19<T>& s, Reload reload, const InstParams<T>& p,
                                           const GridConsts<T>& k) {
  if (FULL || has_s_terms(p)) return voxel_density_body<false>(s, reload, p, k);
  return voxel_density_body<true>(s, reload, p, k);
}

// Forward and adjoint at one voxel. Returns f~ and writes its derivatives with
// respect to u(i), a_a and (negated) b_ab.
template <bool NOS, typename T, typename Reload>
__device__ __forceinline__ T voxel_density_adjoint_body(const Stencil19<T>& s, Reload reload,
                                                        const InstParams<T>& p, const GridConsts<T>& k,
                                                        VoxelAdjoint<T>& a) {
  const Forward<T> fw = forward_chain<NOS>(s, reload, p, k);
  const T tr = fw.tr;
  T f, hrhob, trb0, bxx, byy, bzz, cqh;
  const T rs = fw.rs;
  const T rho = fw.R * rs;                         // 2h rho
  const T c1x2 = p.C1 + p.C1;
  // f~ = C1 N~ + T~ g1 + C5 rho~ S~ + C6 Q with g1 = C2 T~ + C3 S~ + C4 rho~, so
  // df/dT~ = g1 + C2 T~ (the product C2 T~ serves both)
  const T ctr = p.C2 * tr;
  if constexpr (NOS) {
    const T g1 = ctr + p.C4 * rho;
    f = p.C1 * fw.n2 + tr * g1 + p.C6 * fw.Q;
    // ---- reverse sweep ----
    hrhob = (T(0.5) * p.C4) * tr;                  // df/drho~ / 2
    trb0 = g1 + ctr;
    bxx = c1x2 * fw.mxx + trb0;
    byy = c1x2 * fw.myy + trb0;
    bzz = c1x2 * fw.mzz + trb0;
    cqh = T(0.5) * p.C1;
  } else {
    T P, sig;
    softplus_xi(fw.X, p, P, sig);
    const T rsP = P > T(0) ? rsqrt_t(P) : T(0);
    const T S = P * rsP;

    const T g1 = (ctr + p.C3 * S) + p.C4 * rho;
    const T c5r = p.C5 * rho;
    f = p.C1 * fw.n2 + tr * g1 + c5r * S + p.C6 * fw.Q;

    // ---- reverse sweep ----
    const T Sb = p.C3 * tr + c5r;                  // df/dS~
    hrhob = (T(0.5) * p.C4) * tr + (T(0.5) * p.C5) * S;   // df/drho~ / 2
    const T kap = Sb * sig * (T(0.5) * rsP);       // df/dX~  (dS~/dX~ = sig / (2S~); 0 where S~ = 0)
    const T kap2 = kap + kap;
    // df/dm_aa = 2 C1 m_aa + df/dT~ + 2 kap (2 m_aa - T~): the X~ part is
    // written with the difference formed in the forward chain, so no two
    // kap-sized terms cancel.
    trb0 = g1 + ctr;
    bxx = c1x2 * fw.mxx + trb0 + kap2 * fw.dxx;
    byy = c1x2 * fw.myy + trb0 + kap2 * fw.dyy;
    bzz = c1x2 * fw.mzz + trb0 + kap2 * fw.dzz;
    cqh = T(0.5) * p.C1 + kap;
  }
  // qh_ab = 2 df/do_ab = (C1/2 + kap) o_ab = -2 df/db_ab
  const T qxy = cqh * fw.oxy, qxz = cqh * fw.oxz, qyz = cqh * fw.oyz;
  // m_aa = sw a_a^2 - b_aa,  o_ab = 4 sw a_a a_b - b_ab
  a.nbxx = bxx;
  a.nbyy = byy;
  a.nbzz = bzz;
  a.dbxy = qxy;
  a.dbxz = qxz;
  a.dbyz = qyz;

  const T ax = fw.ax, ay = fw.ay, az = fw.az, sw = fw.sw;
  // D_a = b_aa a_a + sum_b qh_ab a_b. Since m_aa and o_ab depend on sw through
  // sw a_a^2 and 4 sw a_a a_b, df/dsw = sum_a a_a D_a, and the part of
  // df/da_a / 2 that goes through m and o is sw D_a.
  const T Dx = bxx * ax + qxy * ay + qxz * az;
  const T Dy = byy * ay + qxy * ax + qyz * az;
  const T Dz = bzz * az + qxz * ax + qyz * ay;
  const T swb = ax * Dx + ay * Dy + az * Dz;                              // df/dsw
  // sw = lam W'(u) / R, R = Q + reg, rho~ = sqrt(R)
  const T swbR = swb * fw.Rinv;
  const T Qb = p.C6 + hrhob * rs - swbR * sw;                             // df/dQ
  const T c = fw.c;
  a.ub = swbR * (p.lam * (T(3) * c * c - T(1)));
  // df/da_a / 2 = sw D_a + Qb a_a
  a.hgx = sw * Dx + Qb * ax;
  a.hgy = sw * Dy + Qb * ay;
  T hgz = sw * Dz + Qb * az;
  if (p.Co != T(0)) {                              // orientation term and its derivative in a
    const T ta = p.thx * ax + p.thy * ay + p.thz * az;
    const T tco = p.Co * ta;
    f += tco * ta;
    a.hgx += tco * p.thx;
    a.hgy += tco * p.thy;
    hgz += tco * p.thz;
  }
  a.gz = hgz + hgz;
  return f;
}

// Forward and adjoint at one voxel, the body picked from the coefficients (FULL:
// always the full body, for coefficient fields).
template <bool FULL = false, typename T, typename Reload>
__device__ __forceinline__ T voxel_density_adjoint(const Stencil19<T>& s, Reload reload, const InstParams<T>& p,
                                                   const GridConsts<T>& k, VoxelAdjoint<T>& a) {
  if (FULL || has_s_terms(p)) return voxel_density_adjoint_body<false>(s, reload, p, k, a);
  return voxel_density_adjoint_body<true>(s, reload, p, k, a);
}

}  // namespace fe
