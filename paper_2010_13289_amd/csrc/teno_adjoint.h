// Adjoint (vector-Jacobian product) of the flux divergence, with every
// smoothness decision and limiter branch frozen at the state the forward
// map is evaluated on.  With the decisions frozen, the TENO-M output is
// linear in the split fluxes (the weights are the constants d_k; gamma and
// chi reach the output only through the decisions), except for the Van
// Albada slope function, which is differentiated as it stands.  The Euler
// flux, the Roe average, the eigenvectors, the Rusanov alpha (at its
// maximising cell) and the split are differentiated exactly.
//
// Branch convention (also that of the reference adjoint): fmin(a, b) passes
// the derivative to a when a <= b, fmax(a, b) to a when a >= b; a minmod
// passes it to its smallest-magnitude argument when all share a strict sign
// and nowhere otherwise; alpha takes the first maximising cell; |u_n| in
// the signal speed passes sgn(u_n), 0 at u_n = 0.
//
//  k_vjp_tile    Euler system: one workgroup per line tile; the tile's cells
//                are staged in LDS, each thread recomputes one face and
//                pushes its cotangent (from the cotangent of dU/dt) back to
//                the K stencil cells through LDS accumulators, and each cell
//                applies its flux Jacobian once and writes out.
//  k_faces_vjp_scalar, k_gather_vjp   scalar system: one thread per face
//                writes the K stencil contributions per face and slot; one
//                thread per cell sums those of the faces whose stencils hold
//                it, in a fixed order (no atomics).
#pragma once

#include "teno_kernels.h"

namespace tenom {

// ---------------------------------------------------------------------------
// reverse of the branch-free helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ void minmod2_vjp(double x, double y, double obar, double& xbar, double& ybar) {
  // branch-free: the derivative goes to the smaller magnitude (x on a tie)
  // when both share a strict sign, nowhere otherwise
  const bool pos = fmin(x, y) > 0.0, neg = fmax(x, y) < 0.0;
  const bool px = pos ? (x <= y) : (x >= y);
  const double g = (pos || neg) ? obar : 0.0;
  xbar += px ? g : 0.0;
  ybar += px ? 0.0 : g;
}

__device__ __forceinline__ void minmod4_vjp(const double (&a)[4], double obar, double (&abar)[4]) {
  // pairs (0,1), (2,3), then the two winners; the first index wins a tie
  const bool pos = fmin(fmin(a[0], a[1]), fmin(a[2], a[3])) > 0.0;
  const bool neg = fmax(fmax(a[0], a[1]), fmax(a[2], a[3])) < 0.0;
  const bool p01 = pos ? (a[0] <= a[1]) : (a[0] >= a[1]);
  const bool p23 = pos ? (a[2] <= a[3]) : (a[2] >= a[3]);
  const double v01 = p01 ? a[0] : a[1], v23 = p23 ? a[2] : a[3];
  const bool pl = pos ? (v01 <= v23) : (v01 >= v23);
  const double g = (pos || neg) ? obar : 0.0;
  abar[0] += (pl && p01) ? g : 0.0;
  abar[1] += (pl && !p01) ? g : 0.0;
  abar[2] += (!pl && p23) ? g : 0.0;
  abar[3] += (!pl && !p23) ? g : 0.0;
}

// fmin(0, x) / fmax(0, x): the derivative reaches x only when x is chosen
__device__ __forceinline__ double zmin_d(double x) { return (0.0 <= x) ? 0.0 : 1.0; }
__device__ __forceinline__ double zmax_d(double x) { return (0.0 >= x) ? 0.0 : 1.0; }

// Adjoint of the MP bounds: lobar, hibar -> Dbar.
template <int K, int LIM>
__device__ __forceinline__ void mp_bounds_vjp(const double (&D)[K - 1], const TenoParams& tp, const MpState& s,
                                              double lobar, double hibar, double (&Dbar)[K - 1]) {
  constexpr int C0 = K / 2 - 1;
  const double dp = D[C0];
  double dpbar = 0.0, mdbar = 0.0, ulbar = 0.0, lcbar = 0.0;
  // lo = fmax(A1, A2), A1 = fmin(fmin(0, dp), md), A2 = fmin(fmin(0, ul), lc)
  {
    const double m1 = fmin(0.0, dp), A1 = fmin(m1, s.md);
    const double m2 = fmin(0.0, s.ul), A2 = fmin(m2, s.lc);
    const bool s1 = A1 >= A2, t1 = m1 <= s.md, t2 = m2 <= s.lc;
    dpbar += (s1 && t1) ? lobar * zmin_d(dp) : 0.0;
    mdbar += (s1 && !t1) ? lobar : 0.0;
    ulbar += (!s1 && t2) ? lobar * zmin_d(s.ul) : 0.0;
    lcbar += (!s1 && !t2) ? lobar : 0.0;
  }
  // hi = fmin(B1, B2), B1 = fmax(fmax(0, dp), md), B2 = fmax(fmax(0, ul), lc)
  {
    const double n1 = fmax(0.0, dp), B1 = fmax(n1, s.md);
    const double n2 = fmax(0.0, s.ul), B2 = fmax(n2, s.lc);
    const bool s1 = B1 <= B2, t1 = n1 >= s.md, t2 = n2 >= s.lc;
    dpbar += (s1 && t1) ? hibar * zmax_d(dp) : 0.0;
    mdbar += (s1 && !t1) ? hibar : 0.0;
    ulbar += (!s1 && t2) ? hibar * zmax_d(s.ul) : 0.0;
    lcbar += (!s1 && !t2) ? hibar : 0.0;
  }
  // ul = 1.25 dm, md = dp/2 - dR/2, lc = dm/2 + (beta/3) dL
  double dmbar = 1.25 * ulbar + 0.5 * lcbar;
  dpbar += 0.5 * mdbar;
  const double dRbar = -0.5 * mdbar, dLbar = tp.mp_beta3 * lcbar;
  double d_im1bar = 0.0, d_ibar = 0.0, d_ip1bar = 0.0;
  if constexpr (LIM == LIM_MP) {
    double aRbar[4] = {0.0, 0.0, 0.0, 0.0}, aLbar[4] = {0.0, 0.0, 0.0, 0.0};
    minmod4_vjp(s.aR, dRbar, aRbar);
    minmod4_vjp(s.aL, dLbar, aLbar);
    // aR = (4 d_i - d_ip1, 4 d_ip1 - d_i, d_i, d_ip1), aL likewise at i-1/2
    d_ibar += 4.0 * aRbar[0] - aRbar[1] + aRbar[2];
    d_ip1bar += -aRbar[0] + 4.0 * aRbar[1] + aRbar[3];
    d_im1bar += 4.0 * aLbar[0] - aLbar[1] + aLbar[2];
    d_ibar += -aLbar[0] + 4.0 * aLbar[1] + aLbar[3];
  } else {
    minmod2_vjp(s.d_i, s.d_ip1, dRbar, d_ibar, d_ip1bar);
    minmod2_vjp(s.d_im1, s.d_i, dLbar, d_im1bar, d_ibar);
  }
  // d_im1 = D[C0-1] - D[C0-2], d_i = D[C0] - D[C0-1], d_ip1 = D[C0+1] - D[C0]
  Dbar[C0 - 2] -= d_im1bar;
  Dbar[C0 - 1] += d_im1bar - d_ibar + dmbar;
  Dbar[C0] += d_ibar - d_ip1bar + dpbar;
  Dbar[C0 + 1] += d_ip1bar;
}

// Adjoint of one TENO-M reconstruction: vbar += rbar * (d r / d v) with the
// decisions of teno_m on the same v.
// The decisions are passed in (bit k of `mask` set = candidate k smooth),
// as taken by teno_m on the same v.
template <int K, int LIM>
__device__ __forceinline__ void teno_m_vjp_given(const double (&v)[K], const TenoParams& tp, uint32_t mask,
                                                 double rbar, double (&vbar)[K]) {
  using T = TenoTables<K>;
  constexpr int NK = K - 2;
  constexpr int C0 = K / 2 - 1;
  double D[K - 1];
#pragma unroll
  for (int j = 0; j < K - 1; ++j) D[j] = v[j + 1] - v[j];
  bool smooth[NK];
#pragma unroll
  for (int k = 0; k < NK; ++k) smooth[k] = (mask >> k) & 1u;
  double cbar[NK];
  double Dbar[K - 1];
#pragma unroll
  for (int j = 0; j < K - 1; ++j) Dbar[j] = 0.0;
  vbar[C0] += rbar;
  const double dm = D[C0 - 1], dp = D[C0];
  if constexpr (LIM == LIM_TENO) {
    double den = 0.0;
#pragma unroll
    for (int k = 0; k < NK; ++k) den = smooth[k] ? den + T::d(k) : den;
    const double w = rbar * rcp(den);
#pragma unroll
    for (int k = 0; k < NK; ++k) cbar[k] = smooth[k] ? T::d(k) * w : 0.0;
  } else if constexpr (LIM == LIM_MP || LIM == LIM_MP_MM) {
    double c[NK];
    T::candidates(D, c);
    MpState ms;
    mp_bounds<K, LIM>(D, tp, ms);
    double lobar = 0.0, hibar = 0.0;
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      // lim = fmin(fmax(c, lo), hi) on a nonsmooth candidate
      const double w = T::d(k) * rbar;
      const bool in_hi = fmax(c[k], ms.lo) <= ms.hi, ge_lo = c[k] >= ms.lo;
      cbar[k] = (smooth[k] || (in_hi && ge_lo)) ? w : 0.0;
      lobar += (!smooth[k] && in_hi && !ge_lo) ? w : 0.0;
      hibar += (!smooth[k] && !in_hi) ? w : 0.0;
    }
    mp_bounds_vjp<K, LIM>(D, tp, ms, lobar, hibar, Dbar);
  } else {
    double fbar = 0.0;  // cotangent of the TVD-type flux
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const double w = T::d(k) * rbar;
      cbar[k] = smooth[k] ? w : 0.0;
      fbar += smooth[k] ? 0.0 : w;
    }
    double dmbar = 0.0, dpbar = 0.0;
    if constexpr (LIM == LIM_TVD_MINMOD) {
      minmod2_vjp(dm, dp, 0.5 * fbar, dmbar, dpbar);
    } else if constexpr (LIM == LIM_TVD5) {
      const double B = tvd5_b<K>(D);
      const double sbar = 0.5 * fbar;
      double Bbar = 0.0;
      // dm > 0: up = fmax(0, u1), u1 = fmin(u0, B), u0 = fmin(2 dm, 2 dp)
      // dm < 0: dn = fmin(0, w1), w1 = fmax(w0, B), w0 = fmax(2 dm, 2 dp)
      const bool pos = dm > 0.0, neg = dm < 0.0;
      // both sides evaluated, then selected (nested or short-circuit
      // conditionals can become branches)
      const double mn0 = fmin(2.0 * dm, 2.0 * dp), mx0 = fmax(2.0 * dm, 2.0 * dp);
      const double u0 = pos ? mn0 : mx0;
      const double mn1 = fmin(u0, B), mx1 = fmax(u0, B);
      const double u1 = pos ? mn1 : mx1;
      const bool live_p = !(0.0 >= u1), live_n = neg & !(0.0 <= u1);
      const bool live = pos ? live_p : live_n;
      const bool first_p = u0 <= B, first_n = u0 >= B;
      const bool first = pos ? first_p : first_n;
      const bool pick_p = 2.0 * dm <= 2.0 * dp, pick_n = 2.0 * dm >= 2.0 * dp;
      const bool pick_m = pos ? pick_p : pick_n;
      const double g = live ? sbar : 0.0;
      dmbar += (first & pick_m) ? 2.0 * g : 0.0;
      dpbar += (first & !pick_m) ? 2.0 * g : 0.0;
      Bbar += first ? 0.0 : g;
      // B = (-2 D[C0-2] + 11 dm + 24 dp - 3 D[C0+1]) / 30
      const double b30 = Bbar * (1.0 / 30.0);
      Dbar[C0 - 2] += -2.0 * b30;
      dmbar += 11.0 * b30;
      dpbar += 24.0 * b30;
      Dbar[C0 + 1] += -3.0 * b30;
    } else if constexpr (LIM == LIM_VA) {
      const double den = va_den(dm, dp);
      const double rden = rcp(den);
      const double phi = 2.0 * dp * dm * rden;
      const double kp = phi * (1.0 / 3.0);
      const double A = fma(1.0 - kp, dm, (1.0 + kp) * dp);
      // ftvd = phi A / 4
      const double phibar = 0.25 * fbar * (A + phi * (dp - dm) * (1.0 / 3.0));
      dmbar += 0.25 * fbar * phi * (1.0 - kp);
      dpbar += 0.25 * fbar * phi * (1.0 + kp);
      // phi = 2 dp dm / den, den = dp^2 + dm^2 unless raised to its floor
      const bool live = fma(dp, dp, dm * dm) > kVaDenMin;
      dmbar += phibar * (2.0 * dp * rden - (live ? phi * 2.0 * dm * rden : 0.0));
      dpbar += phibar * (2.0 * dm * rden - (live ? phi * 2.0 * dp * rden : 0.0));
    }
    Dbar[C0 - 1] += dmbar;
    Dbar[C0] += dpbar;
  }
  T::candidates_vjp(cbar, Dbar);
#pragma unroll
  for (int j = 0; j < K - 1; ++j) {
    vbar[j + 1] += Dbar[j];
    vbar[j] -= Dbar[j];
  }
}

template <int K, int LIM, bool ADAPT>
__device__ __forceinline__ void teno_m_vjp(const double (&v)[K], const TenoParams& tp, double rbar,
                                           double (&vbar)[K]) {
  double D[K - 1];
#pragma unroll
  for (int j = 0; j < K - 1; ++j) D[j] = v[j + 1] - v[j];
  bool smooth[K - 2];
  teno_cutoff<K, ADAPT>(D, tp, smooth);
  uint32_t mask = 0;
#pragma unroll
  for (int k = 0; k < K - 2; ++k) mask |= (smooth[k] ? 1u : 0u) << k;
  teno_m_vjp_given<K, LIM>(v, tp, mask, rbar, vbar);
}

// Adjoint of one TENO-M reconstruction from its decision code (teno_m with
// FLAGS): with every decision known the map is linear, so nothing of the
// forward is recomputed.  All limiters but Van Albada, whose slope function
// is differentiated at its value (teno_m_vjp_given).  With SKIP, a
// wavefront in which no lane sends a cotangent to the limiter (MP: every
// candidate passed through; TVD: every candidate smooth) skips the
// limiter's reverse, which would only add zeros.
template <int K, int LIM, bool SKIP = false>
__device__ __forceinline__ void teno_m_vjp_code(uint32_t code, const TenoParams& tp, double rbar,
                                                double (&vbar)[K]) {
  static_assert(LIM != LIM_VA, "Van Albada needs the values");
  using T = TenoTables<K>;
  constexpr int NK = K - 2;
  constexpr int C0 = K / 2 - 1;
  double cbar[NK], Dbar[K - 1];
#pragma unroll
  for (int j = 0; j < K - 1; ++j) Dbar[j] = 0.0;
  vbar[C0] += rbar;
  if constexpr (LIM == LIM_TENO) {
    double den = 0.0;
#pragma unroll
    for (int k = 0; k < NK; ++k) den = ((code >> k) & 1u) ? den + T::d(k) : den;
    const double w = rbar * rcp(den);
#pragma unroll
    for (int k = 0; k < NK; ++k) cbar[k] = ((code >> k) & 1u) ? T::d(k) * w : 0.0;
  } else if constexpr (LIM == LIM_MP || LIM == LIM_MP_MM) {
    if constexpr (SKIP) {
      const bool clipped = ((code >> 8) & ((1u << (2 * NK)) - 1u)) != 0u;
      if (__builtin_amdgcn_ballot_w64(clipped) == 0) {  // uniform across the wavefront
#pragma unroll
        for (int k = 0; k < NK; ++k) cbar[k] = T::d(k) * rbar;
        T::candidates_vjp(cbar, Dbar);
#pragma unroll
        for (int j = 0; j < K - 1; ++j) {
          vbar[j + 1] += Dbar[j];
          vbar[j] -= Dbar[j];
        }
        return;
      }
    }
    double lobar = 0.0, hibar = 0.0;
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const double w = T::d(k) * rbar;
      const uint32_t sel = (code >> (8 + 2 * k)) & 3u;
      cbar[k] = sel == 0u ? w : 0.0;
      lobar += sel == 1u ? w : 0.0;
      hibar += sel == 2u ? w : 0.0;
    }
    const uint32_t lo = (code >> 20) & 7u, hi = (code >> 23) & 7u;
    const uint32_t pr = (code >> 26) & 7u, pl = (code >> 29) & 7u;
    double dpbar = (lo == 1u ? lobar : 0.0) + (hi == 1u ? hibar : 0.0);
    const double mdbar = (lo == 2u ? lobar : 0.0) + (hi == 2u ? hibar : 0.0);
    const double ulbar = (lo == 3u ? lobar : 0.0) + (hi == 3u ? hibar : 0.0);
    const double lcbar = (lo == 4u ? lobar : 0.0) + (hi == 4u ? hibar : 0.0);
    // ul = 1.25 dm, md = dp/2 - dR/2, lc = dm/2 + (beta/3) dL
    const double dmbar = 1.25 * ulbar + 0.5 * lcbar;
    dpbar += 0.5 * mdbar;
    const double dRbar = -0.5 * mdbar, dLbar = tp.mp_beta3 * lcbar;
    double d_im1bar = 0.0, d_ibar = 0.0, d_ip1bar = 0.0;
    if constexpr (LIM == LIM_MP) {
      // aR = (4 d_i - d_ip1, 4 d_ip1 - d_i, d_i, d_ip1), aL likewise at i-1/2
      const double r0 = pr == 1u ? dRbar : 0.0, r1 = pr == 2u ? dRbar : 0.0;
      const double r2 = pr == 3u ? dRbar : 0.0, r3 = pr == 4u ? dRbar : 0.0;
      const double l0 = pl == 1u ? dLbar : 0.0, l1 = pl == 2u ? dLbar : 0.0;
      const double l2 = pl == 3u ? dLbar : 0.0, l3 = pl == 4u ? dLbar : 0.0;
      d_ibar += 4.0 * r0 - r1 + r2;
      d_ip1bar += -r0 + 4.0 * r1 + r3;
      d_im1bar += 4.0 * l0 - l1 + l2;
      d_ibar += -l0 + 4.0 * l1 + l3;
    } else {
      // dR = minmod(d_i, d_ip1), dL = minmod(d_im1, d_i)
      d_ibar += pr == 1u ? dRbar : 0.0;
      d_ip1bar += pr == 2u ? dRbar : 0.0;
      d_im1bar += pl == 1u ? dLbar : 0.0;
      d_ibar += pl == 2u ? dLbar : 0.0;
    }
    // d_im1 = D[C0-1] - D[C0-2], d_i = D[C0] - D[C0-1], d_ip1 = D[C0+1] - D[C0]
    Dbar[C0 - 2] -= d_im1bar;
    Dbar[C0 - 1] += d_im1bar - d_ibar + dmbar;
    Dbar[C0] += d_ibar - d_ip1bar + dpbar;
    Dbar[C0 + 1] += d_ip1bar;
  } else {
    double fbar = 0.0;  // cotangent of the TVD-type flux
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const bool sm = (code >> k) & 1u;
      const double w = T::d(k) * rbar;
      cbar[k] = sm ? w : 0.0;
      fbar += sm ? 0.0 : w;
    }
    const uint32_t sel = (code >> 8) & 3u;
    if constexpr (LIM == LIM_TVD_MINMOD) {
      // ftvd = minmod(dm, dp) / 2
      Dbar[C0 - 1] += sel == 1u ? 0.5 * fbar : 0.0;
      Dbar[C0] += sel == 2u ? 0.5 * fbar : 0.0;
    } else {
      // ftvd = (2 dm | 2 dp | B) / 2, B = (-2 D[C0-2] + 11 dm + 24 dp - 3 D[C0+1]) / 30
      const double g = 0.5 * fbar;
      const double b30 = (sel == 3u ? g : 0.0) * (1.0 / 30.0);
      Dbar[C0 - 2] += -2.0 * b30;
      Dbar[C0 - 1] += (sel == 1u ? 2.0 * g : 0.0) + 11.0 * b30;
      Dbar[C0] += (sel == 2u ? 2.0 * g : 0.0) + 24.0 * b30;
      Dbar[C0 + 1] += -3.0 * b30;
    }
  }
  T::candidates_vjp(cbar, Dbar);
#pragma unroll
  for (int j = 0; j < K - 1; ++j) {
    vbar[j + 1] += Dbar[j];
    vbar[j] -= Dbar[j];
  }
}

// ---------------------------------------------------------------------------
// reverse of the per-cell physics
// ---------------------------------------------------------------------------

// Fbar (physical flux) and lambar (signal speed) -> Xbar, for cell_physics.
template <int NF>
__device__ __forceinline__ void cell_physics_vjp(const double (&X)[NF], double gamma, const double (&Fbar)[NF],
                                                 double lambar, double (&Xbar)[NF]) {
  constexpr int ND = NF - 2;
  const double gm1 = gamma - 1.0;
  const double rinv = rcp(X[0]);
  const double un = X[1] * rinv;
  double mu = 0.0;
#pragma unroll
  for (int d = 0; d < ND; ++d) mu = fma(X[1 + d], X[1 + d], mu);
  const double e = fma(-0.5 * rinv, mu, X[NF - 1]);
  const double p = gm1 * e;
  const double c = sqrt(gamma * p * rinv);
  // F0 = X1; F1 = X1 un + p; F_{1+t} = X_{1+t} un; F_E = (E + p) un
  double unbar = Fbar[1] * X[1] + Fbar[NF - 1] * (X[NF - 1] + p);
  double pbar = Fbar[1] + Fbar[NF - 1] * un;
  Xbar[1] += Fbar[0] + Fbar[1] * un;
#pragma unroll
  for (int t = 1; t < ND; ++t) {
    unbar += Fbar[1 + t] * X[1 + t];
    Xbar[1 + t] += Fbar[1 + t] * un;
  }
  Xbar[NF - 1] += Fbar[NF - 1] * un;
  // lam = |un| + c, c = sqrt(gamma p / rho)
  if (lambar != 0.0) {
    unbar += (un > 0.0 ? lambar : (un < 0.0 ? -lambar : 0.0));  // sgn(0) = 0
    const double cbar = lambar;
    // c^2 = gamma p rinv: dc = gamma/(2 c) (rinv dp - p rinv^2 drho)
    const double k = gamma * 0.5 * rcp(c) * cbar;
    pbar += k * rinv;
    Xbar[0] -= k * p * rinv * rinv;
  }
  // p = (gamma-1) (E - |m|^2 / (2 rho))
  Xbar[NF - 1] += gm1 * pbar;
#pragma unroll
  for (int d = 0; d < ND; ++d) Xbar[1 + d] -= gm1 * pbar * X[1 + d] * rinv;
  Xbar[0] += gm1 * pbar * 0.5 * mu * rinv * rinv;
  // un = X1 / rho
  Xbar[1] += unbar * rinv;
  Xbar[0] -= unbar * un * rinv;
}

// Cotangents of the Roe inputs of one cell (sqrt(rho), velocity, H) -> Xbar.
template <int NF>
__device__ __forceinline__ void roe_input_vjp(const double (&X)[NF], double gamma, double rsbar,
                                              const double (&ubar)[NF - 2], double Hbar, double (&Xbar)[NF]) {
  constexpr int ND = NF - 2;
  const double rinv = rcp(X[0]);
  const double rs = sqrt(X[0]);
  // H = (E + p)/rho = gamma E / rho - (gamma-1)/2 q2,  q2 = sum u_d^2, u_d = m_d / rho
  double ub[ND];
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    const double u = X[1 + d] * rinv;
    ub[d] = ubar[d] - (gamma - 1.0) * u * Hbar;
  }
  Xbar[NF - 1] += gamma * rinv * Hbar;
  Xbar[0] -= gamma * X[NF - 1] * rinv * rinv * Hbar;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    const double u = X[1 + d] * rinv;
    Xbar[1 + d] += ub[d] * rinv;
    Xbar[0] -= ub[d] * u * rinv;
  }
  Xbar[0] += rsbar * 0.5 * rcp(rs);
}

// ---------------------------------------------------------------------------
// One Euler face, split by characteristic field.  FaceState holds what all
// fields share (alpha and its maximiser, the Roe average and the
// eigenvector constants), computed exactly as the forward face does;
// FaceBars collects the cotangents of those shared values.
// ---------------------------------------------------------------------------
template <int NF>
struct FaceState {
  double alpha;
  int mstar;
  RoeIn<NF> ra, rb;
  double w;  // 1 / (sqrt(rho_a) + sqrt(rho_b))
  double ut[NF - 2], Ht, q2, ct, cinv, b1, b2;
};

template <int NF>
struct FaceBars {
  double ut[NF - 2], b1, b2, cinv, ct, Ht, q2;
};

// Roe average of the face between cells a (left) and b (right) and the
// eigenvector constants, by the forward face's expressions.
template <int NF>
__device__ __forceinline__ void roe_state(const double (&Xa)[NF], const double (&Xb)[NF], double gamma,
                                          FaceState<NF>& s) {
  constexpr int ND = NF - 2;
  const double gm1 = gamma - 1.0;
  roe_input<NF>(Xa, gamma, s.ra);
  roe_input<NF>(Xb, gamma, s.rb);
  s.w = rcp(s.ra.rs + s.rb.rs);
#pragma unroll
  for (int d = 0; d < ND; ++d) s.ut[d] = fma(s.ra.rs, s.ra.u[d], s.rb.rs * s.rb.u[d]) * s.w;
  s.Ht = fma(s.ra.rs, s.ra.H, s.rb.rs * s.rb.H) * s.w;
  s.q2 = 0.0;
#pragma unroll
  for (int d = 0; d < ND; ++d) s.q2 = fma(s.ut[d], s.ut[d], s.q2);
  s.ct = sqrt(gm1 * fma(-0.5, s.q2, s.Ht));
  s.cinv = rcp(s.ct);
  s.b1 = gm1 * s.cinv * s.cinv;
  s.b2 = 0.5 * s.q2 * s.b1;
}

// Row Q of the left-eigenvector projection (the expressions of the forward
// face, so the values are the same bits).
template <int NF, int Q>
__device__ __forceinline__ double project_row(const FaceState<NF>& s, const double (&Y)[NF]) {
  constexpr int ND = NF - 2;
  if constexpr (Q == 0 || Q == 1 || Q == NF - 1) {
    double um = 0.0;
#pragma unroll
    for (int d = 0; d < ND; ++d) um = fma(s.ut[d], Y[1 + d], um);
    const double A = fma(s.b2, Y[0], s.b1 * (Y[NF - 1] - um));
    if constexpr (Q == 1) {
      return Y[0] - A;
    } else {
      const double Bn = fma(s.ut[0], Y[0], -Y[1]);
      return Q == 0 ? 0.5 * fma(Bn, s.cinv, A) : 0.5 * fma(-Bn, s.cinv, A);
    }
  } else {
    return fma(-s.ut[Q - 1], Y[0], Y[Q]);
  }
}

// Gradient of row Q of the projection with respect to the projected vector
// (the row of L: constant across the face's stencil).
template <int NF, int Q>
__device__ __forceinline__ void project_row_grad(const FaceState<NF>& s, double (&g)[NF]) {
  constexpr int ND = NF - 2;
#pragma unroll
  for (int r = 0; r < NF; ++r) g[r] = 0.0;
  if constexpr (Q == 1) {
    // w1 = Y0 - A, A = b2 Y0 + b1 (Y_E - ut . Y_mom)
    g[0] = 1.0 - s.b2;
#pragma unroll
    for (int d = 0; d < ND; ++d) g[1 + d] = s.b1 * s.ut[d];
    g[NF - 1] = -s.b1;
  } else if constexpr (Q == 0 || Q == NF - 1) {
    // w = (A +- Bn cinv) / 2, Bn = ut0 Y0 - Y1
    const double sg = (Q == 0) ? 1.0 : -1.0;
    g[0] = 0.5 * fma(sg * s.ut[0], s.cinv, s.b2);
    g[1] = 0.5 * fma(-s.b1, s.ut[0], -sg * s.cinv);
#pragma unroll
    for (int d = 1; d < ND; ++d) g[1 + d] = -0.5 * s.b1 * s.ut[d];
    g[NF - 1] = 0.5 * s.b1;
  } else {
    // w = Y_Q - ut_{Q-1} Y0
    g[0] = -s.ut[Q - 1];
    g[Q] = 1.0;
  }
}

// Adjoint of project_row: ob -> Yb and the cotangents of the constants.
template <int NF, int Q>
__device__ __forceinline__ void project_row_vjp(const FaceState<NF>& s, const double (&Y)[NF], double ob,
                                                double (&Yb)[NF], FaceBars<NF>& b) {
  constexpr int ND = NF - 2;
  if constexpr (Q == 0 || Q == 1 || Q == NF - 1) {
    double um = 0.0;
#pragma unroll
    for (int d = 0; d < ND; ++d) um = fma(s.ut[d], Y[1 + d], um);
    double Abar;
    if constexpr (Q == 1) {
      Yb[0] += ob;
      Abar = -ob;
    } else {
      const double Bn = fma(s.ut[0], Y[0], -Y[1]);
      const double sg = (Q == 0) ? 0.5 : -0.5;
      Abar = 0.5 * ob;
      const double Bnbar = sg * s.cinv * ob;
      b.cinv += sg * Bn * ob;
      b.ut[0] += Bnbar * Y[0];
      Yb[0] += Bnbar * s.ut[0];
      Yb[1] -= Bnbar;
    }
    // A = b2 Y0 + b1 (Y_E - um)
    b.b2 += Abar * Y[0];
    Yb[0] += Abar * s.b2;
    b.b1 += Abar * (Y[NF - 1] - um);
    Yb[NF - 1] += Abar * s.b1;
    const double umbar = -Abar * s.b1;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      b.ut[d] += umbar * Y[1 + d];
      Yb[1 + d] += umbar * s.ut[d];
    }
  } else {
    Yb[0] -= s.ut[Q - 1] * ob;
    Yb[Q] += ob;
    b.ut[Q - 1] -= Y[0] * ob;
  }
}

// Left-eigenvector projection w = L Y of a conservative vector (the forward
// face's expressions, so the values are the same bits).
template <int NF>
__device__ __forceinline__ void project_all(const FaceState<NF>& s, const double (&Y)[NF], double (&w)[NF]) {
  constexpr int ND = NF - 2;
  double um = 0.0;
#pragma unroll
  for (int d = 0; d < ND; ++d) um = fma(s.ut[d], Y[1 + d], um);
  const double A = fma(s.b2, Y[0], s.b1 * (Y[NF - 1] - um));
  const double Bn = fma(s.ut[0], Y[0], -Y[1]);
  w[0] = 0.5 * fma(Bn, s.cinv, A);
  w[1] = Y[0] - A;
#pragma unroll
  for (int t = 1; t < ND; ++t) w[1 + t] = fma(-s.ut[t], Y[0], Y[1 + t]);
  w[NF - 1] = 0.5 * fma(-Bn, s.cinv, A);
}

// Adjoint of project_all: wb -> Yb (added) and the cotangents of the
// eigenvector constants (added to b).
template <int NF>
__device__ __forceinline__ void project_all_vjp(const FaceState<NF>& s, const double (&Y)[NF], const double (&wb)[NF],
                                                double (&Yb)[NF], FaceBars<NF>& b) {
  constexpr int ND = NF - 2;
  double um = 0.0;
#pragma unroll
  for (int d = 0; d < ND; ++d) um = fma(s.ut[d], Y[1 + d], um);
  const double Bn = fma(s.ut[0], Y[0], -Y[1]);
  // w0 = (A + Bn cinv)/2, wE = (A - Bn cinv)/2, w1 = Y0 - A
  const double Abar = 0.5 * (wb[0] + wb[NF - 1]) - wb[1];
  const double hd = 0.5 * (wb[0] - wb[NF - 1]);
  const double Bnbar = hd * s.cinv;
  b.cinv += hd * Bn;
  Yb[0] += wb[1];
  // w_{1+t} = Y_{1+t} - ut_t Y0
#pragma unroll
  for (int t = 1; t < ND; ++t) {
    Yb[0] -= s.ut[t] * wb[1 + t];
    Yb[1 + t] += wb[1 + t];
    b.ut[t] -= Y[0] * wb[1 + t];
  }
  // Bn = ut0 Y0 - Y1
  b.ut[0] += Bnbar * Y[0];
  Yb[0] += Bnbar * s.ut[0];
  Yb[1] -= Bnbar;
  // A = b2 Y0 + b1 (Y_E - um), um = ut . Y_mom
  b.b2 += Abar * Y[0];
  Yb[0] += Abar * s.b2;
  b.b1 += Abar * (Y[NF - 1] - um);
  Yb[NF - 1] += Abar * s.b1;
  const double umbar = -Abar * s.b1;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    b.ut[d] += umbar * Y[1 + d];
    Yb[1 + d] += umbar * s.ut[d];
  }
}

// Adjoint of the back-projection F = R fc: Fhbar -> fcbar, and the shared
// cotangents (added only when `shared`).
template <int NF>
__device__ __forceinline__ void backproj_vjp(const FaceState<NF>& s, const double (&fc)[NF], const double (&Fhbar)[NF],
                                             double (&fcbar)[NF], FaceBars<NF>& b, bool shared) {
  constexpr int ND = NF - 2;
  const double sum = fc[0] + fc[1] + fc[NF - 1];
  const double dlr = fc[NF - 1] - fc[0];
  const double ebar = Fhbar[NF - 1];
  double sbar = Fhbar[0] + Fhbar[1] * s.ut[0];
  const double dlrbar = Fhbar[1] * s.ct + ebar * s.ut[0] * s.ct;
#pragma unroll
  for (int q = 0; q < NF; ++q) fcbar[q] = 0.0;
  fcbar[0] += ebar * s.Ht;
  fcbar[NF - 1] += ebar * s.Ht;
  fcbar[1] += ebar * 0.5 * s.q2;
#pragma unroll
  for (int t = 1; t < ND; ++t) {
    sbar += Fhbar[1 + t] * s.ut[t];
    fcbar[1 + t] += Fhbar[1 + t] + ebar * s.ut[t];
  }
  fcbar[0] += sbar - dlrbar;
  fcbar[1] += sbar;
  fcbar[NF - 1] += sbar + dlrbar;
  if (shared) {
    b.ut[0] += Fhbar[1] * sum + ebar * s.ct * dlr;
    b.ct += Fhbar[1] * dlr + ebar * s.ut[0] * dlr;
    b.Ht += ebar * (fc[0] + fc[NF - 1]);
    b.q2 += ebar * 0.5 * fc[1];
#pragma unroll
    for (int t = 1; t < ND; ++t) b.ut[t] += Fhbar[1 + t] * sum + ebar * fc[1 + t];
  }
}

// Shared cotangents -> Xbar of the two cells of the Roe average: through the
// eigenvector constants, the Roe average and the Roe inputs.
template <int NF>
__device__ __forceinline__ void shared_vjp(const double (&Xa)[NF], const double (&Xb)[NF], const FaceState<NF>& s,
                                           double gamma, FaceBars<NF> b, double (&Xabar)[NF], double (&Xbbar)[NF]) {
  constexpr int ND = NF - 2;
  const double gm1 = gamma - 1.0;
  // b2 = q2 b1 / 2, b1 = (gamma-1) cinv^2, cinv = 1/ct, ct = sqrt((gamma-1)(Ht - q2/2))
  b.q2 += 0.5 * s.b1 * b.b2;
  b.b1 += 0.5 * s.q2 * b.b2;
  b.cinv += 2.0 * gm1 * s.cinv * b.b1;
  b.ct -= s.cinv * s.cinv * b.cinv;
  {
    const double k = gm1 * 0.5 * s.cinv * b.ct;
    b.Ht += k;
    b.q2 -= 0.5 * k;
  }
#pragma unroll
  for (int d = 0; d < ND; ++d) b.ut[d] += 2.0 * s.ut[d] * b.q2;
  // ut = (rs_a u_a + rs_b u_b) w, Ht = (rs_a H_a + rs_b H_b) w
  double rsabar = 0.0, rsbbar = 0.0, uabar[ND], ubbar[ND];
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    uabar[d] = b.ut[d] * s.ra.rs * s.w;
    ubbar[d] = b.ut[d] * s.rb.rs * s.w;
    rsabar += b.ut[d] * (s.ra.u[d] - s.ut[d]) * s.w;
    rsbbar += b.ut[d] * (s.rb.u[d] - s.ut[d]) * s.w;
  }
  rsabar += b.Ht * (s.ra.H - s.Ht) * s.w;
  rsbbar += b.Ht * (s.rb.H - s.Ht) * s.w;
  roe_input_vjp<NF>(Xa, gamma, rsabar, uabar, b.Ht * s.ra.rs * s.w, Xabar);
  roe_input_vjp<NF>(Xb, gamma, rsbbar, ubbar, b.Ht * s.rb.rs * s.w, Xbbar);
}

// Scalar advection f = a u: Fbar -> ubar.
template <int K, int LIM, bool ADAPT>
__device__ __forceinline__ void scalar_face_vjp(const double (&u)[K], double a, const TenoParams& tp, double Fbar,
                                                double (&ubar)[K]) {
  const double alpha = fabs(a);
  double vp[K], vm[K];
#pragma unroll
  for (int m = 0; m < K; ++m) lf_split2(a * u[m], alpha, u[m], vp[m], vm[K - 1 - m]);
  double vpbar[K], vmbar[K];
#pragma unroll
  for (int m = 0; m < K; ++m) vpbar[m] = vmbar[m] = 0.0;
  teno_m_vjp<K, LIM, ADAPT>(vp, tp, 0.5 * Fbar, vpbar);
  teno_m_vjp<K, LIM, ADAPT>(vm, tp, 0.5 * Fbar, vmbar);
#pragma unroll
  for (int m = 0; m < K; ++m) ubar[m] += (a + alpha) * vpbar[m] + (a - alpha) * vmbar[K - 1 - m];
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// Faces of one axis in the adjoint: n + 1 for a transmissive axis (both
// ends are faces), n for a periodic one (face n is face 0).
struct VjpAxis {
  int nx, ny, nz;  // cells
  int axis, bc;
  int n;           // cells along the axis
  int nfa;         // faces along the axis
  long nfaces;     // faces of the axis
  double inv_dx;
};

__device__ __forceinline__ void vjp_face_line(const VjpAxis& a, long t, Line& L, int& j) {
  const int fnx = a.axis == 0 ? a.nfa : a.nx;
  const int fny = a.axis == 1 ? a.nfa : a.ny;
  const int fx = (int)(t % fnx);
  const int fy = (int)((t / fnx) % fny);
  const int fz = (int)(t / ((long)fnx * fny));
  if (a.axis == 0) {
    L = Line{(long)a.nx * (fy + (long)a.ny * fz), 1, a.n, a.bc};
    j = fx;
  } else if (a.axis == 1) {
    L = Line{fx + (long)a.nx * a.ny * fz, a.nx, a.n, a.bc};
    j = fy;
  } else {
    L = Line{fx + (long)a.nx * fy, (long)a.nx * a.ny, a.n, a.bc};
    j = fz;
  }
}

// Face cotangent from the cotangent of dU/dt: dU/dt_i = -(F_{i+1} - F_i)/dx
// (face j between cells j-1 and j), so Fbar_j = (Lbar_j - Lbar_{j-1}) / dx
// over the cells that exist.
template <int NF>
__device__ __forceinline__ void face_cotangent(const VjpAxis& ax, const Line& L, int j, long N, const int (&fld)[NF],
                                               const double* __restrict__ Lbar, double (&Fhbar)[NF]) {
  const bool per = (ax.bc == 0);
  const bool has_r = per || j < ax.n;
  const bool has_l = per || j > 0;
  const long cr = cell_at(L, per ? j : min(j, ax.n - 1));
  const long cl = cell_at(L, j - 1);
#pragma unroll
  for (int q = 0; q < NF; ++q) {
    const double r = has_r ? Lbar[(long)fld[q] * N + cr] : 0.0;
    const double l = has_l ? Lbar[(long)fld[q] * N + cl] : 0.0;
    Fhbar[q] = (r - l) * ax.inv_dx;
  }
}

// Scalar system: one thread per face.
// contrib[(m * NF + field) * nfaces + face] = d(Lbar . dU/dt)/dU at stencil slot m
template <int K, int LIM, bool ADAPT>
__global__ __launch_bounds__(256) void k_faces_vjp_scalar(const double* __restrict__ U,
                                                          const double* __restrict__ Lbar,
                                                          double* __restrict__ contrib, VjpAxis ax, FaceParams fp) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ax.nfaces) return;
  Line L;
  int j;
  vjp_face_line(ax, t, L, j);
  const long N = (long)ax.nx * ax.ny * ax.nz;
  const int fld[1] = {0};
  double Fhbar[1];
  face_cotangent<1>(ax, L, j, N, fld, Lbar, Fhbar);
  double u[K], ub[K];
#pragma unroll
  for (int m = 0; m < K; ++m) {
    u[m] = U[cell_at(L, j - K / 2 + m)];
    ub[m] = 0.0;
  }
  scalar_face_vjp<K, LIM, ADAPT>(u, fp.adv, fp.tp, Fhbar[0], ub);
#pragma unroll
  for (int m = 0; m < K; ++m) contrib[(long)m * ax.nfaces + t] = ub[m];
}

// Doubled split values of field Q at one face from the staged cells.
template <int NF, int K, int Q, int P>
__device__ __forceinline__ void field_split(const double* sX, const double* sF, int t, const FaceState<NF>& s,
                                            double (&vp)[K], double (&vm)[K], double (&W)[K]) {
#pragma unroll
  for (int m = 0; m < K; ++m) {
    double X[NF], F[NF];
#pragma unroll
    for (int r = 0; r < NF; ++r) {
      X[r] = sX[r * P + t + m];
      F[r] = sF[r * P + t + m];
    }
    W[m] = project_row<NF, Q>(s, X);
    lf_split2(project_row<NF, Q>(s, F), s.alpha, W[m], vp[m], vm[K - 1 - m]);
  }
}

// Forward of field Q at one face: fc_Q = (TENO(g+) + TENO(g-)) / 2 (doubled
// split), with the decision codes of both reconstructions and W_m = row Q
// of L applied to the stencil states (kept for the reverse).
template <int NF, int K, int LIM, bool ADAPT, int Q, int P>
__device__ __forceinline__ double field_fwd(const double* sX, const double* sF, int t, const FaceState<NF>& s,
                                            const TenoParams& tp, double (&W)[K], uint32_t& cp, uint32_t& cm) {
  double vp[K], vm[K];
  field_split<NF, K, Q, P>(sX, sF, t, s, vp, vm, W);
  cp = cm = 0u;
  // (no limiter skip here: where most wavefronts are rough, as in a fluid at
  // rest whose acoustic fields carry rounding noise, the skip's branches
  // cost the kernel 5 %; the reverse keeps its skip, which costs nothing
  // measurable there)
  return 0.5 * (teno_m<K, LIM, true, ADAPT>(vp, tp, cp) + teno_m<K, LIM, true, ADAPT>(vm, tp, cm));
}

// Ordering of LDS accesses between lanes of one wavefront: the hardware
// executes a wavefront's LDS instructions in order, and this keeps the
// compiler from moving accesses across the point.
__device__ __forceinline__ void wave_lds_order() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Per-wavefront accumulators of one field: slot lane + m of each [NF][AP]
// array collects stencil cell m of the face of `lane`.
struct FieldAcc {
  double* x;    // cotangent of the cell state (direct part)
  double* f;    // cotangent of the cell's physical flux
  double* lam;  // cotangent of the cell's signal speed
  int lane;
  bool live;
};

// Reverse of field Q: fcbar -> the cotangents of the field's split values
// (from the decision codes), then of the stencil states and fluxes through
// row Q of L (added to the wave's accumulators), of alpha, and of the
// eigenvector constants (b).
template <int NF, int K, int LIM, int Q, int P, int AP>
__device__ __forceinline__ void field_rev(const double* sX, const double* sF, int t, const FaceState<NF>& s,
                                          const TenoParams& tp, const double (&W)[K], uint32_t cp, uint32_t cm,
                                          double fcbar, const FieldAcc& a, FaceBars<NF>& b) {
  double vpbar[K], vmbar[K];
#pragma unroll
  for (int m = 0; m < K; ++m) vpbar[m] = vmbar[m] = 0.0;
  if constexpr (LIM == LIM_VA) {
    double vp[K], vm[K], Wd[K];
    field_split<NF, K, Q, P>(sX, sF, t, s, vp, vm, Wd);
    teno_m_vjp_given<K, LIM>(vp, tp, cp, 0.5 * fcbar, vpbar);
    teno_m_vjp_given<K, LIM>(vm, tp, cm, 0.5 * fcbar, vmbar);
  } else {
    teno_m_vjp_code<K, LIM, true>(cp, tp, 0.5 * fcbar, vpbar);
    teno_m_vjp_code<K, LIM, true>(cm, tp, 0.5 * fcbar, vmbar);
  }
  double g[NF];
  project_row_grad<NF, Q>(s, g);
  constexpr bool full = (Q == 0 || Q == 1 || Q == NF - 1);
  // The constants' cotangents are bilinear in (row cotangent, projected
  // vector): accumulate sum_m Wb_m U_m and sum_m Gb_m F_m and take the
  // row's adjoint once with cotangent 1.
  double SX[NF], SF[NF];
#pragma unroll
  for (int r = 0; r < NF; ++r) SX[r] = SF[r] = 0.0;
  // vp[m] = G + alpha W, vm[K-1-m] = G - alpha W: the field's part of alphabar
  // first, so that it joins the stencil step of the maximising cell
  double alphabar = 0.0;
#pragma unroll
  for (int m = 0; m < K; ++m) alphabar += W[m] * (vpbar[m] - vmbar[K - 1 - m]);
#pragma unroll
  for (int m = 0; m < K; ++m) {
    const double pb = vpbar[m], mb = vmbar[K - 1 - m];
    const double Wb = s.alpha * (pb - mb), Gb = pb + mb;
#pragma unroll
    for (int r = 0; r < NF; ++r) {
      SX[r] = fma(Wb, sX[r * P + t + m], SX[r]);
      SF[r] = fma(Gb, sF[r * P + t + m], SF[r]);
    }
    wave_lds_order();
    if (a.live) {
#pragma unroll
      for (int r = 0; r < NF; ++r) {
        if (full || r == 0 || r == Q) {
          a.x[r * AP + a.lane + m] += Wb * g[r];
          a.f[r * AP + a.lane + m] += Gb * g[r];
        }
      }
      if (m == s.mstar) a.lam[a.lane + m] += alphabar;
    }
  }
  double dummy[NF];
  project_row_vjp<NF, Q>(s, SX, 1.0, dummy, b);
  project_row_vjp<NF, Q>(s, SF, 1.0, dummy, b);
}

// Tiled Euler adjoint along one axis, one characteristic field per
// wavefront.  A workgroup of (FW faces) x (NF fields) threads owns the cells
// [c0, c1) of one line (c1 - c0 <= FW + 1 - K).
//  1. stage the positions its faces read: state, physical flux, signal
//     speed, and the cotangent of dU/dt (0 beyond a transmissive end);
//  2. thread (f, q) recomputes field q of face f with the decision codes of
//     its two reconstructions; the field values go to LDS;
//  3. each thread back-projects the face cotangent, reverses its field from
//     the codes and adds the stencil contributions (row q of L transposed)
//     to accumulators of its own wavefront (field q; in step m lane l adds
//     to slot l + m, so the lanes of a step meet nowhere); the fields'
//     cotangents of the eigenvector constants are summed in LDS, one field
//     after the other;
//  4. field 0's wavefront reverses the Roe average once per face, into one
//     slot per face for its left cell and one for its right cell, while
//  5a. field 1's wavefront takes one owned cell per lane: it sums the cell's
//     slots over fields (and, at an end of a transmissive line, the clamped
//     positions beyond it) and applies the cell's flux Jacobian and
//     signal-speed derivative once;
//  5b. it adds the Roe average's slots of the cell and writes out.
// The order of every sum is fixed.  Blocks on one XCD (blockIdx mod 8) take
// consecutive lines, so the lines of a strided axis that share cache lines
// meet in one L2.
struct VjpTiles {
  long nlines;  // lines along the axis
  int own;      // cells per tile (FW - K + 1)
};

template <int NF, int K>
struct VjpTileShape {
  static constexpr int FW = 64;               // faces per tile (one wavefront per field)
  static constexpr int P = FW + 2 * (K - 1);  // positions staged by a full tile
  static constexpr int AP = 64 + K - 1;       // accumulator slots per wavefront
  static constexpr int NH = FW / 64;          // wavefronts per field
  static constexpr int NB = NF + 4;           // cotangents of the eigenvector constants
};

template <int NF>
__device__ __forceinline__ void bars_to_array(const FaceBars<NF>& b, double* o) {
#pragma unroll
  for (int d = 0; d < NF - 2; ++d) o[d] = b.ut[d];
  o[NF - 2] = b.b1;
  o[NF - 1] = b.b2;
  o[NF] = b.cinv;
  o[NF + 1] = b.ct;
  o[NF + 2] = b.Ht;
  o[NF + 3] = b.q2;
}

template <int NF>
__device__ __forceinline__ void array_to_bars(const double* o, FaceBars<NF>& b) {
#pragma unroll
  for (int d = 0; d < NF - 2; ++d) b.ut[d] = o[d];
  b.b1 = o[NF - 2];
  b.b2 = o[NF - 1];
  b.cinv = o[NF];
  b.ct = o[NF + 1];
  b.Ht = o[NF + 2];
  b.q2 = o[NF + 3];
}

// Output rule of one adjoint launch, per cell and field of the axis:
//   out = c src + scale (J^T Lbar)      (src = 0 when NULL)
// src may be out itself (accumulation) or another array of out's layout (a
// linear combination of the step adjoint joining the launch); it is read
// before out is written.
struct VjpOut {
  double* out;
  const double* src;
  double c, scale;
};

// Occupancy the tile kernel is compiled for: 3 wavefronts per SIMD (at most
// 168 VGPRs; three 4-wavefront blocks of 46 KB LDS per CU), measured 20%
// faster than 2 without spills; the 5-field tile (65 KB LDS, two blocks per
// CU) cannot reach 3 and keeps 256 VGPRs.
template <int NF>
struct VjpOccupancy {
  static constexpr int WAVES = NF >= 5 ? 2 : 3;
};

template <int NF, int K, int LIM, bool ADAPT>
__global__ __launch_bounds__(64 * NF) __attribute__((amdgpu_waves_per_eu(VjpOccupancy<NF>::WAVES))) void k_vjp_tile(const double* __restrict__ U,
                                                       const double* __restrict__ Lbar, VjpOut vo,
                                                       VjpAxis ax, VjpTiles tl, int fld0, int fld1, int fld2,
                                                       int fld3, int fld4, FaceParams fp) {
  using S = VjpTileShape<NF, K>;
  constexpr int FW = S::FW, P = S::P, AP = S::AP, NB = S::NB, NH = S::NH, H = K / 2;
  __shared__ double sX[NF * P], sF[NF * P], sLam[P], sLb[NF * P], fcs[NF * FW], bS[NF * NB * FW];
  __shared__ double aX[NF * NH][NF * AP], aF[NF * NH][NF * AP], aL[NF * NH][AP];
  __shared__ double rXa[NF * AP], rXb[NF * AP];  // the Roe average's cotangents of its left and right cells
  static_assert(NH == 1, "one wavefront per field: the slot of a face's cell is its lane + offset");
  long g = blockIdx.x;
  const long B = gridDim.x;
  if ((B & 7) == 0) g = (g & 7) * (B >> 3) + (g >> 3);
  const long line = g % tl.nlines;
  const int tile = (int)(g / tl.nlines);
  Line L;
  if (ax.axis == 0) {
    L = Line{line * ax.nx, 1, ax.n, ax.bc};
  } else if (ax.axis == 1) {
    const long x = line % ax.nx, z = line / ax.nx;
    L = Line{x + (long)ax.nx * ax.ny * z, ax.nx, ax.n, ax.bc};
  } else {
    L = Line{line, (long)ax.nx * ax.ny, ax.n, ax.bc};
  }
  const int fall[5] = {fld0, fld1, fld2, fld3, fld4};
  int fld[NF];
#pragma unroll
  for (int q = 0; q < NF; ++q) fld[q] = fall[q];
  const long N = (long)ax.nx * ax.ny * ax.nz;
  const bool per = (ax.bc == 0);
  const int n = ax.n;
  const int c0 = tile * tl.own;
  const int ncell = min(n, c0 + tl.own) - c0;
  const int nface = ncell + K - 1;
  const int npos = nface + K - 1;
  const int pp0 = c0 - K + 1;  // position of slot 0
  const int f = threadIdx.x, q = threadIdx.y;
  const int tid = q * FW + f;
  const int half = f >> 6, lane = f & 63;

  // field 1's thread f finishes owned cell c0 + f (step 5)
  const bool cell_thread = (q == 1 && f < ncell);
  __builtin_amdgcn_s_setprio(3);  // high while loads and stores issue (entry, staging, the write)

  // 1. staging; accumulators and the constants' cotangents cleared
  for (int i = tid; i < npos; i += FW * NF) {
    const int pos = pp0 + i;
    const long cell = cell_at(L, pos);
    const bool inside = per || (pos >= 0 && pos < n);
    double X[NF], F[NF], lam;
#pragma unroll
    for (int r = 0; r < NF; ++r) X[r] = U[fld[r] * N + cell];
    cell_physics<NF>(X, fp.gamma, F, lam);
#pragma unroll
    for (int r = 0; r < NF; ++r) {
      sX[r * P + i] = X[r];
      sF[r * P + i] = F[r];
      sLb[r * P + i] = inside ? Lbar[fld[r] * N + cell] : 0.0;
    }
    sLam[i] = lam;
  }
  for (int i = tid; i < NF * NH * AP; i += FW * NF) {
    const int w = i / AP, e = i - w * AP;
#pragma unroll
    for (int r = 0; r < NF; ++r) aX[w][r * AP + e] = aF[w][r * AP + e] = 0.0;
    aL[w][e] = 0.0;
  }
  for (int i = tid; i < NF * AP; i += FW * NF) rXa[i] = rXb[i] = 0.0;
  __syncthreads();

  __builtin_amdgcn_s_setprio(0);
  // 2. forward of field q at face f, with its decision codes
  const int j = c0 - H + 1 + f;  // face of this thread: between positions j-1 and j
  const bool live = f < nface && (per || (j >= 0 && j <= n));
  const bool wave_live = __ballot(live) != 0;
  const int t = f < nface ? f : nface - 1;  // staged slots for every lane
  FaceState<NF> s;
  double W[K];
  uint32_t cp = 0u, cm = 0u;
  if (wave_live) {
    s.alpha = 0.0;
    s.mstar = 0;
#pragma unroll
    for (int m = 0; m < K; ++m) {
      const double lam = sLam[t + m];
      if (!(s.alpha >= lam)) {  // alpha = fmax(alpha, lam): the first maximum
        s.alpha = lam;
        s.mstar = m;
      }
    }
    double Xa[NF], Xb[NF];
#pragma unroll
    for (int r = 0; r < NF; ++r) {
      Xa[r] = sX[r * P + t + H - 1];
      Xb[r] = sX[r * P + t + H];
    }
    roe_state<NF>(Xa, Xb, fp.gamma, s);
    double fc = 0.0;
    switch (q) {
      case 0: fc = field_fwd<NF, K, LIM, ADAPT, 0, P>(sX, sF, t, s, fp.tp, W, cp, cm); break;
      case 1: fc = field_fwd<NF, K, LIM, ADAPT, 1, P>(sX, sF, t, s, fp.tp, W, cp, cm); break;
      case 2:
        if constexpr (NF > 2) fc = field_fwd<NF, K, LIM, ADAPT, 2, P>(sX, sF, t, s, fp.tp, W, cp, cm);
        break;
      case 3:
        if constexpr (NF > 3) fc = field_fwd<NF, K, LIM, ADAPT, 3, P>(sX, sF, t, s, fp.tp, W, cp, cm);
        break;
      default:
        if constexpr (NF > 4) fc = field_fwd<NF, K, LIM, ADAPT, 4, P>(sX, sF, t, s, fp.tp, W, cp, cm);
        break;
    }
    fcs[q * FW + f] = fc;
  }
  __syncthreads();

  // 3. back-projection and the reverse of field q
  FaceBars<NF> b;
#pragma unroll
  for (int d = 0; d < NF - 2; ++d) b.ut[d] = 0.0;
  b.b1 = b.b2 = b.cinv = b.ct = b.Ht = b.q2 = 0.0;
  if (wave_live) {
    double fcv[NF], Fhbar[NF], fcbar[NF];
#pragma unroll
    for (int r = 0; r < NF; ++r) {
      fcv[r] = fcs[r * FW + f];
      Fhbar[r] = (sLb[r * P + t + H] - sLb[r * P + t + H - 1]) * ax.inv_dx;
    }
    backproj_vjp<NF>(s, fcv, Fhbar, fcbar, b, q == 0);
    const FieldAcc a{aX[q * NH + half], aF[q * NH + half], aL[q * NH + half], lane, live};
    switch (q) {
      case 0: field_rev<NF, K, LIM, 0, P, AP>(sX, sF, t, s, fp.tp, W, cp, cm, fcbar[0], a, b); break;
      case 1: field_rev<NF, K, LIM, 1, P, AP>(sX, sF, t, s, fp.tp, W, cp, cm, fcbar[1], a, b); break;
      case 2:
        if constexpr (NF > 2) field_rev<NF, K, LIM, 2, P, AP>(sX, sF, t, s, fp.tp, W, cp, cm, fcbar[2], a, b);
        break;
      case 3:
        if constexpr (NF > 3) field_rev<NF, K, LIM, 3, P, AP>(sX, sF, t, s, fp.tp, W, cp, cm, fcbar[3], a, b);
        break;
      default:
        if constexpr (NF > 4) field_rev<NF, K, LIM, 4, P, AP>(sX, sF, t, s, fp.tp, W, cp, cm, fcbar[4], a, b);
        break;
    }
  }
  // each field's cotangents of the constants, summed in step 4
  {
    double o[NB];
    bars_to_array<NF>(b, o);
#pragma unroll
    for (int k = 0; k < NB; ++k) bS[(q * NB + k) * FW + f] = o[k];
  }
  __syncthreads();

  // 4. the Roe average, once per face (field 0's wavefront), side by side
  // with 5a. (field 1's wavefront)
  if (q == 0 && wave_live) {
    double o[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      o[k] = bS[k * FW + f];
#pragma unroll
      for (int r = 1; r < NF; ++r) o[k] += bS[(r * NB + k) * FW + f];
    }
    FaceBars<NF> bt;
    array_to_bars<NF>(o, bt);
    double Xa[NF], Xb[NF], xa[NF], xb[NF];
#pragma unroll
    for (int r = 0; r < NF; ++r) {
      Xa[r] = sX[r * P + t + H - 1];
      Xb[r] = sX[r * P + t + H];
      xa[r] = xb[r] = 0.0;
    }
    FaceState<NF> sr;  // the Roe inputs again (cheaper than keeping them live)
    roe_state<NF>(Xa, Xb, fp.gamma, sr);
    shared_vjp<NF>(Xa, Xb, sr, fp.gamma, bt, xa, xb);
    // the left cell of face f sits at slot f + H - 1, the right one at f + H:
    // one lane per slot in each array
    if (live) {
#pragma unroll
      for (int r = 0; r < NF; ++r) {
        rXa[r * AP + lane + H - 1] = xa[r];
        rXb[r * AP + lane + H] = xb[r];
      }
    }
  }

  // 5a. per owned cell: the stencil slots of every field, then the flux
  // Jacobian and the signal speed's derivative
  const int i = K - 1 + f;  // slot of cell c0 + f
  const int c = c0 + f;
  const int lo = (!per && c == 0) ? i - H : i;
  const int hi = (!per && c == n - 1) ? i + H : i;
  double xs[NF];
  // the cell's src values of the output rule, loaded before the slot sums so
  // that their latency hides behind them (loaded at the kernel's entry they
  // held registers through the face and pushed values into scratch)
  double prev[NF];
#pragma unroll
  for (int r = 0; r < NF; ++r) prev[r] = 0.0;
  if (vo.src && cell_thread) {
    const long cell = L.base + (long)(c0 + f) * L.stride;
#pragma unroll
    for (int r = 0; r < NF; ++r) prev[r] = vo.src[(long)fld[r] * N + cell];
  }
  if (cell_thread) {
    double fs[NF], ls = 0.0, X[NF];
#pragma unroll
    for (int r = 0; r < NF; ++r) {
      xs[r] = fs[r] = 0.0;
      X[r] = sX[r * P + i];
    }
    for (int k = lo; k <= hi; ++k) {
#pragma unroll
      for (int w = 0; w < NF; ++w) {
#pragma unroll
        for (int r = 0; r < NF; ++r) {
          xs[r] += aX[w][r * AP + k];
          fs[r] += aF[w][r * AP + k];
        }
        ls += aL[w][k];
      }
    }
    cell_physics_vjp<NF>(X, fp.gamma, fs, ls, xs);
  }
  __syncthreads();

  // 5b. the Roe average's part, and the write
  __builtin_amdgcn_s_setprio(3);
  if (cell_thread) {
    for (int k = lo; k <= hi; ++k) {
#pragma unroll
      for (int r = 0; r < NF; ++r) xs[r] += rXa[r * AP + k] + rXb[r * AP + k];
    }
    const long cell = L.base + (long)c * L.stride;
#pragma unroll
    for (int r = 0; r < NF; ++r) vo.out[(long)fld[r] * N + cell] = vo.c * prev[r] + vo.scale * xs[r];
  }
}

// out[f][cell] by the output rule, with s the sum of the contributions of
// every (face, slot) whose stencil cell is `cell`, faces in increasing order.
template <int NF, int K>
__global__ __launch_bounds__(256) void k_gather_vjp(const double* __restrict__ contrib, VjpOut vo, VjpAxis ax) {
  const long N = (long)ax.nx * ax.ny * ax.nz;
  const long cell = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= N) return;
  const int x = (int)(cell % ax.nx);
  const int y = (int)((cell / ax.nx) % ax.ny);
  const int z = (int)(cell / ((long)ax.nx * ax.ny));
  const int c = ax.axis == 0 ? x : (ax.axis == 1 ? y : z);
  // face index of line position j
  auto face = [&](int jj) -> long {
    if (ax.axis == 0) return jj + (long)ax.nfa * (y + (long)ax.ny * z);
    if (ax.axis == 1) return x + (long)ax.nx * (jj + (long)ax.nfa * z);
    return x + (long)ax.nx * (y + (long)ax.ny * jj);
  };
  double s[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) s[f] = 0.0;
  const int n = ax.n;
  if (ax.bc == 0) {
    // periodic: face (c + K/2 - m) mod n holds cell c at slot m
#pragma unroll
    for (int m = K - 1; m >= 0; --m) {
      int jj = c + K / 2 - m;
      jj = jj >= n ? jj - n : (jj < 0 ? jj + n : jj);
      const long tf = face(jj);
#pragma unroll
      for (int f = 0; f < NF; ++f) s[f] += contrib[((long)m * NF + f) * ax.nfaces + tf];
    }
  } else if (c > 0 && c < n - 1) {
#pragma unroll
    for (int m = K - 1; m >= 0; --m) {
      const int jj = c + K / 2 - m;
      if (jj < 0 || jj > n) continue;
      const long tf = face(jj);
#pragma unroll
      for (int f = 0; f < NF; ++f) s[f] += contrib[((long)m * NF + f) * ax.nfaces + tf];
    }
  } else {
    // an end cell also receives every slot clamped onto it
    for (int jj = (c == 0 ? 0 : n - K / 2); jj <= (c == 0 ? K / 2 : n); ++jj) {
      const long tf = face(jj);
      for (int m = 0; m < K; ++m) {
        const int raw = jj - K / 2 + m;
        const bool hit = (c == 0) ? (raw <= 0) : (raw >= n - 1);
        if (!hit) continue;
#pragma unroll
        for (int f = 0; f < NF; ++f) s[f] += contrib[((long)m * NF + f) * ax.nfaces + tf];
      }
    }
  }
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    const long o = (long)f * N + cell;
    vo.out[o] = (vo.src ? vo.c * vo.src[o] : 0.0) + vo.scale * s[f];
  }
}

struct VjpLaunch {
  const double* U;
  const double* Lbar;
  double* contrib;
  VjpOut out;
  VjpAxis ax;
  int fld[5];
  FaceParams fp;
  hipStream_t stream;
};

template <int NF, int K, int LIM, bool ADAPT>
hipError_t launch_vjp(const VjpLaunch& a) {
  if constexpr (NF == 1) {
    const unsigned fb = (unsigned)((a.ax.nfaces + 255) / 256);
    hipLaunchKernelGGL((k_faces_vjp_scalar<K, LIM, ADAPT>), dim3(fb), dim3(256), 0, a.stream, a.U, a.Lbar,
                       a.contrib, a.ax, a.fp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long N = (long)a.ax.nx * a.ax.ny * a.ax.nz;
    const unsigned cb = (unsigned)((N + 255) / 256);
    hipLaunchKernelGGL((k_gather_vjp<NF, K>), dim3(cb), dim3(256), 0, a.stream, a.contrib, a.out, a.ax);
  } else {
    const long N = (long)a.ax.nx * a.ax.ny * a.ax.nz;
    VjpTiles tl;
    tl.nlines = N / a.ax.n;
    tl.own = VjpTileShape<NF, K>::FW - K + 1;
    const long ntile = (a.ax.n + tl.own - 1) / tl.own;
    hipLaunchKernelGGL((k_vjp_tile<NF, K, LIM, ADAPT>), dim3((unsigned)(tl.nlines * ntile)),
                       dim3(VjpTileShape<NF, K>::FW, NF), 0,
                       a.stream, a.U, a.Lbar, a.out, a.ax, tl, a.fld[0], a.fld[1], a.fld[2], a.fld[3], a.fld[4],
                       a.fp);
  }
  return hipGetLastError();
}

}  // namespace tenom
