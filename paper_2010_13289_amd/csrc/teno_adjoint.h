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
//  k_faces_vjp_euler  one wavefront per (64 faces, characteristic field) of
//                one axis: recompute the face and push the face cotangent
//                (from the cotangent of dU/dt) back to the K x NF stencil
//                inputs, written per face and slot (k_faces_vjp_scalar: one
//                thread per face of the scalar system).
//  k_gather_vjp  one thread per cell: sum the contributions of the faces
//                whose stencils hold the cell, in a fixed order (no atomics).
#pragma once

#include "teno_kernels.h"

namespace tenom {

// ---------------------------------------------------------------------------
// reverse of the branch-free helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ void minmod2_vjp(double x, double y, double obar, double& xbar, double& ybar) {
  const double lo = fmin(x, y), hi = fmax(x, y);
  if (lo > 0.0) {
    if (x <= y) xbar += obar; else ybar += obar;
  } else if (hi < 0.0) {
    if (x >= y) xbar += obar; else ybar += obar;
  }
}

__device__ __forceinline__ void minmod4_vjp(const double (&a)[4], double obar, double (&abar)[4]) {
  const double lo = fmin(fmin(a[0], a[1]), fmin(a[2], a[3]));
  const double hi = fmax(fmax(a[0], a[1]), fmax(a[2], a[3]));
  if (lo > 0.0) {
    const int i01 = a[0] <= a[1] ? 0 : 1, i23 = a[2] <= a[3] ? 2 : 3;
    const int i = a[i01] <= a[i23] ? i01 : i23;
    abar[i] += obar;
  } else if (hi < 0.0) {
    const int i01 = a[0] >= a[1] ? 0 : 1, i23 = a[2] >= a[3] ? 2 : 3;
    const int i = a[i01] >= a[i23] ? i01 : i23;
    abar[i] += obar;
  }
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
    if (A1 >= A2) {
      if (m1 <= s.md) dpbar += lobar * zmin_d(dp); else mdbar += lobar;
    } else {
      if (m2 <= s.lc) ulbar += lobar * zmin_d(s.ul); else lcbar += lobar;
    }
  }
  // hi = fmin(B1, B2), B1 = fmax(fmax(0, dp), md), B2 = fmax(fmax(0, ul), lc)
  {
    const double n1 = fmax(0.0, dp), B1 = fmax(n1, s.md);
    const double n2 = fmax(0.0, s.ul), B2 = fmax(n2, s.lc);
    if (B1 <= B2) {
      if (n1 >= s.md) dpbar += hibar * zmax_d(dp); else mdbar += hibar;
    } else {
      if (n2 >= s.lc) ulbar += hibar * zmax_d(s.ul); else lcbar += hibar;
    }
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
      const double w = T::d(k) * rbar;
      cbar[k] = 0.0;
      if (smooth[k]) {
        cbar[k] = w;
      } else {
        // lim = fmin(fmax(c, lo), hi)
        if (fmax(c[k], ms.lo) <= ms.hi) {
          if (c[k] >= ms.lo) cbar[k] = w; else lobar += w;
        } else {
          hibar += w;
        }
      }
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
      if (dm > 0.0) {
        // up = fmax(0, u1), u1 = fmin(u0, B), u0 = fmin(2 dm, 2 dp)
        const double u0 = fmin(2.0 * dm, 2.0 * dp), u1 = fmin(u0, B);
        if (!(0.0 >= u1)) {
          if (u0 <= B) {
            if (2.0 * dm <= 2.0 * dp) dmbar += 2.0 * sbar; else dpbar += 2.0 * sbar;
          } else {
            Bbar += sbar;
          }
        }
      } else if (dm < 0.0) {
        // dn = fmin(0, w1), w1 = fmax(w0, B), w0 = fmax(2 dm, 2 dp)
        const double w0 = fmax(2.0 * dm, 2.0 * dp), w1 = fmax(w0, B);
        if (!(0.0 <= w1)) {
          if (w0 >= B) {
            if (2.0 * dm >= 2.0 * dp) dmbar += 2.0 * sbar; else dpbar += 2.0 * sbar;
          } else {
            Bbar += sbar;
          }
        }
      }
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

template <int NF, int K>
__device__ __forceinline__ void face_state(const double (&X)[K][NF], double gamma, FaceState<NF>& s) {
  constexpr int ND = NF - 2;
  constexpr int H = K / 2;
  const double gm1 = gamma - 1.0;
  s.alpha = 0.0;
  s.mstar = 0;
#pragma unroll
  for (int m = 0; m < K; ++m) {
    double Fm[NF], lam;
    cell_physics<NF>(X[m], gamma, Fm, lam);
    if (!(s.alpha >= lam)) {  // alpha = fmax(alpha, lam): the first maximum
      s.alpha = lam;
      s.mstar = m;
    }
  }
  roe_input<NF>(X[H - 1], gamma, s.ra);
  roe_input<NF>(X[H], gamma, s.rb);
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

// Component Q of the left-eigenvector projection (the expressions of the
// forward face, so the values are the same bits).
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

// Adjoint of project_row: ob -> Yb and the shared cotangents.
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

// Per-field intermediates the forward pass keeps for the adjoint.
template <int K>
struct FieldKeep {
  double vp[K], vm[K];  // doubled split values (vm mirrored)
  double W[K], G[K];    // row Q of the projections of U and F
  uint32_t mp, mm;      // smoothness decisions of the two reconstructions
};

// Field Q of the forward face: fc_Q = (TENO(g+) + TENO(g-)) / 2 (doubled split).
template <int NF, int K, int LIM, bool ADAPT, int Q>
__device__ __forceinline__ double field_forward(const double (&X)[K][NF], const FaceState<NF>& s, double gamma,
                                                const TenoParams& tp, FieldKeep<K>& f) {
#pragma unroll
  for (int m = 0; m < K; ++m) {
    double Fm[NF], lam;
    cell_physics<NF>(X[m], gamma, Fm, lam);
    f.W[m] = project_row<NF, Q>(s, X[m]);
    f.G[m] = project_row<NF, Q>(s, Fm);
    lf_split2(f.G[m], s.alpha, f.W[m], f.vp[m], f.vm[K - 1 - m]);
  }
  f.mp = f.mm = 0u;
  return 0.5 * (teno_m<K, LIM, true, ADAPT>(f.vp, tp, f.mp) + teno_m<K, LIM, true, ADAPT>(f.vm, tp, f.mm));
}

// Adjoint of field Q: fcbar_Q -> Xbar (through the reconstructions, the
// split, row Q of both projections, the cell fluxes and alpha) and the
// shared cotangents.
template <int NF, int K, int LIM, int Q>
__device__ __forceinline__ void field_vjp(const double (&X)[K][NF], const FaceState<NF>& s, double gamma,
                                          const TenoParams& tp, double fcbar, FieldKeep<K>& f,
                                          double (&Xbar)[K][NF], FaceBars<NF>& b) {
  double vpbar[K], vmbar[K];
#pragma unroll
  for (int m = 0; m < K; ++m) vpbar[m] = vmbar[m] = 0.0;
  teno_m_vjp_given<K, LIM>(f.vp, tp, f.mp, 0.5 * fcbar, vpbar);
  teno_m_vjp_given<K, LIM>(f.vm, tp, f.mm, 0.5 * fcbar, vmbar);
  double alphabar = 0.0;
#pragma unroll
  for (int m = 0; m < K; ++m) {
    // vp[m] = G + alpha W, vm[K-1-m] = G - alpha W
    const double pb = vpbar[m], mb = vmbar[K - 1 - m];
    alphabar += f.W[m] * (pb - mb);
    f.G[m] = pb + mb;
    f.W[m] = s.alpha * (pb - mb);
  }
#pragma unroll
  for (int m = 0; m < K; ++m) {
    project_row_vjp<NF, Q>(s, X[m], f.W[m], Xbar[m], b);
    double Fm[NF], lam, Fb[NF];
    cell_physics<NF>(X[m], gamma, Fm, lam);
#pragma unroll
    for (int r = 0; r < NF; ++r) Fb[r] = 0.0;
    project_row_vjp<NF, Q>(s, Fm, f.G[m], Fb, b);
    cell_physics_vjp<NF>(X[m], gamma, Fb, m == s.mstar ? alphabar : 0.0, Xbar[m]);
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

// Shared cotangents -> Xbar: eigenvector constants, Roe average, Roe inputs.
template <int NF, int K>
__device__ __forceinline__ void shared_vjp(const double (&X)[K][NF], const FaceState<NF>& s, double gamma,
                                           FaceBars<NF> b, double (&Xbar)[K][NF]) {
  constexpr int ND = NF - 2;
  constexpr int H = K / 2;
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
  roe_input_vjp<NF>(X[H - 1], gamma, rsabar, uabar, b.Ht * s.ra.rs * s.w, Xbar[H - 1]);
  roe_input_vjp<NF>(X[H], gamma, rsbbar, ubbar, b.Ht * s.rb.rs * s.w, Xbar[H]);
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

// Euler system: a workgroup of NF wavefronts handles 64 faces, wavefront q
// (threadIdx.y, uniform in the wave) the characteristic field q.  Every wave
// recomputes the shared face state; the forward field results are exchanged
// through LDS for the back-projection; each wave pushes its cotangents back
// to the stencil (the shared ones included: the map is linear in them) and
// the NF partial stencil cotangents are summed in LDS in the order q = 0,
// 1, ... .
template <int NF, int K, int LIM, bool ADAPT>
__global__ __launch_bounds__(64 * NF) void k_faces_vjp_euler(const double* __restrict__ U,
                                                             const double* __restrict__ Lbar,
                                                             double* __restrict__ contrib, VjpAxis ax, int fld0,
                                                             int fld1, int fld2, int fld3, int fld4, FaceParams fp) {
  __shared__ double fcs[NF][64];
  __shared__ double acc[K * NF][64];
  const int lane = threadIdx.x;
  const int q = threadIdx.y;
  const long t = (long)blockIdx.x * 64 + lane;
  const bool valid = t < ax.nfaces;
  const long tt = valid ? t : ax.nfaces - 1;  // every thread takes part in the barriers
  Line L;
  int j;
  vjp_face_line(ax, tt, L, j);
  const long N = (long)ax.nx * ax.ny * ax.nz;
  const int fall[5] = {fld0, fld1, fld2, fld3, fld4};
  int fld[NF];
#pragma unroll
  for (int r = 0; r < NF; ++r) fld[r] = fall[r];
  double X[K][NF], Xbar[K][NF];
#pragma unroll
  for (int m = 0; m < K; ++m) {
    const long cell = cell_at(L, j - K / 2 + m);
#pragma unroll
    for (int r = 0; r < NF; ++r) {
      X[m][r] = U[(long)fld[r] * N + cell];
      Xbar[m][r] = 0.0;
    }
  }
  FaceState<NF> s;
  face_state<NF, K>(X, fp.gamma, s);
  // forward field q (its intermediates kept for the adjoint)
  FieldKeep<K> keep;
  double fcq = 0.0;
  switch (q) {
    case 0: fcq = field_forward<NF, K, LIM, ADAPT, 0>(X, s, fp.gamma, fp.tp, keep); break;
    case 1: fcq = field_forward<NF, K, LIM, ADAPT, 1>(X, s, fp.gamma, fp.tp, keep); break;
    case 2: fcq = field_forward<NF, K, LIM, ADAPT, 2>(X, s, fp.gamma, fp.tp, keep); break;
    default:
      if constexpr (NF > 3) {
        if (q == 3) fcq = field_forward<NF, K, LIM, ADAPT, 3>(X, s, fp.gamma, fp.tp, keep);
      }
      if constexpr (NF > 4) {
        if (q == 4) fcq = field_forward<NF, K, LIM, ADAPT, 4>(X, s, fp.gamma, fp.tp, keep);
      }
      break;
  }
  fcs[q][lane] = fcq;
  __syncthreads();
  double fc[NF], Fhbar[NF], fcbar[NF];
#pragma unroll
  for (int r = 0; r < NF; ++r) fc[r] = fcs[r][lane];
  face_cotangent<NF>(ax, L, j, N, fld, Lbar, Fhbar);
  FaceBars<NF> b;
#pragma unroll
  for (int d = 0; d < NF - 2; ++d) b.ut[d] = 0.0;
  b.b1 = b.b2 = b.cinv = b.ct = b.Ht = b.q2 = 0.0;
  backproj_vjp<NF>(s, fc, Fhbar, fcbar, b, q == 0);
  switch (q) {
    case 0: field_vjp<NF, K, LIM, 0>(X, s, fp.gamma, fp.tp, fcbar[0], keep, Xbar, b); break;
    case 1: field_vjp<NF, K, LIM, 1>(X, s, fp.gamma, fp.tp, fcbar[1], keep, Xbar, b); break;
    case 2: field_vjp<NF, K, LIM, 2>(X, s, fp.gamma, fp.tp, fcbar[2], keep, Xbar, b); break;
    default:
      if constexpr (NF > 3) {
        if (q == 3) field_vjp<NF, K, LIM, 3>(X, s, fp.gamma, fp.tp, fcbar[3], keep, Xbar, b);
      }
      if constexpr (NF > 4) {
        if (q == 4) field_vjp<NF, K, LIM, 4>(X, s, fp.gamma, fp.tp, fcbar[4], keep, Xbar, b);
      }
      break;
  }
  shared_vjp<NF, K>(X, s, fp.gamma, b, Xbar);
  // sum the partial stencil cotangents over the fields, q = 0, 1, ...
#pragma unroll 1
  for (int r = 0; r < NF; ++r) {
    if (q == r) {
#pragma unroll
      for (int m = 0; m < K; ++m)
#pragma unroll
        for (int c = 0; c < NF; ++c) acc[m * NF + c][lane] = (r == 0 ? 0.0 : acc[m * NF + c][lane]) + Xbar[m][c];
    }
    __syncthreads();
  }
  if (valid) {
    for (int e = q; e < K * NF; e += NF) {
      const int m = e / NF, c = e - m * NF;
      contrib[((long)m * NF + fall[c]) * ax.nfaces + t] = acc[e][lane];
    }
  }
}

// out[f][cell] = (acc ? out : 0) + scale * sum of the contributions of every
// (face, slot) whose stencil cell is `cell`, faces in increasing order.
template <int NF, int K>
__global__ __launch_bounds__(256) void k_gather_vjp(const double* __restrict__ contrib, double* __restrict__ out,
                                                    VjpAxis ax, double scale, int acc) {
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
    out[o] = (acc ? out[o] : 0.0) + scale * s[f];
  }
}

struct VjpLaunch {
  const double* U;
  const double* Lbar;
  double* contrib;
  double* out;
  double scale;
  int acc;
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
  } else {
    const unsigned fb = (unsigned)((a.ax.nfaces + 63) / 64);
    hipLaunchKernelGGL((k_faces_vjp_euler<NF, K, LIM, ADAPT>), dim3(fb), dim3(64, NF), 0, a.stream, a.U, a.Lbar,
                       a.contrib, a.ax, a.fld[0], a.fld[1], a.fld[2], a.fld[3], a.fld[4], a.fp);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long N = (long)a.ax.nx * a.ax.ny * a.ax.nz;
  const unsigned cb = (unsigned)((N + 255) / 256);
  hipLaunchKernelGGL((k_gather_vjp<NF, K>), dim3(cb), dim3(256), 0, a.stream, a.contrib, a.out, a.ax, a.scale, a.acc);
  return hipGetLastError();
}

}  // namespace tenom
