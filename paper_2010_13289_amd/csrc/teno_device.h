// Device code of the TENO-M face reconstruction for gfx950 (FP64 throughout).
//
// One thread computes the complete numerical flux of one face: K cell
// states along the sweep axis -> (Euler) Roe-average characteristic
// projection and Rusanov splitting -> two mirrored TENO-M reconstructions
// per characteristic field -> back-projection.  Everything stays in
// registers; there is no matrix-shaped work worth MFMA (each face has its
// own 5x5 eigenvector basis, and FP64 MFMA is no faster than FP64 VALU).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "teno_tables.h"

namespace tenom {

// Eq. measureTENO: gamma_k = (C + tau_K / (beta_k + eps))^q, C = 1, q = 6.
// The reconstruction runs on twice the split fluxes (see lf_split2), which
// scales beta and tau by 4; eps is scaled by the same exact factor, so every
// rounding step is the same as on the halved values.
constexpr double kEps = 1e-40;
constexpr double kEps2x = 4.0 * kEps;

// Limiter kinds (template values).  The C ABI's limiter IDs map onto them:
// MP with d^M4 (IDs 1, 5) and with d^MM (IDs 6, 7, 8) differ only in the
// runtime beta of Eq. large_curvature.
enum : int { LIM_TENO = 0, LIM_MP = 1, LIM_TVD_MINMOD = 2, LIM_TVD5 = 3, LIM_VA = 4, LIM_MP_MM = 6 };

// Runtime parameters of one reconstruction.
struct TenoParams {
  double C_T;       // cutoff (ignored with the adaptive cutoff)
  double mp_beta3;  // beta / 3 of Eq. large_curvature (MP limiters)
};

// Sec. 2.4: Ren-type indicator (xi = 1e-3, C_r = 0.23) and the cutoff
// adaptation (alpha_1 = 10.5, alpha_2 = 3.5) of the eight-point schemes.
constexpr double kRenCr = 0.23;
constexpr double kRenEps = 0.9 * kRenCr / (1.0 - 0.9 * kRenCr) * 1e-3 * 1e-3;

// minmod of two / four arguments (Eqs. minmod222, minmod444), branch-free:
// the smallest-magnitude argument if all share a sign, else 0.
__device__ __forceinline__ double minmod2(double x, double y) {
  return fmax(fmin(x, y), 0.0) + fmin(fmax(x, y), 0.0);
}
__device__ __forceinline__ double minmod4(double a, double b, double c, double d) {
  const double lo = fmin(fmin(a, b), fmin(c, d));
  const double hi = fmax(fmax(a, b), fmax(c, d));
  return fmax(lo, 0.0) + fmin(hi, 0.0);
}

// 1/x from the hardware estimate (relative error ~5e-8) plus two
// Newton-Raphson steps: equal to IEEE 1/x for normal x.
__device__ __forceinline__ double rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// 1/x with one Newton-Raphson step (relative error ~2e-15).  Used only for
// the scale-separation measure, which reaches the output through the
// cutoff comparison alone.
__device__ __forceinline__ double rcp1(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}

// 1/b_k of the K - 2 indicator denominators b_k = beta_k + eps, in pairs
// from one reciprocal of each pair's product (1/b_0 = b_1 / (b_0 b_1)): one
// transcendental per two denominators.  Relative error a few units in the
// last place, as for rcp1; like rcp1 it only reaches the output through the
// cutoff comparison.  Every b_k >= 4e-40, so no product underflows; a product
// stays below 2^1000 (its reciprocal normal) while b_k < 2^500, i.e. for
// split fluxes below about 1e75 in magnitude.
template <int N>
__device__ __forceinline__ void rcp_pairs(const double (&b)[N], double (&inv)[N]) {
  static_assert(N % 2 == 0, "pairs of denominators");
#pragma unroll
  for (int k = 0; k < N; k += 2) {
    const double r = rcp1(b[k] * b[k + 1]);
    inv[k] = b[k + 1] * r;
    inv[k + 1] = b[k] * r;
  }
}

// ---------------------------------------------------------------------------
// Pieces of one TENO-M reconstruction at x_{i+1/2} from v[0..K-1] =
// f_{i-K/2+1..i+K/2} (Secs. 2.2-3.3), computed relative to v_i in the
// differences D[j] = v[j+1] - v[j].  The inputs are twice the split fluxes
// (lf_split2) and so is the result: every step is homogeneous, with eps
// scaled to match, so the result is exactly twice the reconstruction of the
// halved values.  The forward reconstruction (teno_m) and its adjoint share
// these functions, so both take the same decisions.
// ---------------------------------------------------------------------------

// Smoothness decisions delta_k (true = smooth): indicators, tau_K, gamma_k
// and the cutoff (Eqs. measureTENO, taukTENO, normalize, cut-off); with
// ADAPT the cutoff of Sec. 2.4 (Eqs. shock_indicator, cut-off_adjust).
template <int K, bool ADAPT>
__device__ __forceinline__ void teno_cutoff(const double (&D)[K - 1], const TenoParams& tp, bool (&smooth)[K - 2]) {
  using T = TenoTables<K>;
  constexpr int NK = K - 2;
  constexpr int C0 = K / 2 - 1;  // index of v_i
  double C_T = tp.C_T;
  if constexpr (ADAPT) {
    // eta at cells i-1 .. i+2 (eps scaled by 4 for the doubled values), the
    // minimum, m = 1 - min(1, eta / C_r)
    double eta = 0.0;
#pragma unroll
    for (int j = C0 - 1; j <= C0 + 2; ++j) {
      const double a = D[j], b = D[j - 1];
      const double num = fabs(2.0 * a * b) + 4.0 * kRenEps;
      const double den = fma(a, a, fma(b, b, 4.0 * kRenEps));
      const double e = num * rcp1(den);
      eta = (j == C0 - 1) ? e : fmin(eta, e);
    }
    const double m = 1.0 - fmin(1.0, eta * (1.0 / kRenCr));
    // g = (1-m)^4 (1+4m), beta = 10.5 - 3.5 (1 - g), C_T = 10^-floor(beta)
    // with floor(beta) in {7, 8, 9, 10}
    const double om = 1.0 - m, om2 = om * om;
    const double g = om2 * om2 * fma(4.0, m, 1.0);
    const double fl = floor(fma(-3.5, 1.0 - g, 10.5));
    // written as selects of constants: a nested conditional can become
    // branches, around which the compiler computes every reconstruction's
    // cutoff first and holds the results (about 70 more vector registers)
    C_T = (fl >= 8.0) ? 1e-8 : 1e-7;
    C_T = (fl >= 9.0) ? 1e-9 : C_T;
    C_T = (fl >= 10.0) ? 1e-10 : C_T;
  }
  double beta[NK], betaK;
  T::betas(D, beta, betaK);
  const double tau = fabs(fma(fma(4.0, beta[0], beta[1] + beta[2]), -1.0 / 6.0, betaK));
  // gamma_k and the cutoff: chi_k = gamma_k / sum < C_T  <=>  gamma_k < C_T sum
  // the tables may scale every beta by T::beta_scale; eps follows
  constexpr double eps = kEps2x * T::beta_scale;
  double b[NK], binv[NK];
#pragma unroll
  for (int k = 0; k < NK; ++k) b[k] = beta[k] + eps;
  rcp_pairs<NK>(b, binv);
  double g[NK];
  double sum = 0.0;
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    const double s = fma(tau, binv[k], 1.0);
    const double s2 = s * s;
    const double s4 = s2 * s2;
    g[k] = s4 * s2;
    sum = (k == 0) ? g[0] : fma(s4, s2, sum);  // the sum takes gamma_k unrounded
  }
  const double thr = C_T * sum;
#pragma unroll
  for (int k = 0; k < NK; ++k) smooth[k] = !(g[k] < thr);
}

// MP bounds relative to v_i (Eqs. curvature, maximal_curvature or
// maximal_curvature1, upper_limiter, median_value, large_curvature,
// value_min_max), with every intermediate the adjoint needs.
struct MpState {
  double d_im1, d_i, d_ip1;  // curvatures at i-1, i, i+1
  double aR[4], aL[4];       // minmod arguments at i+1/2 and i-1/2
  double dR, dL;             // curvature measures at i+1/2 and i-1/2
  double ul, md, lc;
  double lo, hi;             // f_min - f_i, f_max - f_i
};

template <int K, int LIM>
__device__ __forceinline__ void mp_bounds(const double (&D)[K - 1], const TenoParams& tp, MpState& s) {
  constexpr int C0 = K / 2 - 1;
  const double dm = D[C0 - 1];  // f_i - f_{i-1}
  const double dp = D[C0];      // f_{i+1} - f_i
  s.d_im1 = D[C0 - 1] - D[C0 - 2];
  s.d_i = D[C0] - D[C0 - 1];
  s.d_ip1 = D[C0 + 1] - D[C0];
  if constexpr (LIM == LIM_MP) {
    s.aR[0] = fma(4.0, s.d_i, -s.d_ip1);
    s.aR[1] = fma(4.0, s.d_ip1, -s.d_i);
    s.aR[2] = s.d_i;
    s.aR[3] = s.d_ip1;
    s.aL[0] = fma(4.0, s.d_im1, -s.d_i);
    s.aL[1] = fma(4.0, s.d_i, -s.d_im1);
    s.aL[2] = s.d_im1;
    s.aL[3] = s.d_i;
    s.dR = minmod4(s.aR[0], s.aR[1], s.aR[2], s.aR[3]);
    s.dL = minmod4(s.aL[0], s.aL[1], s.aL[2], s.aL[3]);
  } else {
    s.aR[0] = s.d_i;
    s.aR[1] = s.d_ip1;
    s.aL[0] = s.d_im1;
    s.aL[1] = s.d_i;
    s.dR = minmod2(s.d_i, s.d_ip1);
    s.dL = minmod2(s.d_im1, s.d_i);
  }
  // alpha = 1.25; 0 (= f_i) lies in both brackets, so lo <= 0 <= hi
  s.ul = 1.25 * dm;
  s.md = fma(0.5, dp, -0.5 * s.dR);
  s.lc = fma(tp.mp_beta3, s.dL, 0.5 * dm);
  s.lo = fmax(fmin(fmin(0.0, dp), s.md), fmin(fmin(0.0, s.ul), s.lc));
  s.hi = fmin(fmax(fmax(0.0, dp), s.md), fmax(fmax(0.0, s.ul), s.lc));
}

// Decision code of the MP limiter (bits relative to `shift`): which argument
// the lower and upper bounds pass their derivative to (0 none, 1 dp, 2 md,
// 3 ul, 4 lc; 3 bits each) and which argument each minmod of the curvature
// measures picks (0 none, else 1 + index; 3 bits each).  Ties go to the
// first argument, a bound of 0 passes nothing.
__device__ __forceinline__ uint32_t minmod_pick(const double* a, int na) {
  const bool pos = na == 4 ? fmin(fmin(a[0], a[1]), fmin(a[2], a[3])) > 0.0 : fmin(a[0], a[1]) > 0.0;
  const bool neg = na == 4 ? fmax(fmax(a[0], a[1]), fmax(a[2], a[3])) < 0.0 : fmax(a[0], a[1]) < 0.0;
  const bool p01 = pos ? (a[0] <= a[1]) : (a[0] >= a[1]);
  uint32_t i = p01 ? 0u : 1u;
  if (na == 4) {
    const bool p23 = pos ? (a[2] <= a[3]) : (a[2] >= a[3]);
    const double v01 = p01 ? a[0] : a[1], v23 = p23 ? a[2] : a[3];
    const bool pl = pos ? (v01 <= v23) : (v01 >= v23);
    const uint32_t i23 = p23 ? 2u : 3u;
    i = pl ? i : i23;
  }
  return (pos || neg) ? i + 1u : 0u;
}

template <int K, int LIM>
__device__ __forceinline__ uint32_t mp_code(const double (&D)[K - 1], const MpState& s) {
  constexpr int C0 = K / 2 - 1;
  const double dp = D[C0];
  // one select per statement: nested conditionals can become branches
  uint32_t lo, hi;
  {
    const double m1 = fmin(0.0, dp), A1 = fmin(m1, s.md);
    const double m2 = fmin(0.0, s.ul), A2 = fmin(m2, s.lc);
    const uint32_t c1 = (0.0 <= dp) ? 0u : 1u, c2 = (0.0 <= s.ul) ? 0u : 3u;
    const uint32_t l1 = (m1 <= s.md) ? c1 : 2u, l2 = (m2 <= s.lc) ? c2 : 4u;
    lo = (A1 >= A2) ? l1 : l2;
  }
  {
    const double n1 = fmax(0.0, dp), B1 = fmax(n1, s.md);
    const double n2 = fmax(0.0, s.ul), B2 = fmax(n2, s.lc);
    const uint32_t c1 = (0.0 >= dp) ? 0u : 1u, c2 = (0.0 >= s.ul) ? 0u : 3u;
    const uint32_t h1 = (n1 >= s.md) ? c1 : 2u, h2 = (n2 >= s.lc) ? c2 : 4u;
    hi = (B1 <= B2) ? h1 : h2;
  }
  constexpr int NA = (LIM == LIM_MP) ? 4 : 2;
  const uint32_t r = minmod_pick(s.aR, NA), l = minmod_pick(s.aL, NA);
  return lo | (hi << 3) | (r << 6) | (l << 9);
}

// TVD5 flux on the five cells centred at i, relative to v_i (Eqs. high order
// TVD, TVDhighorder2, TVDbeta multiplied through by delta^-: division-free,
// equal wherever the slope ratios exist).
template <int K>
__device__ __forceinline__ double tvd5_b(const double (&D)[K - 1]) {
  constexpr int C0 = K / 2 - 1;
  return fma(-3.0, D[C0 + 1], fma(24.0, D[C0], fma(11.0, D[C0 - 1], -2.0 * D[C0 - 2]))) * (1.0 / 30.0);
}

// Van Albada with kappa = 1/3 (Eqs. van_Albada_limiter, slop_ratio, vAflux):
// phi = 2 r/(r^2 + 1) = 2 d+ d- / (d+^2 + d-^2), 0 when both vanish.
// Branch-free: the denominator is raised to the smallest normal, which
// changes nothing unless |d+|, |d-| < 1e-154, and gives 0 * finite = 0 when
// both differences vanish.
constexpr double kVaDenMin = 2.2250738585072014e-308;

__device__ __forceinline__ double va_den(double dm, double dp) { return fmax(fma(dp, dp, dm * dm), kVaDenMin); }

// One TENO-M reconstruction (Secs. 2.2-3.3).  With SKIP, a wavefront in
// which every candidate of every lane is smooth skips the limiter, which only
// reaches nonsmooth candidates: the assembly then adds the same terms in the
// same order, so the result has the same bits.  When FLAGS, `bits` receives
// delta_k (1 = smooth) in bit k and, above bit 7, the limiter's decisions
// (what the adjoint with frozen branches needs): MP limiters, per candidate
// k the median's choice in bits 8 + 2k (0 the candidate, 1 the lower bound,
// 2 the upper) and mp_code in bits 20..31; TVD minmod, the minmod's pick in
// bits 8..9 (0 none, 1 d-, 2 d+); TVD5, bits 8..9 (0 none, 1 2d-, 2 2d+,
// 3 the fifth-order slope).
template <int K, int LIM, bool FLAGS, bool ADAPT, bool SKIP = false>
__device__ __forceinline__ double teno_m(const double (&v)[K], const TenoParams& tp, uint32_t& bits) {
  using T = TenoTables<K>;
  constexpr int NK = K - 2;
  constexpr int C0 = K / 2 - 1;  // index of v_i

  double D[K - 1];
#pragma unroll
  for (int j = 0; j < K - 1; ++j) D[j] = v[j + 1] - v[j];

  // candidate fluxes (Table 1), minus v_i
  double c[NK];
  T::candidates(D, c);
  bool smooth[NK];
  teno_cutoff<K, ADAPT>(D, tp, smooth);

  if constexpr (SKIP && LIM != LIM_TENO) {
    bool rough = false;
#pragma unroll
    for (int k = 0; k < NK; ++k) rough |= !smooth[k];
    if (__builtin_amdgcn_ballot_w64(rough) == 0) {  // uniform across the wavefront
      // codes: every candidate smooth, no limiter decision (none reaches
      // the result, and the adjoint's reverse reads none)
      if constexpr (FLAGS) bits |= (1u << NK) - 1u;
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < NK; ++k) acc = fma(T::d(k), c[k], acc);
      return v[C0] + acc;
    }
  }

  // limiter on the nonsmooth candidates (Eq. mp_flux), relative to v_i
  const double dm = D[C0 - 1];  // f_i - f_{i-1}
  const double dp = D[C0];      // f_{i+1} - f_i
  double lo = 0.0, hi = 0.0, ftvd = 0.0;
  if constexpr (LIM == LIM_MP || LIM == LIM_MP_MM) {
    MpState ms;
    mp_bounds<K, LIM>(D, tp, ms);
    lo = ms.lo;
    hi = ms.hi;
    if constexpr (FLAGS) {
      bits |= mp_code<K, LIM>(D, ms) << 20;
#pragma unroll
      for (int k = 0; k < NK; ++k) {
        const uint32_t in_lo = (c[k] >= lo) ? 0u : 1u;
        const uint32_t clip = (fmax(c[k], lo) <= hi) ? in_lo : 2u;
        const uint32_t sel = smooth[k] ? 0u : clip;
        bits |= sel << (8 + 2 * k);
      }
    }
  } else if constexpr (LIM == LIM_TVD_MINMOD) {
    ftvd = 0.5 * minmod2(dm, dp);
    if constexpr (FLAGS) {
      const double a[2] = {dm, dp};
      bits |= minmod_pick(a, 2) << 8;
    }
  } else if constexpr (LIM == LIM_TVD5) {
    const double B = tvd5_b<K>(D);
    const double up = fmax(0.0, fmin(fmin(2.0 * dm, 2.0 * dp), B));
    const double dn = fmin(0.0, fmax(fmax(2.0 * dm, 2.0 * dp), B));
    const double dn0 = (dm < 0.0) ? dn : 0.0;
    ftvd = 0.5 * ((dm > 0.0) ? up : dn0);
    if constexpr (FLAGS) {
      // the same choices as the fmin/fmax chains, first argument on a tie
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
      const uint32_t pm = pick_m ? 1u : 2u;
      const uint32_t pf = first ? pm : 3u;
      bits |= (live ? pf : 0u) << 8;
    }
  } else if constexpr (LIM == LIM_VA) {
    const double phi = 2.0 * dp * dm * rcp(va_den(dm, dp));
    const double kp = phi * (1.0 / 3.0);
    ftvd = 0.25 * phi * fma(1.0 - kp, dm, (1.0 + kp) * dp);
  }

  if constexpr (LIM == LIM_TENO) {
    // classic TENO: nonsmooth candidates dropped, weights renormalised
    // (Eq. weight_renormalize); at least one candidate is smooth for C_T <= 1/(K-2)
    double num = 0.0, den = 0.0;
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      num = smooth[k] ? fma(T::d(k), c[k], num) : num;
      den = smooth[k] ? den + T::d(k) : den;
      if constexpr (FLAGS) bits |= (smooth[k] ? 1u : 0u) << k;
    }
    return fma(num, rcp(den), v[C0]);
  } else {
    // assembly with the optimal weights, no renormalisation (Eq. reconstuction)
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      double lim;
      if constexpr (LIM == LIM_MP || LIM == LIM_MP_MM) {
        lim = fmin(fmax(c[k], lo), hi);  // median(f_k, f_min, f_max), lo <= hi
      } else {
        lim = ftvd;
      }
      acc = fma(T::d(k), smooth[k] ? c[k] : lim, acc);
      if constexpr (FLAGS) bits |= (smooth[k] ? 1u : 0u) << k;
    }
    return v[C0] + acc;
  }
}

// ---------------------------------------------------------------------------
// Addressing of the K stencil cells of face j along one axis.
// ---------------------------------------------------------------------------
struct Line {
  long base;    // linear index of the line's cell 0
  long stride;  // index step along the axis
  int n;        // cells along the axis
  int bc;       // 0 periodic, 1 transmissive
};

// cell index of axis position jj (|jj| < 2n for periodic) under the rule
__device__ __forceinline__ long cell_at(const Line& L, int jj) {
  int q;
  if (L.bc == 0) {
    q = jj < 0 ? jj + L.n : (jj >= L.n ? jj - L.n : jj);
  } else {
    q = jj < 0 ? 0 : (jj >= L.n ? L.n - 1 : jj);
  }
  return L.base + (long)q * L.stride;
}

// Rusanov split f+- = (f +- alpha u)/2 of one value, returned doubled
// (f +- alpha u): the halving is applied once to the reconstructed sum.
// alpha*u is rounded once and added without contraction, so the side that
// vanishes mathematically (e.g. f+ when f = a u with a < 0) is exactly zero
// instead of the rounding error of alpha*u, which the smoothness indicators
// would classify.
__device__ __forceinline__ void lf_split2(double f, double alpha, double u, double& plus2, double& minus2) {
#pragma clang fp contract(off)
  const double au = alpha * u;
  plus2 = f + au;
  minus2 = f - au;
}

// ---------------------------------------------------------------------------
// Per-cell physics of the Euler system, in a frame rotated so that
// component 1 is the momentum normal to the face (storage field of rotated
// component q: fld[q]).
// ---------------------------------------------------------------------------

// physical flux along the normal and signal speed |u_n| + c
//
// The per-cell arithmetic here, in roe_input and in the characteristic
// projection is compiled without contraction and every fused multiply-add
// is written out: each cell then goes through the same roundings wherever
// it sits in a stencil, so cells with equal values (a transmissive ghost
// region, a uniform state) give exactly equal split values, zero
// differences and beta_k = 0, whatever the instantiation around them.
template <int NF>
struct CellPrim {
  double rinv, un, e, p;  // 1/rho, normal velocity, internal energy per volume, pressure
};

template <int NF>
__device__ __forceinline__ CellPrim<NF> cell_prim(const double (&X)[NF], double gamma) {
#pragma clang fp contract(off)
  constexpr int ND = NF - 2;
  CellPrim<NF> c;
  c.rinv = rcp(X[0]);
  c.un = X[1] * c.rinv;
  double mu = 0.0;
#pragma unroll
  for (int d = 0; d < ND; ++d) mu = fma(X[1 + d], X[1 + d], mu);
  c.e = fma(-0.5 * c.rinv, mu, X[NF - 1]);
  c.p = (gamma - 1.0) * c.e;
  return c;
}

template <int NF>
__device__ __forceinline__ void cell_flux(const double (&X)[NF], const CellPrim<NF>& c, double gamma, double (&F)[NF]) {
#pragma clang fp contract(off)
  constexpr int ND = NF - 2;
  F[0] = X[1];
  F[1] = fma(X[1], c.un, c.p);
#pragma unroll
  for (int t = 1; t < ND; ++t) F[1 + t] = X[1 + t] * c.un;
  F[NF - 1] = fma(gamma - 1.0, c.e, X[NF - 1]) * c.un;
}

template <int NF>
__device__ __forceinline__ double cell_speed(const CellPrim<NF>& c, double gamma) {
#pragma clang fp contract(off)
  return fabs(c.un) + sqrt(gamma * c.p * c.rinv);
}

template <int NF>
__device__ __forceinline__ void cell_physics(const double (&X)[NF], double gamma, double (&F)[NF], double& lam) {
  const CellPrim<NF> c = cell_prim<NF>(X, gamma);
  cell_flux<NF>(X, c, gamma, F);
  lam = cell_speed<NF>(c, gamma);
}

// what the Roe average needs of one cell: sqrt(rho), velocity, enthalpy
template <int NF>
struct RoeIn {
  double rs;
  double u[NF - 2];
  double H;
};

template <int NF>
__device__ __forceinline__ void roe_input(const double (&X)[NF], double gamma, RoeIn<NF>& r) {
#pragma clang fp contract(off)
  constexpr int ND = NF - 2;
  const double rinv = rcp(X[0]);
  double q2 = 0.0;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    r.u[d] = X[1 + d] * rinv;
    q2 = fma(r.u[d], r.u[d], q2);
  }
  const double e = fma(-0.5 * X[0], q2, X[NF - 1]);
  r.H = fma(gamma - 1.0, e, X[NF - 1]) * rinv;  // (E + p) / rho
  r.rs = sqrt(X[0]);
}

// ---------------------------------------------------------------------------
// Euler face flux from a cell provider P:
//   prov.cell(m, X, F, lam)  window cell m = 0..K-1 (cells i-K/2+1 .. i+K/2)
//   prov.roe(s, r)           Roe input of cell i (s = 0) and i+1 (s = 1)
// Characteristic fields are ordered (u_n - c, entropy, shear waves in
// ascending axis order, u_n + c).
// ---------------------------------------------------------------------------
template <int NF, int K, int LIM, bool FLAGS, bool ADAPT, class P>
__device__ __forceinline__ void euler_face(P& prov, double gamma, const TenoParams& tp, double (&Fh)[NF],
                                           uint32_t (&bits)[2][NF]) {
  constexpr int ND = NF - 2;
  const double gm1 = gamma - 1.0;

  // Roe average of cells i and i+1
  double ut[ND], Ht, ct;
  {
    RoeIn<NF> a, b;
    prov.roe(0, a);
    prov.roe(1, b);
    const double w = rcp(a.rs + b.rs);
#pragma unroll
    for (int d = 0; d < ND; ++d) ut[d] = fma(a.rs, a.u[d], b.rs * b.u[d]) * w;
    Ht = fma(a.rs, a.H, b.rs * b.H) * w;
    double q2 = 0.0;
#pragma unroll
    for (int d = 0; d < ND; ++d) q2 = fma(ut[d], ut[d], q2);
    ct = sqrt(gm1 * fma(-0.5, q2, Ht));
  }
  const double cinv = rcp(ct);
  const double b1 = gm1 * cinv * cinv;
  double q2t = 0.0;
#pragma unroll
  for (int d = 0; d < ND; ++d) q2t = fma(ut[d], ut[d], q2t);
  const double b2 = 0.5 * q2t * b1;

  // left eigenvectors applied to a conservative vector X
  // (no contraction: the same roundings for every stencil cell)
  auto project = [&](const double (&X)[NF], double (&w)[NF]) {
#pragma clang fp contract(off)
    double um = 0.0;
#pragma unroll
    for (int d = 0; d < ND; ++d) um = fma(ut[d], X[1 + d], um);
    const double A = fma(b2, X[0], b1 * (X[NF - 1] - um));
    const double Bn = fma(ut[0], X[0], -X[1]);  // B = Bn / c
    w[0] = 0.5 * fma(Bn, cinv, A);
    w[1] = X[0] - A;
#pragma unroll
    for (int t = 1; t < ND; ++t) w[1 + t] = fma(-ut[t], X[0], X[1 + t]);
    w[NF - 1] = 0.5 * fma(-Bn, cinv, A);
  };

  double fc[NF];
  if constexpr (!FLAGS && P::kReread && LIM != LIM_TENO) {
    // Group by group of fields from the staged cells: each group's stencil
    // values are projected from a fresh read of the cells (only the group's
    // rows of the eigenvectors survive), so that no array of every field's
    // projections stays live across the limiter skips of the
    // reconstructions.  The same operations in the same order as below: the
    // same bits.
    double alpha = 0.0;
#pragma unroll
    for (int m = 0; m < K; ++m) alpha = fmax(alpha, prov.speed(m));
    auto group = [&](uint32_t mask) {
      const P pq = prov.fresh();
      double vp[NF][K], vm[NF][K];
#pragma unroll
      for (int m = 0; m < K; ++m) {
        double X[NF], F[NF], w[NF], g[NF];
        pq.state_flux(m, X, F);
        project(X, w);
        project(F, g);
#pragma unroll
        for (int q = 0; q < NF; ++q)
          if ((mask >> q) & 1u) lf_split2(g[q], alpha, w[q], vp[q][m], vm[q][K - 1 - m]);
      }
#pragma unroll
      for (int q = 0; q < NF; ++q) {
        if ((mask >> q) & 1u) {
          bits[0][q] = bits[1][q] = 0u;
          fc[q] = 0.5 * (teno_m<K, LIM, false, ADAPT, true>(vp[q], tp, bits[0][q]) +
                         teno_m<K, LIM, false, ADAPT, true>(vm[q], tp, bits[1][q]));
        }
      }
    };
    // The acoustic and entropy fields share their projection's terms.  In 2D
    // and 3D they form one group and each shear field is alone; in 1D the
    // acoustic pair is one group and the entropy field another (one group of
    // all three needs 190 VGPRs in the batched kernel against 162, and was
    // 10 % slower there).
    if constexpr (NF == 3) {
      group(1u | 4u);
      group(2u);
    } else {
      group(3u | (1u << (NF - 1)));
#pragma unroll
      for (int q = 2; q < NF - 1; ++q) group(1u << q);
    }
  } else {
    // stencil cells: characteristic projections of U and F, Rusanov alpha
    double W[K][NF], G[K][NF];
    double alpha = 0.0;
#pragma unroll
    for (int m = 0; m < K; ++m) {
      double X[NF], F[NF], lam;
      prov.cell(m, X, F, lam);
      alpha = fmax(alpha, lam);
      project(X, W[m]);
      project(F, G[m]);
    }

    // Rusanov split and two mirrored TENO-M reconstructions per field
#pragma unroll
    for (int q = 0; q < NF; ++q) {
      double vp[K], vm[K];
#pragma unroll
      for (int m = 0; m < K; ++m) lf_split2(G[m][q], alpha, W[m][q], vp[m], vm[K - 1 - m]);
      bits[0][q] = bits[1][q] = 0u;
      fc[q] = 0.5 * (teno_m<K, LIM, FLAGS, ADAPT>(vp, tp, bits[0][q]) + teno_m<K, LIM, FLAGS, ADAPT>(vm, tp, bits[1][q]));
    }
  }

  // back to conservative variables with the right eigenvectors
  const double s = fc[0] + fc[1] + fc[NF - 1];
  const double dlr = fc[NF - 1] - fc[0];
  Fh[0] = s;
  Fh[1] = fma(ut[0], s, ct * dlr);
  double e = fma(Ht, fc[0] + fc[NF - 1], ut[0] * ct * dlr);
  e = fma(0.5 * q2t, fc[1], e);
#pragma unroll
  for (int t = 1; t < ND; ++t) {
    Fh[1 + t] = fma(ut[t], s, fc[1 + t]);
    e = fma(ut[t], fc[1 + t], e);
  }
  Fh[NF - 1] = e;
}

// ---------------------------------------------------------------------------
// Scalar advection face flux from a provider: prov.value(m) = u of window
// cell m.  f = a u, Rusanov split with alpha = |a|.
// ---------------------------------------------------------------------------
template <int K, int LIM, bool FLAGS, bool ADAPT, class P>
__device__ __forceinline__ void scalar_face(P& prov, double a, const TenoParams& tp, double& F, uint32_t (&bits)[2]) {
  const double alpha = fabs(a);
  double vp[K], vm[K];
#pragma unroll
  for (int m = 0; m < K; ++m) {
    const double u = prov.value(m);
    lf_split2(a * u, alpha, u, vp[m], vm[K - 1 - m]);  // f- side stored mirrored
  }
  bits[0] = bits[1] = 0u;
  constexpr bool SKIP = P::kReread;
  F = 0.5 * (teno_m<K, LIM, FLAGS, ADAPT, SKIP>(vp, tp, bits[0]) + teno_m<K, LIM, FLAGS, ADAPT, SKIP>(vm, tp, bits[1]));
}

struct FaceParams {
  double gamma;
  double adv;  // advection speed along the axis (scalar system)
  TenoParams tp;
};

// Dispatch on the system: NF == 1 is scalar advection, otherwise Euler.
template <int NF, int K, int LIM, bool ADAPT, bool FLAGS, class P>
__device__ __forceinline__ void face_flux(P& prov, const FaceParams& fp, double (&F)[NF], uint32_t (&bits)[2][NF]) {
  if constexpr (NF == 1) {
    uint32_t b[2];
    scalar_face<K, LIM, FLAGS, ADAPT>(prov, fp.adv, fp.tp, F[0], b);
    bits[0][0] = b[0];
    bits[1][0] = b[1];
  } else {
    euler_face<NF, K, LIM, FLAGS, ADAPT>(prov, fp.gamma, fp.tp, F, bits);
  }
}

// ---------------------------------------------------------------------------
// Cell providers
// ---------------------------------------------------------------------------

// straight from global memory (face j of a line)
template <int NF, int K>
struct GlobalCells {
  static constexpr bool kReread = false;  // re-reads would go to memory
  const double* __restrict__ U;
  long N;
  const int* fld;
  Line L;
  int j;
  double gamma;
  __device__ __forceinline__ void load(int pos, double (&X)[NF]) const {
    const long cell = cell_at(L, pos);
#pragma unroll
    for (int q = 0; q < NF; ++q) X[q] = U[fld[q] * N + cell];
  }
  __device__ __forceinline__ void cell(int m, double (&X)[NF], double (&F)[NF], double& lam) const {
    load(j - K / 2 + m, X);
    cell_physics<NF>(X, gamma, F, lam);
  }
  __device__ __forceinline__ void roe(int s, RoeIn<NF>& r) const {
    double X[NF];
    load(j - 1 + s, X);
    roe_input<NF>(X, gamma, r);
  }
  __device__ __forceinline__ double value(int m) const { return U[cell_at(L, j - K / 2 + m)]; }
};

}  // namespace tenom
