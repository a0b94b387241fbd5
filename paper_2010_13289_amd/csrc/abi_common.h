// Host-side helpers shared by the C-ABI sources: the per-thread error
// message, scheme and limiter decoding, and the per-kernel event timing.
#pragma once

#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <mutex>
#include <vector>

#include "../../include/tenom.h"
#include "teno_device.h"

namespace tenom {
namespace abi {

inline thread_local char g_err[512] = "";

inline int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

inline int hip_fail(hipError_t e, const char* what) {
  return fail(TENOM_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// One SSP-RK3 step with dt from the CFL condition on the device, on the
// workspace ws of ws_bytes bytes (tenom_rk3_step_cfl; defined in
// tenom_abi.hip).
int rk3_step_cfl_ws(const tenom_grid* grid, int scheme, int limiter, double C_T, double gamma, double cfl, double* U,
                    void* ws, size_t ws_bytes, double* dt_out, hipStream_t s);

// scheme -> K (0 if invalid) and the adaptive-cutoff flag
inline int scheme_K(int scheme, bool* adaptive) {
  const int K = scheme & 0xff;
  *adaptive = (scheme & TENOM_SCHEME_ADAPTIVE) != 0;
  if (scheme & ~(0xff | TENOM_SCHEME_ADAPTIVE)) return 0;
  if (K != 6 && K != 8) return 0;
  if (*adaptive && K != 8) return 0;
  return K;
}

// limiter ID -> kernel limiter kind and the beta of Eq. large_curvature
inline bool limiter_kind(int id, int* kind, double* beta) {
  *beta = 4.0;
  switch (id) {
    case TENOM_LIM_TENO: *kind = LIM_TENO; return true;
    case TENOM_LIM_MP: *kind = LIM_MP; return true;
    case TENOM_LIM_TVD_MINMOD: *kind = LIM_TVD_MINMOD; return true;
    case TENOM_LIM_TVD5: *kind = LIM_TVD5; return true;
    case TENOM_LIM_VA: *kind = LIM_VA; return true;
    case TENOM_LIM_MP_M4_B2: *kind = LIM_MP; *beta = 2.0; return true;
    case TENOM_LIM_MP_MM_B4: *kind = LIM_MP_MM; return true;
    case TENOM_LIM_MP_MM_B2: *kind = LIM_MP_MM; *beta = 2.0; return true;
    case TENOM_LIM_MP_MM_B1: *kind = LIM_MP_MM; *beta = 1.0; return true;
    default: return false;
  }
}

// scheme, limiter, C_T and gamma checks common to every compute call
inline int check_method(int scheme, int limiter, double C_T, double gamma, bool euler, int* K_out, bool* adaptive,
                        int* kind) {
  const int K = scheme_K(scheme, adaptive);
  if (!K) return fail(TENOM_EUNSUPPORTED, "unknown scheme %d (use 6, 8 or TENOM_SCHEME_8A)", scheme);
  double beta;
  if (!limiter_kind(limiter, kind, &beta)) return fail(TENOM_EUNSUPPORTED, "unknown limiter %d", limiter);
  if (!*adaptive) {
    if (!(C_T >= 0.0)) return fail(TENOM_EINVAL, "C_T must be >= 0 (got %g)", C_T);
    // classic TENO keeps at least one candidate only if C_T <= 1/(K-2)
    if (limiter == TENOM_LIM_TENO && C_T > 1.0 / (K - 2))
      return fail(TENOM_EINVAL, "classic TENO needs C_T <= 1/(K-2) (got %g)", C_T);
  }
  if (euler && !(gamma > 1.0 && isfinite(gamma)))
    return fail(TENOM_EINVAL, "gamma must be finite and > 1 (got %g)", gamma);
  *K_out = K;
  return TENOM_OK;
}

inline TenoParams teno_params(int limiter, double C_T) {
  int kind;
  double beta;
  limiter_kind(limiter, &kind, &beta);
  TenoParams tp;
  tp.C_T = C_T;
  tp.mp_beta3 = beta / 3.0;
  return tp;
}

// ---------------------------------------------------------------------------
// kernel timing (tenom_profile_enable / tenom_profile_read)
// ---------------------------------------------------------------------------
struct ProfRec {
  int kind;
  hipEvent_t a, b;
};

inline std::mutex g_prof_mu;
inline bool g_prof_on = false;
inline std::vector<hipEvent_t> g_event_pool;
inline std::vector<ProfRec> g_prof_recs;
constexpr size_t kMaxProf = 4096;

inline hipEvent_t pool_event() {
  if (!g_event_pool.empty()) {
    hipEvent_t e = g_event_pool.back();
    g_event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets the launches made in its lifetime with two events on stream s.
// Inactive while a stream is being captured into a graph.
struct ProfScope {
  int kind;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  bool on = false;
  ProfScope(int k, hipStream_t st) : kind(k), s(st) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_on || g_prof_recs.size() >= kMaxProf) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    a = pool_event();
    b = pool_event();
    if (!a || !b) return;
    on = hipEventRecord(a, s) == hipSuccess;
  }
  ~ProfScope() {
    if (!on) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (hipEventRecord(b, s) == hipSuccess) g_prof_recs.push_back(ProfRec{kind, a, b});
  }
};

}  // namespace abi
}  // namespace tenom
