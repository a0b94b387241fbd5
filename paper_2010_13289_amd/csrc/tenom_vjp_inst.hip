// One adjoint instantiation unit: every limiter kind (and, for K = 8, the
// adaptive cutoff) for TENOM_NF fields and K = TENOM_K.
#include <type_traits>

#include "vjp_dispatch.h"

#ifndef TENOM_NF
#error "TENOM_NF must be defined"
#endif
#ifndef TENOM_K
#error "TENOM_K must be defined"
#endif

#define TENOM_VJP_CAT(a, b, c, d) a##b##c##d
#define TENOM_VJP_NAME(nf, k) TENOM_VJP_CAT(tenom_vjp_nf, nf, _k, k)
#define TENOM_VJP_EXPAND(nf, k) TENOM_VJP_NAME(nf, k)

using namespace tenom;

namespace {

template <bool ADAPT>
hipError_t by_limiter(int lim, const VjpLaunch& a) {
  constexpr int NF = TENOM_NF, K = TENOM_K;
  switch (lim) {
    case LIM_TENO: return launch_vjp<NF, K, LIM_TENO, ADAPT>(a);
    case LIM_MP: return launch_vjp<NF, K, LIM_MP, ADAPT>(a);
    case LIM_TVD_MINMOD: return launch_vjp<NF, K, LIM_TVD_MINMOD, ADAPT>(a);
    case LIM_TVD5: return launch_vjp<NF, K, LIM_TVD5, ADAPT>(a);
    case LIM_VA: return launch_vjp<NF, K, LIM_VA, ADAPT>(a);
    case LIM_MP_MM: return launch_vjp<NF, K, LIM_MP_MM, ADAPT>(a);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t TENOM_VJP_EXPAND(TENOM_NF, TENOM_K)(int lim, int adapt, const VjpLaunch& a) {
  if (!adapt) return by_limiter<false>(lim, a);
#if TENOM_K == 8
  return by_limiter<true>(lim, a);
#else
  return hipErrorInvalidValue;  // the adaptive cutoff is defined for K = 8 only
#endif
}
