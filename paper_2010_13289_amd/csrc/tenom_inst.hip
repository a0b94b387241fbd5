// One instantiation unit: every limiter kind (and, for K = 8, the adaptive
// cutoff) for TENOM_NF fields and K = TENOM_K; with TENOM_TILE_UNIT the
// tile sweeps, else the face kernel and the row and march sweeps.
#include <type_traits>

#include "dispatch.h"

#ifndef TENOM_NF
#error "TENOM_NF must be defined"
#endif
#ifndef TENOM_K
#error "TENOM_K must be defined"
#endif

#define TENOM_CAT3(a, b, c, d, e) a##b##c##d##e
#define TENOM_NAME(kind, nf, k) TENOM_CAT3(tenom_, kind, _nf##nf, _k, k)
#define TENOM_UNIT_FACES(nf, k) TENOM_NAME(faces, nf, k)
#define TENOM_UNIT_SWEEP(nf, k) TENOM_NAME(sweep, nf, k)
#define TENOM_EXPAND_FACES(nf, k) TENOM_UNIT_FACES(nf, k)
#define TENOM_EXPAND_SWEEP(nf, k) TENOM_UNIT_SWEEP(nf, k)

using namespace tenom;

template <bool ADAPT, class Launch, class Fn>
static hipError_t by_limiter(int lim, const Launch& a, Fn fn) {
  switch (lim) {
    case LIM_TENO: return fn(std::integral_constant<int, LIM_TENO>{}, std::bool_constant<ADAPT>{}, a);
    case LIM_MP: return fn(std::integral_constant<int, LIM_MP>{}, std::bool_constant<ADAPT>{}, a);
    case LIM_TVD_MINMOD: return fn(std::integral_constant<int, LIM_TVD_MINMOD>{}, std::bool_constant<ADAPT>{}, a);
    case LIM_TVD5: return fn(std::integral_constant<int, LIM_TVD5>{}, std::bool_constant<ADAPT>{}, a);
    case LIM_VA: return fn(std::integral_constant<int, LIM_VA>{}, std::bool_constant<ADAPT>{}, a);
    case LIM_MP_MM: return fn(std::integral_constant<int, LIM_MP_MM>{}, std::bool_constant<ADAPT>{}, a);
    default: return hipErrorInvalidValue;
  }
}

template <class Launch, class Fn>
static hipError_t by_scheme(int lim, int adapt, const Launch& a, Fn fn) {
  if (!adapt) return by_limiter<false>(lim, a, fn);
  if constexpr (TENOM_K == 8) return by_limiter<true>(lim, a, fn);
  return hipErrorInvalidValue;  // the adaptive cutoff is defined for K = 8 only
}

#ifdef TENOM_TILE_UNIT
// The tile sweeps alone.  This unit is compiled without machine-level
// loop-invariant code motion: hoisting the constants of the face out of
// the chunk loop spills them into vector-register lanes that every face
// reads back.
#define TENOM_UNIT_TILE(nf, k) TENOM_NAME(tile, nf, k)
#define TENOM_EXPAND_TILE(nf, k) TENOM_UNIT_TILE(nf, k)
hipError_t TENOM_EXPAND_TILE(TENOM_NF, TENOM_K)(int lim, int adapt, const SweepLaunch& a) {
  return by_scheme(lim, adapt, a, [](auto L, auto A, const SweepLaunch& x) {
    return launch_tile<TENOM_NF, TENOM_K, decltype(L)::value, decltype(A)::value>(x);
  });
}
#else
hipError_t TENOM_EXPAND_FACES(TENOM_NF, TENOM_K)(int lim, int adapt, const FacesLaunch& a) {
  return by_scheme(lim, adapt, a, [](auto L, auto A, const FacesLaunch& x) {
    return launch_faces<TENOM_NF, TENOM_K, decltype(L)::value, decltype(A)::value>(x);
  });
}

hipError_t TENOM_EXPAND_SWEEP(TENOM_NF, TENOM_K)(int lim, int adapt, const SweepLaunch& a) {
  return by_scheme(lim, adapt, a, [](auto L, auto A, const SweepLaunch& x) {
    return launch_sweep<TENOM_NF, TENOM_K, decltype(L)::value, decltype(A)::value>(x);
  });
}
#endif
