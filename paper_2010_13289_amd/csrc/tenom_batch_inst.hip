// One batched-path instantiation unit: the tile shape kTiles[TENOM_TILE]
// (or, with TENOM_PERSIST, the persistent kernel), every limiter kind, K = 6,
// K = 8 and the adaptive cutoff of K = 8.
#include "batch_dispatch.h"

#ifdef TENOM_PERSIST

using namespace tenom;

namespace {

template <int K, bool ADAPT>
hipError_t by_limiter(int lim, const PersistLaunch& a) {
  switch (lim) {
    case LIM_TENO: return launch_batch_persist<K, LIM_TENO, ADAPT>(a);
    case LIM_MP: return launch_batch_persist<K, LIM_MP, ADAPT>(a);
    case LIM_TVD_MINMOD: return launch_batch_persist<K, LIM_TVD_MINMOD, ADAPT>(a);
    case LIM_TVD5: return launch_batch_persist<K, LIM_TVD5, ADAPT>(a);
    case LIM_VA: return launch_batch_persist<K, LIM_VA, ADAPT>(a);
    case LIM_MP_MM: return launch_batch_persist<K, LIM_MP_MM, ADAPT>(a);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t tenom_batch_persist(int K, int lim, int adapt, const PersistLaunch& a) {
  if (K == 6 && !adapt) return by_limiter<6, false>(lim, a);
  if (K == 8) return adapt ? by_limiter<8, true>(lim, a) : by_limiter<8, false>(lim, a);
  return hipErrorInvalidValue;
}

#else

#ifndef TENOM_TILE
#error "TENOM_TILE must be defined"
#endif

#define TENOM_BATCH_CAT(a, b) a##b
#define TENOM_BATCH_NAME(t) TENOM_BATCH_CAT(tenom_batch_row_tile, t)

using namespace tenom;

namespace {

constexpr int TPB = kTiles[TENOM_TILE].tpb;
constexpr int FPT = kTiles[TENOM_TILE].fpt;

template <int K, bool ADAPT>
hipError_t by_limiter(int lim, const BatchLaunch& a) {
  switch (lim) {
    case LIM_TENO: return launch_batch_row<K, LIM_TENO, ADAPT, TPB, FPT>(a);
    case LIM_MP: return launch_batch_row<K, LIM_MP, ADAPT, TPB, FPT>(a);
    case LIM_TVD_MINMOD: return launch_batch_row<K, LIM_TVD_MINMOD, ADAPT, TPB, FPT>(a);
    case LIM_TVD5: return launch_batch_row<K, LIM_TVD5, ADAPT, TPB, FPT>(a);
    case LIM_VA: return launch_batch_row<K, LIM_VA, ADAPT, TPB, FPT>(a);
    case LIM_MP_MM: return launch_batch_row<K, LIM_MP_MM, ADAPT, TPB, FPT>(a);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t TENOM_BATCH_NAME(TENOM_TILE)(int K, int lim, int adapt, const BatchLaunch& a) {
  if (K == 6 && !adapt) return by_limiter<6, false>(lim, a);
  if (K == 8) return adapt ? by_limiter<8, true>(lim, a) : by_limiter<8, false>(lim, a);
  return hipErrorInvalidValue;
}

#endif  // TENOM_PERSIST
