// One instantiation unit: all limiters for TENOM_NF fields and K = TENOM_K.
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

hipError_t TENOM_EXPAND_FACES(TENOM_NF, TENOM_K)(int lim, const FacesLaunch& a) {
  switch (lim) {
    case LIM_MP: return launch_faces<TENOM_NF, TENOM_K, LIM_MP>(a);
    case LIM_TVD_MINMOD: return launch_faces<TENOM_NF, TENOM_K, LIM_TVD_MINMOD>(a);
    case LIM_TVD5: return launch_faces<TENOM_NF, TENOM_K, LIM_TVD5>(a);
    default: return hipErrorInvalidValue;
  }
}

hipError_t TENOM_EXPAND_SWEEP(TENOM_NF, TENOM_K)(int lim, const SweepLaunch& a) {
  switch (lim) {
    case LIM_MP: return launch_sweep<TENOM_NF, TENOM_K, LIM_MP>(a);
    case LIM_TVD_MINMOD: return launch_sweep<TENOM_NF, TENOM_K, LIM_TVD_MINMOD>(a);
    case LIM_TVD5: return launch_sweep<TENOM_NF, TENOM_K, LIM_TVD5>(a);
    default: return hipErrorInvalidValue;
  }
}
