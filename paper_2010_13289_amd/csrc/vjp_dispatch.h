// Entry points of the adjoint instantiation units.  Each unit is
// tenom_vjp_inst.hip compiled with -DTENOM_NF=<fields> -DTENOM_K=<K>.
#pragma once

#include "teno_adjoint.h"

// lim: limiter kind (tenom::LIM_*), adapt: 1 for the adaptive cutoff (K = 8)
#define TENOM_DECLARE_VJP_UNIT(NF, K) \
  hipError_t tenom_vjp_nf##NF##_k##K(int lim, int adapt, const tenom::VjpLaunch& a);

TENOM_DECLARE_VJP_UNIT(1, 6)
TENOM_DECLARE_VJP_UNIT(1, 8)
TENOM_DECLARE_VJP_UNIT(3, 6)
TENOM_DECLARE_VJP_UNIT(3, 8)
TENOM_DECLARE_VJP_UNIT(4, 6)
TENOM_DECLARE_VJP_UNIT(4, 8)
TENOM_DECLARE_VJP_UNIT(5, 6)
TENOM_DECLARE_VJP_UNIT(5, 8)
