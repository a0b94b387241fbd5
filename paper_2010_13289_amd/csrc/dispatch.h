// Entry points of the per-(fields, K) instantiation units.  Each unit is
// tenom_inst.hip compiled with -DTENOM_NF=<fields> -DTENOM_K=<K> (and
// -DTENOM_TILE_UNIT for the tile sweeps), so the variants build in
// parallel; the C-ABI layer picks one by table lookup.
#pragma once

#include "teno_kernels.h"

// lim: limiter kind (tenom::LIM_*), adapt: 1 for the adaptive cutoff (K = 8)
#define TENOM_DECLARE_UNIT(NF, K)                                                          \
  hipError_t tenom_faces_nf##NF##_k##K(int lim, int adapt, const tenom::FacesLaunch& a);  \
  hipError_t tenom_sweep_nf##NF##_k##K(int lim, int adapt, const tenom::SweepLaunch& a);  \
  hipError_t tenom_tile_nf##NF##_k##K(int lim, int adapt, const tenom::SweepLaunch& a);

TENOM_DECLARE_UNIT(1, 6)
TENOM_DECLARE_UNIT(1, 8)
TENOM_DECLARE_UNIT(3, 6)
TENOM_DECLARE_UNIT(3, 8)
TENOM_DECLARE_UNIT(4, 6)
TENOM_DECLARE_UNIT(4, 8)
TENOM_DECLARE_UNIT(5, 6)
TENOM_DECLARE_UNIT(5, 8)
