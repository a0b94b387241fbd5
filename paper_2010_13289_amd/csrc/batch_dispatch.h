// Entry points of the batched-path instantiation units.  Each unit is
// tenom_batch_inst.hip compiled with -DTENOM_TILE=<i>, one per tile shape
// kTiles[i], holding K = 6, K = 8 and the adaptive K = 8 for every limiter.
#pragma once

#include "teno_batch.h"

// K: 6 or 8; lim: limiter kind (tenom::LIM_*); adapt: 1 for the adaptive cutoff (K = 8)
#define TENOM_DECLARE_BATCH_TILE(T) \
  hipError_t tenom_batch_row_tile##T(int K, int lim, int adapt, const tenom::BatchLaunch& a);

TENOM_DECLARE_BATCH_TILE(0)
TENOM_DECLARE_BATCH_TILE(1)
TENOM_DECLARE_BATCH_TILE(2)
TENOM_DECLARE_BATCH_TILE(3)
TENOM_DECLARE_BATCH_TILE(4)
TENOM_DECLARE_BATCH_TILE(5)

// The persistent batched kernel (tenom_batch_inst.hip with -DTENOM_PERSIST):
// K = 6, K = 8 and the adaptive K = 8 for every limiter.
hipError_t tenom_batch_persist(int K, int lim, int adapt, const tenom::PersistLaunch& a);
