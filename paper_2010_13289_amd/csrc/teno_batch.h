// Kernels of the batched path: many independent 1D Euler problems of
// uneven size, packed end to end in one structure-of-arrays state
// [field][cell] (field pitch = total cells of the batch).
//
//  k_batch_row  one workgroup per segment of one problem (TPB * FPT faces;
//               a segment table maps workgroups to (problem, first cell)):
//               the row sweep of the single-grid path with the problem's own
//               bounds, boundary rule, 1/dx and dt, fused with the RK stage
//               update Uout = a U^n + b (Us + dt div).  The tile shape
//               (TPB threads, FPT faces per thread) is a template argument;
//               the arithmetic of a face does not depend on it, so every
//               tile gives the same bits.
#pragma once

#include "teno_kernels.h"

namespace tenom {

struct TileShape {
  int tpb, fpt;
};
constexpr int kNumTiles = 6;
constexpr TileShape kTiles[kNumTiles] = {{64, 1}, {128, 1}, {128, 2}, {256, 1}, {256, 2}, {512, 1}};

template <int NF>
struct BatchParams {
  const double* U;       // stage state the stencils read
  const double* U0;      // U^n (read where a != 0)
  double* Uout;          // stage output
  double a, b;           // Uout = a U^n + b (Us + dt div)
  const long* off;       // [count + 1] first cell of each problem
  const double* inv_dx;  // [count] 1/dx of each problem
  const double* dt;      // [count] step of each problem
  const int2* segs;      // (problem, first cell within the problem) per workgroup
  long total;            // field pitch
  int bc;                // boundary rule at both ends of every problem
  FaceParams fp;
};

// Faces per workgroup: TPB * FPT.  A segment holds TPB * FPT - 1 cells (its
// TPB * FPT faces include both ends), except that a periodic problem of at
// most TPB * FPT cells is one segment whose n faces wrap around.
template <int TPB, int FPT>
struct BatchTile {
  static constexpr int FACES = TPB * FPT;
  static constexpr int CELLS = FACES - 1;
};

template <int NF, int K, int LIM, bool ADAPT, int TPB, int FPT>
__global__ __launch_bounds__(TPB) void k_batch_row(BatchParams<NF> p) {
  constexpr int SEG = BatchTile<TPB, FPT>::FACES;  // faces per workgroup
  constexpr int NC = SEG + K - 1;                  // staged cells
  constexpr int NE = RowStage<NF>::NE;
  __shared__ double stage[NE * NC];
  const int2 sg = p.segs[blockIdx.x];
  const int prob = sg.x;
  const int c_begin = sg.y;
  const long base = p.off[prob];
  const int n = (int)(p.off[prob + 1] - base);
  const bool wrap = (p.bc == 0) && (n <= SEG);  // a whole periodic problem
  const int ncell = wrap ? n : min(SEG - 1, n - c_begin);
  const int nface = wrap ? n : ncell + 1;
  const int nstage = nface + K - 1;
  const Line L{base, 1, n, p.bc};
  const int t = threadIdx.x;
  __builtin_amdgcn_s_setprio(3);  // high while loads and stores issue, as in the row sweep

  for (int c = t; c < nstage; c += TPB) {
    const long cell = cell_at(L, c_begin - K / 2 + c);
    double X[NF];
#pragma unroll
    for (int q = 0; q < NF; ++q) X[q] = p.U[q * p.total + cell];
#pragma unroll
    for (int q = 0; q < NF; ++q) stage[q * NC + c] = X[q];
    double F[NF], lam;
    RoeIn<NF> r;
    cell_physics<NF>(X, p.fp.gamma, F, lam);
    roe_input<NF>(X, p.fp.gamma, r);
#pragma unroll
    for (int q = 0; q < NF; ++q) stage[(NF + q) * NC + c] = F[q];
    stage[(2 * NF) * NC + c] = lam;
    stage[(2 * NF + 1) * NC + c] = r.rs;
#pragma unroll
    for (int d = 0; d < NF - 2; ++d) stage[(2 * NF + 2 + d) * NC + c] = r.u[d];
    stage[(3 * NF) * NC + c] = r.H;
  }
  __syncthreads();
  __builtin_amdgcn_s_setprio(0);

  double F[FPT][NF];
  double us[FPT][NF];
#pragma unroll
  for (int f = 0; f < FPT; ++f) {
    const int j = t + f * TPB;
    if (j < nface) {
      StagedCells<NF, K, 1, true> prov{stage, NC, j};
      uint32_t bits[2][NF];
      face_flux<NF, K, LIM, ADAPT, false>(prov, p.fp, F[f], bits);
    }
    if (j < ncell) {
#pragma unroll
      for (int q = 0; q < NF; ++q) us[f][q] = stage[q * NC + j + K / 2];
    }
  }
  __syncthreads();  // every face has read the staged cells
  double* Fs = stage;  // reuse: [NF][SEG + 1]
#pragma unroll
  for (int f = 0; f < FPT; ++f) {
    const int j = t + f * TPB;
    if (j < nface) {
#pragma unroll
      for (int q = 0; q < NF; ++q) Fs[q * (SEG + 1) + j] = F[f][q];
    }
  }
  __syncthreads();
  __builtin_amdgcn_s_setprio(3);
  const double dt = p.dt[prob];
  const double idx = p.inv_dx[prob];
#pragma unroll
  for (int f = 0; f < FPT; ++f) {
    const int j = t + f * TPB;
    if (j < ncell) {
      const long cell = base + c_begin + j;
      const int r = (wrap && j == n - 1) ? 0 : j + 1;
#pragma unroll
      for (int q = 0; q < NF; ++q) {
        const long o = q * p.total + cell;
        const double div = (Fs[q * (SEG + 1) + j] - Fs[q * (SEG + 1) + r]) * idx;
        const double v = fma(dt, div, us[f][q]);
        p.Uout[o] = (p.a != 0.0) ? fma(p.a, p.U0[o], p.b * v) : p.b * v;
      }
    }
  }
}

struct BatchLaunch {
  const double* U;
  const double* U0;
  double* Uout;
  double a, b;
  const long* off;
  const double* inv_dx;
  const double* dt;
  const int2* segs;
  int nseg;
  long total;
  int bc;
  FaceParams fp;
  hipStream_t stream;
};

template <int K, int LIM, bool ADAPT, int TPB, int FPT>
hipError_t launch_batch_row(const BatchLaunch& a) {
  if (a.nseg <= 0) return hipSuccess;
  BatchParams<3> p;
  p.U = a.U;
  p.U0 = a.U0;
  p.Uout = a.Uout;
  p.a = a.a;
  p.b = a.b;
  p.off = a.off;
  p.inv_dx = a.inv_dx;
  p.dt = a.dt;
  p.segs = a.segs;
  p.total = a.total;
  p.bc = a.bc;
  p.fp = a.fp;
  hipLaunchKernelGGL((k_batch_row<3, K, LIM, ADAPT, TPB, FPT>), dim3(a.nseg), dim3(TPB), 0, a.stream, p);
  return hipGetLastError();
}

}  // namespace tenom
