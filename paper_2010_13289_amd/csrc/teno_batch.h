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

// One segment of one problem, as seen by batch_segment: TPB * FPT faces
// starting at cell c_begin of the problem (cells base .. base + n - 1 of the
// state), and the stage update of the segment's cells:
// Uout = a U0 + b (Us + dt div), U0 read only where a != 0.
struct SegIn {
  const double* Us;
  const double* U0;
  double* Uout;
  double a, b, dt, idx;
  long base, total;
  int n, c_begin, bc;
};

// One segment, staged in LDS (`stage`: at least RowStage<NF>::NE *
// (TPB * FPT + K - 1) doubles; `Fs`: the faces' fluxes, NF * (TPB * FPT + 1)
// doubles).  Every thread of the workgroup calls it; both arrays may be
// rewritten once every thread has returned.  `g` may live in LDS: its fields
// are read where they are used, so that nothing of it is held through the
// face.
template <int NF, int K, int LIM, bool ADAPT, int TPB, int FPT>
__device__ __forceinline__ void batch_segment(const SegIn& g, const FaceParams& fp, double* stage, double* Fs) {
  constexpr int SEG = BatchTile<TPB, FPT>::FACES;  // faces per workgroup
  constexpr int NC = SEG + K - 1;                  // staged cells
  const int t = threadIdx.x;
  __builtin_amdgcn_s_setprio(3);  // high while loads and stores issue, as in the row sweep
  {
    const int n = g.n, c_begin = g.c_begin;
    const bool wrap = (g.bc == 0) && (n <= SEG);  // a whole periodic problem
    const int ncell = wrap ? n : min(SEG - 1, n - c_begin);
    const int nface = wrap ? n : ncell + 1;
    const int nstage = nface + K - 1;
    const Line L{g.base, 1, n, g.bc};
    const double* Us = g.Us;
    const long total = g.total;
  for (int c = t; c < nstage; c += TPB) {
    const long cell = cell_at(L, c_begin - K / 2 + c);
    double X[NF];
#pragma unroll
    for (int q = 0; q < NF; ++q) X[q] = Us[q * total + cell];
#pragma unroll
    for (int q = 0; q < NF; ++q) stage[q * NC + c] = X[q];
    double F[NF], lam;
    RoeIn<NF> r;
    cell_physics<NF>(X, fp.gamma, F, lam);
    roe_input<NF>(X, fp.gamma, r);
#pragma unroll
    for (int q = 0; q < NF; ++q) stage[(NF + q) * NC + c] = F[q];
    stage[(2 * NF) * NC + c] = lam;
    stage[(2 * NF + 1) * NC + c] = r.rs;
#pragma unroll
    for (int d = 0; d < NF - 2; ++d) stage[(2 * NF + 2 + d) * NC + c] = r.u[d];
    stage[(3 * NF) * NC + c] = r.H;
  }
  }
  __syncthreads();
  __builtin_amdgcn_s_setprio(0);

  int nface, ncell;
  {
    const int n = g.n;
    const bool wrap = (g.bc == 0) && (n <= SEG);
    ncell = wrap ? n : min(SEG - 1, n - g.c_begin);
    nface = wrap ? n : ncell + 1;
  }
#pragma unroll
  for (int f = 0; f < FPT; ++f) {
    const int j = t + f * TPB;
    if (j < nface) {
      StagedCells<NF, K, 1, true> prov{stage, NC, j};
      uint32_t bits[2][NF];
      double F[NF];
      face_flux<NF, K, LIM, ADAPT, false>(prov, fp, F, bits);
#pragma unroll
      for (int q = 0; q < NF; ++q) Fs[q * (SEG + 1) + j] = F[q];
    }
  }
  __syncthreads();  // every face's flux is in Fs
  __builtin_amdgcn_s_setprio(3);
  {
    const int n = g.n;
    const bool wrap = (g.bc == 0) && (n <= SEG);
    const long base = g.base + g.c_begin, total = g.total;
    const double a = g.a, b = g.b, dt = g.dt, idx = g.idx;
    const double* U0 = g.U0;
    double* Uout = g.Uout;
#pragma unroll
  for (int f = 0; f < FPT; ++f) {
    const int j = t + f * TPB;
    if (j < ncell) {
      const long cell = base + j;
      const int r = (wrap && j == n - 1) ? 0 : j + 1;
#pragma unroll
      for (int q = 0; q < NF; ++q) {
        const long o = q * total + cell;
        const double div = (Fs[q * (SEG + 1) + j] - Fs[q * (SEG + 1) + r]) * idx;
        const double v = fma(dt, div, stage[q * NC + j + K / 2]);
        Uout[o] = (a != 0.0) ? fma(a, U0[o], b * v) : b * v;
      }
    }
  }
  }
}

template <int NF, int K, int LIM, bool ADAPT, int TPB, int FPT>
__global__ __launch_bounds__(TPB) void k_batch_row(BatchParams<NF> p) {
  constexpr int NC = BatchTile<TPB, FPT>::FACES + K - 1;
  __shared__ double stage[RowStage<NF>::NE * NC];
  __shared__ double Fs[NF * (BatchTile<TPB, FPT>::FACES + 1)];
  const int2 sg = p.segs[blockIdx.x];
  const int prob = sg.x;
  SegIn g;
  g.Us = p.U;
  g.U0 = p.U0;
  g.Uout = p.Uout;
  g.a = p.a;
  g.b = p.b;
  g.dt = p.dt[prob];
  g.idx = p.inv_dx[prob];
  g.base = p.off[prob];
  g.n = (int)(p.off[prob + 1] - g.base);
  g.c_begin = sg.y;
  g.total = p.total;
  g.bc = p.bc;
  batch_segment<NF, K, LIM, ADAPT, TPB, FPT>(g, p.fp, stage, Fs);
}

// Signal rate (|u| + c)/dx of one 1D Euler cell (the CFL condition, Sec. 4).
__device__ __forceinline__ double euler1d_rate(double rho, double m, double E, double gamma, double inv_dx) {
  const double ri = 1.0 / rho;
  const double u = m * ri;
  const double p = (gamma - 1.0) * (E - 0.5 * rho * (u * u));
  const double c = sqrt(gamma * p * ri);
  return (fabs(u) + c) * inv_dx;
}

// Step size of one problem by one 256-thread workgroup: the largest signal
// rate over the problem's cells (as an unsigned maximum of the bit
// patterns, which orders non-negative doubles and puts NaN above all, taken
// with an LDS atomic: exact and independent of the order) and
// dt = cfl / rate; every thread returns it.  `m` is one value of shared
// memory.
__device__ __forceinline__ double batch_step_size(const double* __restrict__ U, long total, long b, long e,
                                                  double inv_dx, double gamma, double cfl, unsigned long long* m) {
  // the thread index through an opaque copy: its addresses are formed here,
  // not hoisted by the caller's loops and held through the faces
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  asm volatile("" : "+s"(gamma));  // likewise gamma - 1
  if (t == 0) *m = 0ull;
  __syncthreads();
  double best = 0.0;
  bool nan = false;
  // four cells' loads in flight per thread (the maximum does not depend on
  // the order)
  long i = b + t;
  for (; i + 768 < e; i += 1024) {
    double r[4], m[4], E[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      r[k] = U[i + 256 * k];
      m[k] = U[total + i + 256 * k];
      E[k] = U[2 * total + i + 256 * k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double s = euler1d_rate(r[k], m[k], E[k], gamma, inv_dx);
      nan |= (s != s);
      best = fmax(best, s);
    }
  }
  for (; i < e; i += 256) {
    const double s = euler1d_rate(U[i], U[total + i], U[2 * total + i], gamma, inv_dx);
    nan |= (s != s);
    best = fmax(best, s);
  }
  const unsigned long long bits = nan ? 0x7ff8000000000000ull : (unsigned long long)__double_as_longlong(best);
  atomicMax(m, bits);
  __syncthreads();
  const unsigned long long r = *m;
  __syncthreads();  // m is free again
  return cfl / __longlong_as_double((long long)r);
}

// Persistent batched SSP-RK3: one launch runs `steps` steps of every
// problem.  Each workgroup takes the next problem of `order` (longest first)
// from a queue counter, and runs it whole: per step the step size, then the
// three stages, each as the problem's 256-face segments in order, with the
// problem's stage states in U1, U2 (global memory) and a barrier between
// stages; then it takes the next.  Problems are independent, so no workgroup
// waits for another.  The last workgroup to finish clears the queue for the
// next launch.  The faces, step sizes and updates are those of
// k_batch_dt and k_batch_row: the same bits.
struct PersistParams {
  double* U;
  double* U1;
  double* U2;
  long total;
  const long* off;
  const double* inv_dx;
  double* dt;      // [count] last step of each problem
  double* tclock;  // [count] clock of each problem
  const int* order;         // [count] problems, longest first
  unsigned* queue;          // [2] next index of order, workgroups finished (0 between launches)
  int count;
  int bc;
  int steps;
  double cfl;
  FaceParams fp;
};

template <int K, int LIM, bool ADAPT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_batch_persist(PersistParams p) {
  constexpr int NF = 3, TPB = 256, FPT = 1;
  constexpr int SEG = BatchTile<TPB, FPT>::FACES;
  constexpr int NC = SEG + K - 1;
  __shared__ double stage[RowStage<NF>::NE * NC];
  __shared__ double Fs[NF * (SEG + 1)];
  __shared__ unsigned long long rate;
  // The walk over (problem, step, stage, segment) is one loop; its four
  // counters are the only values carried from pass to pass (the arguments
  // are read anew in each pass, the segment's description goes through LDS),
  // so that the face computation holds nothing else in registers.
  __shared__ SegIn g;
  // the current problem, loaded once when a workgroup takes it
  __shared__ int next, cur_n;
  __shared__ long cur_base;
  __shared__ double cur_idx;
  auto take = [&](const PersistParams& q) {  // thread 0
    next = (int)atomicAdd(q.queue, 1u);
    if (next < q.count) {
      const int prob = q.order[next];
      cur_base = q.off[prob];
      cur_n = (int)(q.off[prob + 1] - cur_base);
      cur_idx = q.inv_dx[prob];
    }
  };
  if (threadIdx.x == 0) take(p);
  __syncthreads();
  int i = next, step = 0, st = 0, c = 0;
  for (;;) {
    long off0 = 0;
    asm volatile("" : "+s"(off0));
    const PersistParams& q = *(const PersistParams*)((const char*)&p + off0);
    if (i >= q.count || q.steps <= 0) break;
    const long base = cur_base;
    const int n = cur_n;
    if (st == 0 && c == 0) {  // a step begins: its size, as k_batch_dt
      const double dt = batch_step_size(q.U, q.total, base, base + n, cur_idx, q.fp.gamma, q.cfl, &rate);
      if (threadIdx.x == 0) {
        const int prob = q.order[i];
        q.dt[prob] = dt;
        q.tclock[prob] += dt;
        g.dt = dt;
      }
    }
    if (threadIdx.x == 0) {
      g.Us = st == 0 ? q.U : (st == 1 ? q.U1 : q.U2);
      g.U0 = q.U;
      g.Uout = st == 0 ? q.U1 : (st == 1 ? q.U2 : q.U);
      g.a = st == 0 ? 0.0 : (st == 1 ? 0.75 : 1.0 / 3.0);
      g.b = st == 0 ? 1.0 : (st == 1 ? 0.25 : 2.0 / 3.0);
      g.idx = cur_idx;
      g.base = base;
      g.total = q.total;
      g.n = n;
      g.c_begin = c;
      g.bc = q.bc;
    }
    // the next position: segments of 255 cells, or one wrapped segment for
    // a periodic problem of at most 256 cells; then the next stage, step,
    // problem
    bool done = false;  // the problem's last segment
    c += ((q.bc == 0) && (n <= SEG)) ? n : SEG - 1;
    if (c >= n) {
      c = 0;
      if (++st == 3) {
        st = 0;
        if (++step == q.steps) {
          step = 0;
          done = true;
        }
      }
    }
    __syncthreads();  // g is written
    // the face's parameters read anew through an opaque pointer to the
    // argument (held from the kernel's start they would be spilled)
    long off = 0;
    asm volatile("" : "+s"(off));
    const PersistParams& pe = *(const PersistParams*)((const char*)&p + off);
    batch_segment<NF, K, LIM, ADAPT, TPB, FPT>(g, pe.fp, stage, Fs);
    if (done && threadIdx.x == 0) take(pe);
    // the next pass rewrites g and the staging array, and when it begins a
    // new stage (or step, or problem) it reads what every thread of the
    // workgroup wrote to global memory in this stage: the barrier's
    // workgroup-scope fences order both (the workgroup runs on one CU)
    __syncthreads();
    if (done) i = next;
  }
  // every workgroup has taken its last index once it counts itself finished:
  // the last one clears the queue
  if (threadIdx.x == 0) {
    long off = 0;
    asm volatile("" : "+s"(off));
    const PersistParams& pe = *(const PersistParams*)((const char*)&p + off);
    if (atomicAdd(pe.queue + 1, 1u) == gridDim.x - 1) {
      atomicExch(pe.queue, 0u);
      atomicExch(pe.queue + 1, 0u);
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

struct PersistLaunch {
  PersistParams p;
  int nblk;
  hipStream_t stream;
};

template <int K, int LIM, bool ADAPT>
hipError_t launch_batch_persist(const PersistLaunch& a) {
  if (a.nblk <= 0 || a.p.steps <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_batch_persist<K, LIM, ADAPT>), dim3(a.nblk), dim3(256), 0, a.stream, a.p);
  return hipGetLastError();
}

}  // namespace tenom
