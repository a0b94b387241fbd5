// C-ABI layer of the batched path: many independent 1D Euler problems in
// one state, each advanced by SSP-RK3 with its own CFL step.  See
// include/tenom.h (tenom_batch_*).
#include <hip/hip_runtime.h>

#include <limits.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "../../include/tenom.h"
#include "abi_common.h"
#include "batch_dispatch.h"

using namespace tenom;
using namespace tenom::abi;

struct tenom_batch_plan {
  int device = 0;
  int count = 0;
  long total = 0;
  int bc = TENOM_BC_TRANSMISSIVE;
  int min_n = 0;
  std::vector<long> off;  // [count + 1] first cell of each problem (host)
  long* off_d = nullptr;
  double* inv_dx_d = nullptr;
  double* dt_d = nullptr;
  double* t_d = nullptr;
  double* U1 = nullptr;  // stage states, [3][total] each
  double* U2 = nullptr;
  struct Tiling {
    int2* segs_d = nullptr;
    std::vector<int> first;  // [count + 1] first segment of each problem
  } tiling[kNumTiles];
  int tile = 3;
  // persistent path: the problems longest first, and the queue counters
  int nblk = 0;
  int* order_d = nullptr;
  unsigned* queue_d = nullptr;
  hipStream_t cap = nullptr;  // capture stream of the graph path
  hipGraphExec_t exec = nullptr;
  struct Key {
    int scheme, limiter, steps, tile;
    double C_T, gamma, cfl;
    const double* U;
    bool operator==(const Key& o) const {
      return scheme == o.scheme && limiter == o.limiter && steps == o.steps && tile == o.tile &&
             memcmp(&C_T, &o.C_T, sizeof(double)) == 0 && memcmp(&gamma, &o.gamma, sizeof(double)) == 0 &&
             memcmp(&cfl, &o.cfl, sizeof(double)) == 0 && U == o.U;
    }
  } key{};
};

namespace {

// Step sizes: one workgroup of 256 threads per problem p0 + blockIdx.x
// computes the largest signal rate (|u| + c)/dx over the problem's cells,
// its step dt = cfl / rate and the problem's clock t += dt.
__global__ __launch_bounds__(256) void k_batch_dt(const double* __restrict__ U, long total,
                                                  const long* __restrict__ off, const double* __restrict__ inv_dx,
                                                  double gamma, double cfl, int p0, double* __restrict__ dt,
                                                  double* __restrict__ tclock) {
  const int prob = p0 + blockIdx.x;
  __shared__ unsigned long long rate;
  const double d = batch_step_size(U, total, off[prob], off[prob + 1], inv_dx[prob], gamma, cfl, &rate);
  if (threadIdx.x == 0) {
    dt[prob] = d;
    tclock[prob] += d;
  }
}

using RowFn = hipError_t (*)(int, int, int, const BatchLaunch&);
const RowFn kRow[kNumTiles] = {tenom_batch_row_tile0, tenom_batch_row_tile1, tenom_batch_row_tile2,
                               tenom_batch_row_tile3, tenom_batch_row_tile4, tenom_batch_row_tile5};

// Segments of one tile: (problem, first cell).  A segment covers FACES - 1
// cells; a periodic problem of at most FACES cells is one wrapped segment
// (the rule k_batch_row applies).
void build_segments(const std::vector<long>& off, int bc, int faces, std::vector<int2>& segs,
                    std::vector<int>& first) {
  const int count = (int)off.size() - 1;
  first.assign(count + 1, 0);
  segs.clear();
  for (int p = 0; p < count; ++p) {
    first[p] = (int)segs.size();
    const long n = off[p + 1] - off[p];
    if (bc == TENOM_BC_PERIODIC && n <= faces) {
      segs.push_back(make_int2(p, 0));
    } else {
      for (long c = 0; c < n; c += faces - 1) segs.push_back(make_int2(p, (int)c));
    }
  }
  first[count] = (int)segs.size();
}

// Problems of the persistent path, longest first (ties by index).
std::vector<int> longest_first(const std::vector<long>& off) {
  const int count = (int)off.size() - 1;
  std::vector<int> order(count);
  for (int p = 0; p < count; ++p) order[p] = p;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return off[a + 1] - off[a] > off[b + 1] - off[b]; });
  return order;
}

void release(tenom_batch_plan* P) {
  if (!P) return;
  if (P->exec) hipGraphExecDestroy(P->exec);
  if (P->cap) hipStreamDestroy(P->cap);
  for (auto& T : P->tiling)
    if (T.segs_d) hipFree(T.segs_d);
  hipFree(P->order_d);
  hipFree(P->queue_d);
  hipFree(P->off_d);
  hipFree(P->inv_dx_d);
  hipFree(P->dt_d);
  hipFree(P->t_d);
  hipFree(P->U1);
  hipFree(P->U2);
  delete P;
}

int check_device(const tenom_batch_plan* P) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != P->device) return fail(TENOM_EINVAL, "the plan belongs to device %d, device %d is current", P->device, dev);
  return TENOM_OK;
}

struct Method {
  int K;
  bool adapt;
  int kind;
  FaceParams fp;
};

int check_call(const tenom_batch_plan* P, int scheme, int limiter, double C_T, double gamma, double cfl, int steps,
               const double* U, Method* m) {
  if (!P) return fail(TENOM_EINVAL, "plan is NULL");
  int rc = check_method(scheme, limiter, C_T, gamma, true, &m->K, &m->adapt, &m->kind);
  if (rc) return rc;
  if (P->count > 0 && P->min_n < m->K)
    return fail(TENOM_EINVAL, "a problem has %d cells, fewer than K = %d", P->min_n, m->K);
  if (!(cfl > 0.0) || !isfinite(cfl)) return fail(TENOM_EINVAL, "cfl must be finite and > 0 (got %g)", cfl);
  if (steps < 0) return fail(TENOM_EINVAL, "steps must be >= 0 (got %d)", steps);
  if (P->count > 0 && !U) return fail(TENOM_EINVAL, "U must not be NULL");
  m->fp.gamma = gamma;
  m->fp.adv = 0.0;
  m->fp.tp = teno_params(limiter, C_T);
  return check_device(P);
}

// Enqueue `steps` SSP-RK3 steps of problems [first, first + cnt) on s.
int enqueue(tenom_batch_plan* P, const Method& m, double cfl, int steps, int first, int cnt, double* U,
            hipStream_t s) {
  if (cnt <= 0 || steps <= 0) return TENOM_OK;
  const auto& T = P->tiling[P->tile];
  const int sb = T.first[first], se = T.first[first + cnt];
  BatchLaunch L;
  L.off = P->off_d;
  L.inv_dx = P->inv_dx_d;
  L.dt = P->dt_d;
  L.segs = T.segs_d + sb;
  L.nseg = se - sb;
  L.total = P->total;
  L.bc = P->bc;
  L.fp = m.fp;
  L.stream = s;
  // Uout = a U^n + b (Us + dt L(Us)) per stage
  const double A[3] = {0.0, 0.75, 1.0 / 3.0};
  const double B[3] = {1.0, 0.25, 2.0 / 3.0};
  const double* Uin[3] = {U, P->U1, P->U2};
  double* Uo[3] = {P->U1, P->U2, U};
  for (int step = 0; step < steps; ++step) {
    hipError_t e;
    {
      ProfScope ps(5, s);
      hipLaunchKernelGGL(k_batch_dt, dim3(cnt), dim3(256), 0, s, U, P->total, P->off_d, P->inv_dx_d, m.fp.gamma, cfl,
                         first, P->dt_d, P->t_d);
      e = hipGetLastError();
    }
    if (e != hipSuccess) return hip_fail(e, "batched step-size kernel launch");
    for (int st = 0; st < 3; ++st) {
      L.U = Uin[st];
      L.U0 = U;
      L.Uout = Uo[st];
      L.a = A[st];
      L.b = B[st];
      {
        ProfScope ps(4, s);
        e = kRow[P->tile](m.K, m.kind, m.adapt ? 1 : 0, L);
      }
      if (e != hipSuccess) return hip_fail(e, "batched sweep launch");
    }
  }
  return TENOM_OK;
}

}  // namespace

extern "C" {

int tenom_batch_create(int count, const int64_t* n, const double* dx, int bc, tenom_batch_plan** plan) {
  g_err[0] = 0;
  if (!plan) return fail(TENOM_EINVAL, "plan must not be NULL");
  *plan = nullptr;
  if (count < 0) return fail(TENOM_EINVAL, "count must be >= 0 (got %d)", count);
  if (count > 0 && (!n || !dx)) return fail(TENOM_EINVAL, "n and dx must not be NULL");
  if (bc != TENOM_BC_PERIODIC && bc != TENOM_BC_TRANSMISSIVE) return fail(TENOM_EINVAL, "bc %d is not a boundary rule", bc);
  std::vector<long> off(count + 1, 0);
  int min_n = INT_MAX;
  for (int p = 0; p < count; ++p) {
    if (n[p] < 6) return fail(TENOM_EINVAL, "problem %d has %lld cells, fewer than 6", p, (long long)n[p]);
    if (!(dx[p] > 0.0) || !isfinite(dx[p])) return fail(TENOM_EINVAL, "dx[%d] must be finite and > 0", p);
    off[p + 1] = off[p] + (long)n[p];
    if (off[p + 1] > (long)INT_MAX) return fail(TENOM_EINVAL, "the batch has more than 2^31-1 cells");
    if (n[p] < min_n) min_n = (int)n[p];
  }
  tenom_batch_plan* P = new (std::nothrow) tenom_batch_plan;
  if (!P) return fail(TENOM_EINVAL, "out of host memory");
  P->count = count;
  P->total = off[count];
  P->bc = bc;
  P->min_n = count > 0 ? min_n : 0;
  P->off = off;
  hipError_t e = hipGetDevice(&P->device);
  const size_t state = (size_t)3 * (size_t)P->total * sizeof(double);
  std::vector<double> inv(count);
  for (int p = 0; p < count; ++p) inv[p] = 1.0 / dx[p];
  if (e == hipSuccess) e = hipMalloc(&P->off_d, (count + 1) * sizeof(long));
  if (e == hipSuccess) e = hipMalloc(&P->inv_dx_d, (count + 1) * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&P->dt_d, (count + 1) * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&P->t_d, (count + 1) * sizeof(double));
  if (e == hipSuccess && state) e = hipMalloc(&P->U1, state);
  if (e == hipSuccess && state) e = hipMalloc(&P->U2, state);
  if (e == hipSuccess) e = hipMemcpy(P->off_d, off.data(), (count + 1) * sizeof(long), hipMemcpyHostToDevice);
  if (e == hipSuccess && count) e = hipMemcpy(P->inv_dx_d, inv.data(), count * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(P->dt_d, 0, (count + 1) * sizeof(double));
  if (e == hipSuccess) e = hipMemset(P->t_d, 0, (count + 1) * sizeof(double));
  for (int t = 0; t < kNumTiles && e == hipSuccess; ++t) {
    std::vector<int2> segs;
    build_segments(off, bc, kTiles[t].tpb * kTiles[t].fpt, segs, P->tiling[t].first);
    if (!segs.empty()) {
      e = hipMalloc(&P->tiling[t].segs_d, segs.size() * sizeof(int2));
      if (e == hipSuccess) e = hipMemcpy(P->tiling[t].segs_d, segs.data(), segs.size() * sizeof(int2), hipMemcpyHostToDevice);
    }
  }
  if (e == hipSuccess && count > 0) {
    // three 256-thread workgroups per compute unit (the persistent kernel's
    // occupancy), at most one per problem
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, P->device);
    if (e == hipSuccess) {
      P->nblk = std::min(count, std::max(1, 3 * cus));
      const std::vector<int> order = longest_first(off);
      e = hipMalloc(&P->order_d, order.size() * sizeof(int));
      if (e == hipSuccess) e = hipMalloc(&P->queue_d, 2 * sizeof(unsigned));
      if (e == hipSuccess) e = hipMemcpy(P->order_d, order.data(), order.size() * sizeof(int), hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipMemset(P->queue_d, 0, 2 * sizeof(unsigned));
    }
  }
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&P->cap, hipStreamNonBlocking);
  if (e != hipSuccess) {
    release(P);
    return hip_fail(e, "batch plan allocation");
  }
  *plan = P;
  return TENOM_OK;
}

int tenom_batch_destroy(tenom_batch_plan* plan) {
  g_err[0] = 0;
  if (!plan) return TENOM_OK;
  hipError_t e = hipDeviceSynchronize();
  release(plan);
  return e == hipSuccess ? TENOM_OK : hip_fail(e, "hipDeviceSynchronize");
}

int64_t tenom_batch_cells(const tenom_batch_plan* plan) { return plan ? (int64_t)plan->total : -1; }

int tenom_batch_tile_shape(int tile, int* threads, int* faces_per_thread) {
  g_err[0] = 0;
  if (tile < 0 || tile >= kNumTiles) return fail(TENOM_EINVAL, "tile %d not in [0, %d)", tile, kNumTiles);
  if (threads) *threads = kTiles[tile].tpb;
  if (faces_per_thread) *faces_per_thread = kTiles[tile].fpt;
  return TENOM_OK;
}

int tenom_batch_set_tile(tenom_batch_plan* plan, int tile) {
  g_err[0] = 0;
  if (!plan) return fail(TENOM_EINVAL, "plan is NULL");
  if (tile < 0 || tile >= kNumTiles) return fail(TENOM_EINVAL, "tile %d not in [0, %d)", tile, kNumTiles);
  plan->tile = tile;
  return TENOM_OK;
}

int tenom_batch_get_tile(const tenom_batch_plan* plan) { return plan ? plan->tile : -1; }

int tenom_batch_rk3(tenom_batch_plan* plan, int scheme, int limiter, double C_T, double gamma, double cfl, int steps,
                    int first, int count, double* U, void* stream) {
  g_err[0] = 0;
  Method m;
  int rc = check_call(plan, scheme, limiter, C_T, gamma, cfl, steps, U, &m);
  if (rc) return rc;
  if (first < 0 || count < 0 || first > plan->count - count)
    return fail(TENOM_EINVAL, "problems [%d, %d + %d) not within [0, %d)", first, first, count, plan->count);
  return enqueue(plan, m, cfl, steps, first, count, U, (hipStream_t)stream);
}

int tenom_batch_rk3_graph(tenom_batch_plan* plan, int scheme, int limiter, double C_T, double gamma, double cfl,
                          int steps, double* U, void* stream) {
  g_err[0] = 0;
  Method m;
  int rc = check_call(plan, scheme, limiter, C_T, gamma, cfl, steps, U, &m);
  if (rc) return rc;
  if (plan->count == 0 || steps == 0) return TENOM_OK;
  tenom_batch_plan::Key k{scheme, limiter, steps, plan->tile, C_T, gamma, cfl, U};
  hipError_t e;
  if (!plan->exec || !(k == plan->key)) {
    if (plan->exec) {
      hipGraphExecDestroy(plan->exec);
      plan->exec = nullptr;
    }
    e = hipStreamBeginCapture(plan->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    rc = enqueue(plan, m, cfl, steps, 0, plan->count, U, plan->cap);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(plan->cap, &g);
    if (rc || e != hipSuccess) {
      if (g) hipGraphDestroy(g);
      return rc ? rc : hip_fail(e, "hipStreamEndCapture");
    }
    e = hipGraphInstantiate(&plan->exec, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) {
      plan->exec = nullptr;
      return hip_fail(e, "hipGraphInstantiate");
    }
    plan->key = k;
  }
  {
    ProfScope ps(6, (hipStream_t)stream);
    e = hipGraphLaunch(plan->exec, (hipStream_t)stream);
  }
  return e == hipSuccess ? TENOM_OK : hip_fail(e, "hipGraphLaunch");
}

int tenom_batch_rk3_persistent(tenom_batch_plan* plan, int scheme, int limiter, double C_T, double gamma, double cfl,
                               int steps, double* U, void* stream) {
  g_err[0] = 0;
  Method m;
  int rc = check_call(plan, scheme, limiter, C_T, gamma, cfl, steps, U, &m);
  if (rc) return rc;
  if (plan->count == 0 || steps == 0) return TENOM_OK;
  PersistLaunch L;
  L.p.U = U;
  L.p.U1 = plan->U1;
  L.p.U2 = plan->U2;
  L.p.total = plan->total;
  L.p.off = plan->off_d;
  L.p.inv_dx = plan->inv_dx_d;
  L.p.dt = plan->dt_d;
  L.p.tclock = plan->t_d;
  L.p.order = plan->order_d;
  L.p.queue = plan->queue_d;
  L.p.count = plan->count;
  L.p.bc = plan->bc;
  L.p.steps = steps;
  L.p.cfl = cfl;
  L.p.fp = m.fp;
  L.nblk = plan->nblk;
  L.stream = (hipStream_t)stream;
  hipError_t e;
  {
    ProfScope ps(8, L.stream);
    e = tenom_batch_persist(m.K, m.kind, m.adapt ? 1 : 0, L);
  }
  return e == hipSuccess ? TENOM_OK : hip_fail(e, "persistent batched launch");
}

int tenom_batch_autotune(tenom_batch_plan* plan, int scheme, int limiter, double C_T, double gamma, double cfl,
                         const double* U, int steps, float* ms_per_step, int* best, void* stream) {
  g_err[0] = 0;
  Method m;
  int rc = check_call(plan, scheme, limiter, C_T, gamma, cfl, steps, U, &m);
  if (rc) return rc;
  if (steps < 1) return fail(TENOM_EINVAL, "autotuning needs steps >= 1");
  if (plan->count == 0) {
    if (best) *best = plan->tile;
    return TENOM_OK;
  }
  hipStream_t s = (hipStream_t)stream;
  const size_t state = (size_t)3 * (size_t)plan->total * sizeof(double);
  const size_t clocks = (size_t)(plan->count + 1) * sizeof(double);
  double* tmp = nullptr;
  double* save = nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipMalloc(&tmp, state);
  if (e == hipSuccess) e = hipMalloc(&save, 2 * clocks);
  if (e == hipSuccess) e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  if (e == hipSuccess) e = hipMemcpyAsync(save, plan->t_d, clocks, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync((char*)save + clocks, plan->dt_d, clocks, hipMemcpyDeviceToDevice, s);
  const int keep = plan->tile;
  int pick = keep;
  float best_ms = 0.f;
  for (int t = 0; t < kNumTiles && e == hipSuccess && rc == TENOM_OK; ++t) {
    plan->tile = t;
    // one untimed step, then `steps` timed steps from the same state
    e = hipMemcpyAsync(tmp, U, state, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) rc = enqueue(plan, m, cfl, 1, 0, plan->count, tmp, s);
    if (e == hipSuccess && !rc) e = hipMemcpyAsync(tmp, U, state, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && !rc) e = hipEventRecord(a, s);
    if (e == hipSuccess && !rc) rc = enqueue(plan, m, cfl, steps, 0, plan->count, tmp, s);
    if (e == hipSuccess && !rc) e = hipEventRecord(b, s);
    if (e == hipSuccess && !rc) e = hipEventSynchronize(b);
    float ms = 0.f;
    if (e == hipSuccess && !rc) e = hipEventElapsedTime(&ms, a, b);
    ms /= (float)steps;
    if (ms_per_step) ms_per_step[t] = ms;
    if (e == hipSuccess && !rc && (t == 0 || ms < best_ms)) {
      best_ms = ms;
      pick = t;
    }
  }
  plan->tile = (e == hipSuccess && !rc) ? pick : keep;
  if (save) {
    hipMemcpyAsync(plan->t_d, save, clocks, hipMemcpyDeviceToDevice, s);
    hipMemcpyAsync(plan->dt_d, (char*)save + clocks, clocks, hipMemcpyDeviceToDevice, s);
  }
  hipError_t e2 = hipStreamSynchronize(s);
  if (a) hipEventDestroy(a);
  if (b) hipEventDestroy(b);
  hipFree(tmp);
  hipFree(save);
  if (rc) return rc;
  if (e != hipSuccess) return hip_fail(e, "autotuning");
  if (e2 != hipSuccess) return hip_fail(e2, "autotuning");
  if (best) *best = plan->tile;
  return TENOM_OK;
}

int tenom_batch_times(const tenom_batch_plan* plan, double* t, double* dt, void* stream) {
  g_err[0] = 0;
  if (!plan) return fail(TENOM_EINVAL, "plan is NULL");
  int rc = check_device(plan);
  if (rc) return rc;
  if (plan->count == 0) return TENOM_OK;
  hipStream_t s = (hipStream_t)stream;
  const size_t bytes = (size_t)plan->count * sizeof(double);
  hipError_t e = hipSuccess;
  if (t) e = hipMemcpyAsync(t, plan->t_d, bytes, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && dt) e = hipMemcpyAsync(dt, plan->dt_d, bytes, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e == hipSuccess ? TENOM_OK : hip_fail(e, "batch clock readback");
}

int tenom_batch_reset_times(tenom_batch_plan* plan, void* stream) {
  g_err[0] = 0;
  if (!plan) return fail(TENOM_EINVAL, "plan is NULL");
  int rc = check_device(plan);
  if (rc) return rc;
  hipError_t e = hipMemsetAsync(plan->t_d, 0, (size_t)(plan->count + 1) * sizeof(double), (hipStream_t)stream);
  if (e == hipSuccess) e = hipMemsetAsync(plan->dt_d, 0, (size_t)(plan->count + 1) * sizeof(double), (hipStream_t)stream);
  return e == hipSuccess ? TENOM_OK : hip_fail(e, "batch clock reset");
}

}  // extern "C"
