// C-ABI layer of libtenom: argument checks, workspace layout, the sweep
// schedule of the flux divergence and the SSP-RK3 step, the wave-speed
// reduction, and optional per-kernel timing.  See include/tenom.h.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <mutex>
#include <vector>

#include "../../include/tenom.h"
#include "abi_common.h"
#include "dispatch.h"
#include "vjp_dispatch.h"

using namespace tenom;

namespace {

using namespace tenom::abi;

int nfields(const tenom_grid* g) {
  if (!g) return 0;
  if (g->system == TENOM_SYS_SCALAR) return 1;
  if (g->system == TENOM_SYS_EULER && g->ndim >= 1 && g->ndim <= 3) return g->ndim + 2;
  return 0;
}

struct Dims {
  int nx, ny, nz;
  long N;
};

Dims dims(const tenom_grid* g) {
  Dims d{g->n[0], g->ndim > 1 ? g->n[1] : 1, g->ndim > 2 ? g->n[2] : 1, 0};
  d.N = (long)d.nx * d.ny * d.nz;
  return d;
}

int check_grid(const tenom_grid* g, int K) {
  if (!g) return fail(TENOM_EINVAL, "grid is NULL");
  if (g->ndim < 1 || g->ndim > 3) return fail(TENOM_EINVAL, "ndim %d not in {1,2,3}", g->ndim);
  if (g->system != TENOM_SYS_SCALAR && g->system != TENOM_SYS_EULER)
    return fail(TENOM_EUNSUPPORTED, "unknown system %d", g->system);
  long cells = 1;
  for (int d = 0; d < g->ndim; ++d) {
    if (g->n[d] < K) return fail(TENOM_EINVAL, "axis %d has %d cells, fewer than K = %d", d, g->n[d], K);
    if (!(g->dx[d] > 0.0) || !isfinite(g->dx[d])) return fail(TENOM_EINVAL, "dx[%d] must be finite and > 0", d);
    if (g->bc[d] != TENOM_BC_PERIODIC && g->bc[d] != TENOM_BC_TRANSMISSIVE)
      return fail(TENOM_EINVAL, "bc[%d] = %d is not a boundary rule", d, g->bc[d]);
    if (g->system == TENOM_SYS_SCALAR && !isfinite(g->adv[d]))
      return fail(TENOM_EINVAL, "adv[%d] must be finite", d);
    cells *= g->n[d];
    if (cells > (1L << 31) - 1) return fail(TENOM_EINVAL, "grid has more than 2^31-1 cells");
  }
  return TENOM_OK;
}

int check_scheme(const tenom_grid* g, int scheme, int limiter, double C_T, double gamma) {
  bool adaptive;
  const int K = scheme_K(scheme, &adaptive);
  if (!K) return fail(TENOM_EUNSUPPORTED, "unknown scheme %d (use 6, 8 or TENOM_SCHEME_8A)", scheme);
  int kind;
  double beta;
  if (!limiter_kind(limiter, &kind, &beta)) return fail(TENOM_EUNSUPPORTED, "unknown limiter %d", limiter);
  int rc = check_grid(g, K);
  if (rc) return rc;
  if (!adaptive) {
    if (!(C_T >= 0.0)) return fail(TENOM_EINVAL, "C_T must be >= 0 (got %g)", C_T);
    // classic TENO keeps at least one candidate only if C_T <= 1/(K-2)
    if (limiter == TENOM_LIM_TENO && C_T > 1.0 / (K - 2))
      return fail(TENOM_EINVAL, "classic TENO needs C_T <= 1/(K-2) (got %g)", C_T);
  }
  if (g->system == TENOM_SYS_EULER && !(gamma > 1.0 && isfinite(gamma)))
    return fail(TENOM_EINVAL, "gamma must be finite and > 1 (got %g)", gamma);
  return TENOM_OK;
}

// rotated component q -> storage field, for the sweep axis
void field_map(const tenom_grid* g, int axis, int (&fld)[5]) {
  for (int q = 0; q < 5; ++q) fld[q] = 0;
  if (g->system == TENOM_SYS_SCALAR) return;
  const int nd = g->ndim;
  fld[0] = 0;
  fld[1] = 1 + axis;
  int q = 2;
  for (int t = 0; t < nd; ++t)
    if (t != axis) fld[q++] = 1 + t;
  fld[nd + 1] = nd + 1;
}

FaceParams face_params(const tenom_grid* g, int axis, int limiter, double C_T, double gamma) {
  FaceParams fp;
  int kind;
  double beta;
  limiter_kind(limiter, &kind, &beta);
  fp.gamma = gamma;
  fp.adv = (g->system == TENOM_SYS_SCALAR) ? g->adv[axis] : 0.0;
  fp.tp.C_T = C_T;
  fp.tp.mp_beta3 = beta / 3.0;
  return fp;
}

using FacesFn = hipError_t (*)(int, int, const FacesLaunch&);
using SweepFn = hipError_t (*)(int, int, const SweepLaunch&);

bool pick(int nf, int K, FacesFn* f, SweepFn* s, SweepFn* tile = nullptr) {
#define TENOM_CASE(NF, KK)                      \
  if (nf == NF && K == KK) {                    \
    *f = tenom_faces_nf##NF##_k##KK;            \
    *s = tenom_sweep_nf##NF##_k##KK;            \
    if (tile) *tile = tenom_tile_nf##NF##_k##KK; \
    return true;                                \
  }
  TENOM_CASE(1, 6)
  TENOM_CASE(1, 8)
  TENOM_CASE(3, 6)
  TENOM_CASE(3, 8)
  TENOM_CASE(4, 6)
  TENOM_CASE(4, 8)
  TENOM_CASE(5, 6)
  TENOM_CASE(5, 8)
#undef TENOM_CASE
  return false;
}

using VjpFn = hipError_t (*)(int, int, const VjpLaunch&);

VjpFn pick_vjp(int nf, int K) {
#define TENOM_VCASE(NF, KK) \
  if (nf == NF && K == KK) return tenom_vjp_nf##NF##_k##KK;
  TENOM_VCASE(1, 6)
  TENOM_VCASE(1, 8)
  TENOM_VCASE(3, 6)
  TENOM_VCASE(3, 8)
  TENOM_VCASE(4, 6)
  TENOM_VCASE(4, 8)
  TENOM_VCASE(5, 6)
  TENOM_VCASE(5, 8)
#undef TENOM_VCASE
  return nullptr;
}

// faces of `axis` in the adjoint (n + 1 transmissive, n periodic)
long vjp_faces(const tenom_grid* g, int axis) {
  const Dims d = dims(g);
  const long n = axis == 0 ? d.nx : (axis == 1 ? d.ny : d.nz);
  return d.N / n * (n + (g->bc[axis] == TENOM_BC_TRANSMISSIVE ? 1 : 0));
}

// out by the output rule `base` for the first axis, then += base.scale
// J_axis^T Lbar for each further axis
int vjp_axes(const tenom_grid* g, int scheme, int limiter, double C_T, double gamma, const double* U,
             const double* Lbar, const VjpOut& base, double* contrib, hipStream_t s) {
  bool adaptive;
  const int K = scheme_K(scheme, &adaptive);
  int kind;
  double beta;
  limiter_kind(limiter, &kind, &beta);
  VjpFn fn = pick_vjp(nfields(g), K);
  if (!fn) return fail(TENOM_EUNSUPPORTED, "no adjoint kernel for %d fields, K = %d", nfields(g), K);
  const Dims d = dims(g);
  for (int ax = 0; ax < g->ndim; ++ax) {
    VjpLaunch L;
    L.U = U;
    L.Lbar = Lbar;
    L.contrib = contrib;
    L.out = ax == 0 ? base : VjpOut{base.out, base.out, 1.0, base.scale};
    L.ax.nx = d.nx;
    L.ax.ny = d.ny;
    L.ax.nz = d.nz;
    L.ax.axis = ax;
    L.ax.bc = g->bc[ax];
    L.ax.n = ax == 0 ? d.nx : (ax == 1 ? d.ny : d.nz);
    L.ax.nfa = L.ax.n + (g->bc[ax] == TENOM_BC_TRANSMISSIVE ? 1 : 0);
    L.ax.nfaces = vjp_faces(g, ax);
    L.ax.inv_dx = 1.0 / g->dx[ax];
    field_map(g, ax, L.fld);
    L.fp = face_params(g, ax, limiter, C_T, gamma);
    L.stream = s;
    hipError_t e;
    {
      ProfScope ps(7, s);
      e = fn(kind, adaptive ? 1 : 0, L);
    }
    if (e != hipSuccess) return hip_fail(e, "adjoint kernel launch");
  }
  return TENOM_OK;
}

// out = c0 x + c1 y1 + c2 y2 elementwise over M values, rounded as
// fma(c2, y2, fma(c1, y1, c0 x))
__global__ __launch_bounds__(256) void k_comb3(double* out, double c0, const double* x, double c1,
                                               const double* __restrict__ y1, double c2,
                                               const double* __restrict__ y2, long M) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (long)gridDim.x * blockDim.x)
    out[i] = fma(c2, y2[i], fma(c1, y1[i], c0 * x[i]));
}

int comb3(double* out, double c0, const double* x, double c1, const double* y1, double c2, const double* y2, long M,
          hipStream_t s) {
  long blocks = (M + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_comb3, dim3((unsigned)blocks), dim3(256), 0, s, out, c0, x, c1, y1, c2, y2, M);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? TENOM_OK : hip_fail(e, "combination launch");
}

// kernel of the sweeps (tenom_set_sweep_kernel)
std::atomic<int> g_sweep_kernel{TENOM_SWEEP_AUTO};

int march_segment(int n, int nx, int n_other) {
  static int env = -1;
  if (env < 0) {
    const char* s = getenv("TENOM_MARCH_SEG");
    env = s ? atoi(s) : 0;
    if (env < 0) env = 0;
  }
  if (env > 0) return env;
  // aim for >= 4096 waves (two full rounds at two waves per SIMD on 256
  // CUs); segments of at least 8 cells (one redundant face per segment:
  // 8-cell segments measured faster than 4, 16 or 32 on a 1024^2 y sweep,
  // whose x groups alone give only 16 waves)
  const long waves_per_set = (long)((nx + 63) / 64) * n_other;
  long nseg = (4096 + waves_per_set - 1) / waves_per_set;
  if (nseg < 1) nseg = 1;
  long seg = (n + nseg - 1) / nseg;
  if (seg < 8) seg = (n < 8) ? n : 8;
  return (int)seg;
}

// Launch one sweep of `axis` with the given epilogue.  In the RK modes the
// stage state U_s of the update is U, the state the stencils read.
int sweep(const tenom_grid* g, int scheme, int limiter, double C_T, double gamma, int axis, const double* U,
          double* R, const double* U0, double* Uout, double a, double b, double dt, int mode, hipStream_t stream,
          const double* dtp = nullptr) {
  FacesFn ff;
  SweepFn sf, tf;
  const int nf = nfields(g);
  bool adaptive;
  const int K = scheme_K(scheme, &adaptive);
  int kind;
  double beta;
  limiter_kind(limiter, &kind, &beta);
  if (!pick(nf, K, &ff, &sf, &tf)) return fail(TENOM_EUNSUPPORTED, "no kernel for %d fields, K = %d", nf, K);
  const Dims d = dims(g);
  SweepLaunch L;
  L.axis = axis;
  L.U = U;
  L.R = R;
  L.U0 = U0;
  L.Uout = Uout;
  L.a = a;
  L.b = b;
  L.dt = dt;
  L.dtp = dtp;
  L.mode = mode;
  L.nx = d.nx;
  L.ny = d.ny;
  L.nz = d.nz;
  L.bc = g->bc[axis];
  L.inv_dx = 1.0 / g->dx[axis];
  const int n_axis = axis == 0 ? d.nx : (axis == 1 ? d.ny : d.nz);
  L.seg = axis == 0 ? 0 : march_segment(n_axis, d.nx, axis == 1 ? d.nz : d.ny);
  // The tile sweep walks whole lines, so it is taken when the lines alone
  // give at least 512 workgroups (two per CU); else the line kernels: the row
  // sweep for x (which also splits long rows), the march for y and z (which
  // splits lines into segments).  Along x the row sweep's contiguous strips
  // need no halo rows staged twice: at eight points it measured faster than
  // the tile, at six points slower (256^3 Euler, one box).
  const long tiles = tile_count(axis, d.nx, d.ny, d.nz);
  const int choice = g_sweep_kernel.load(std::memory_order_relaxed);
  const bool tile = choice == TENOM_SWEEP_TILE ||
                    (choice == TENOM_SWEEP_AUTO && tiles >= 512 && (axis != 0 || K == 6));
  field_map(g, axis, L.fld);
  L.fp = face_params(g, axis, limiter, C_T, gamma);
  L.stream = stream;
  hipError_t e;
  {
    ProfScope ps(1 + axis, stream);
    e = (tile ? tf : sf)(kind, adaptive ? 1 : 0, L);
  }
  if (e != hipSuccess) return hip_fail(e, "sweep launch");
  return TENOM_OK;
}

// small per-device buffer for the reductions
std::mutex g_red_mu;
void* g_red_buf[64] = {nullptr};

int reduction_buffer(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= 64) return fail(TENOM_EHIP, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_red_mu);
  if (!g_red_buf[dev]) {
    e = hipMalloc(&g_red_buf[dev], 16);
    if (e != hipSuccess) {
      g_red_buf[dev] = nullptr;
      return hip_fail(e, "hipMalloc reduction buffer");
    }
  }
  *out = g_red_buf[dev];
  return TENOM_OK;
}

// max over cells of sum_d (|u_d| + c)/dx_d, as the ordered bit pattern of a
// non-negative double (NaN patterns order above every finite value)
__global__ __launch_bounds__(256) void k_wave_speed(const double* __restrict__ U, long N, int ndim, int system,
                                                    double gamma, double ix0, double ix1, double ix2, double a0,
                                                    double a1, double a2, unsigned long long* out,
                                                    unsigned long long* part_out) {
  double best = 0.0;
  bool nan = false;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (long)gridDim.x * blockDim.x) {
    double s;
    if (system == TENOM_SYS_SCALAR) {
      s = fabs(a0) * ix0 + (ndim > 1 ? fabs(a1) * ix1 : 0.0) + (ndim > 2 ? fabs(a2) * ix2 : 0.0);
    } else {
      const double rho = U[i];
      const double ri = 1.0 / rho;
      double vel[3] = {0.0, 0.0, 0.0}, q2 = 0.0;
      for (int d = 0; d < ndim; ++d) {
        vel[d] = U[(1 + d) * N + i] * ri;
        q2 += vel[d] * vel[d];
      }
      const double p = (gamma - 1.0) * (U[(ndim + 1) * N + i] - 0.5 * rho * q2);
      const double c = sqrt(gamma * p * ri);
      s = (fabs(vel[0]) + c) * ix0;
      if (ndim > 1) s += (fabs(vel[1]) + c) * ix1;
      if (ndim > 2) s += (fabs(vel[2]) + c) * ix2;
    }
    if (s != s) nan = true;
    best = fmax(best, s);
  }
  unsigned long long bits = nan ? 0x7ff8000000000000ull : (unsigned long long)__double_as_longlong(best);
  // wave then block reduction of the unsigned ordering
  for (int off = 32; off > 0; off >>= 1) {
    unsigned long long o = __shfl_down(bits, off, 64);
    bits = o > bits ? o : bits;
  }
  __shared__ unsigned long long part[4];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) part[wid] = bits;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long m = part[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = part[w] > m ? part[w] : m;
    if (part_out)
      part_out[blockIdx.x] = m;
    else
      atomicMax(out, m);
  }
}

// The same maximum for the Euler equations in ND dimensions: each thread
// loads four cells before it computes any of them, so that four loads per
// field are in flight.  The arithmetic per cell is that of k_wave_speed.
template <int ND>
__global__ __launch_bounds__(256) void k_wave_speed_euler(const double* __restrict__ U, long N, double gamma,
                                                          double ix0, double ix1, double ix2,
                                                          unsigned long long* out, unsigned long long* part_out) {
  constexpr int NF = ND + 2, UNR = 4;
  const double ix[3] = {ix0, ix1, ix2};
  const long stride = (long)gridDim.x * blockDim.x;
  double best = 0.0;
  bool nan = false;
  for (long i0 = (long)blockIdx.x * blockDim.x + threadIdx.x; i0 < N; i0 += UNR * stride) {
    double X[UNR][NF];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const long i = i0 + u * stride;
      const long j = i < N ? i : i0;  // past the end: cell i0 again, which leaves the maximum unchanged
#pragma unroll
      for (int q = 0; q < NF; ++q) X[u][q] = U[q * N + j];
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const double rho = X[u][0];
      const double ri = 1.0 / rho;
      double vel[ND], q2 = 0.0;
#pragma unroll
      for (int d = 0; d < ND; ++d) {
        vel[d] = X[u][1 + d] * ri;
        q2 += vel[d] * vel[d];
      }
      const double p = (gamma - 1.0) * (X[u][NF - 1] - 0.5 * rho * q2);
      const double c = sqrt(gamma * p * ri);
      double s = (fabs(vel[0]) + c) * ix[0];
#pragma unroll
      for (int d = 1; d < ND; ++d) s += (fabs(vel[d]) + c) * ix[d];
      if (s != s) nan = true;
      best = fmax(best, s);
    }
  }
  unsigned long long bits = nan ? 0x7ff8000000000000ull : (unsigned long long)__double_as_longlong(best);
  for (int off = 32; off > 0; off >>= 1) {
    unsigned long long o = __shfl_down(bits, off, 64);
    bits = o > bits ? o : bits;
  }
  __shared__ unsigned long long part[4];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) part[wid] = bits;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long m = part[0];
    for (int w = 1; w < 4; ++w) m = part[w] > m ? part[w] : m;
    if (part_out)
      part_out[blockIdx.x] = m;
    else
      atomicMax(out, m);
  }
}

// dt = cfl / (largest signal rate) from the per-block maxima of the rate
// kernels (their ordered bit patterns), by one block of 256 threads.  A NaN
// rate orders above every finite one and gives dt = NaN; a zero rate gives
// dt = inf.
__global__ __launch_bounds__(256) void k_cfl_dt(const unsigned long long* __restrict__ part, int nparts, double cfl,
                                                double* dt_ws, double* dt_out) {
  unsigned long long bits = 0;
  for (int i = threadIdx.x; i < nparts; i += 256) bits = part[i] > bits ? part[i] : bits;
  for (int off = 32; off > 0; off >>= 1) {
    unsigned long long o = __shfl_down(bits, off, 64);
    bits = o > bits ? o : bits;
  }
  __shared__ unsigned long long w4[4];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) w4[wid] = bits;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long m = w4[0];
    for (int w = 1; w < 4; ++w) m = w4[w] > m ? w4[w] : m;
    const double dt = cfl / __longlong_as_double((long long)m);
    *dt_ws = dt;
    if (dt_out) *dt_out = dt;
  }
}

// Grid of the rate kernels: at most kRateBlocks blocks of 256 threads.
constexpr long kRateBlocks = 4096;

long rate_blocks(long N) {
  long blocks = (N + 255) / 256;
  return blocks > kRateBlocks ? kRateBlocks : blocks;
}

// Launch the rate kernel of the grid's system: per-block maxima into
// part_out, or (part_out NULL) the atomic maximum into out.
hipError_t launch_rate(const tenom_grid* grid, double gamma, const double* U, long N, unsigned long long* out,
                       unsigned long long* part_out, hipStream_t s) {
  const long blocks = rate_blocks(N);
  const double ix0 = 1.0 / grid->dx[0], ix1 = grid->ndim > 1 ? 1.0 / grid->dx[1] : 0.0,
               ix2 = grid->ndim > 2 ? 1.0 / grid->dx[2] : 0.0;
  if (grid->system == TENOM_SYS_EULER && grid->ndim == 3)
    hipLaunchKernelGGL(k_wave_speed_euler<3>, dim3((unsigned)blocks), dim3(256), 0, s, U, N, gamma, ix0, ix1, ix2, out,
                       part_out);
  else if (grid->system == TENOM_SYS_EULER && grid->ndim == 2)
    hipLaunchKernelGGL(k_wave_speed_euler<2>, dim3((unsigned)blocks), dim3(256), 0, s, U, N, gamma, ix0, ix1, ix2, out,
                       part_out);
  else if (grid->system == TENOM_SYS_EULER)
    hipLaunchKernelGGL(k_wave_speed_euler<1>, dim3((unsigned)blocks), dim3(256), 0, s, U, N, gamma, ix0, ix1, ix2, out,
                       part_out);
  else
    hipLaunchKernelGGL(k_wave_speed, dim3((unsigned)blocks), dim3(256), 0, s, U, N, grid->ndim, grid->system, gamma,
                       ix0, ix1, ix2, grid->adv[0], grid->adv[1], grid->adv[2], out, part_out);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_nonfinite(const double* __restrict__ U, long M, unsigned int* out) {
  bool bad = false;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (long)gridDim.x * blockDim.x)
    bad |= !isfinite(U[i]);
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(out, 1u);
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int tenom_num_fields(const tenom_grid* grid) { return nfields(grid); }

const char* tenom_strerror(int code) {
  switch (code) {
    case TENOM_OK: return "success";
    case TENOM_EINVAL: return "invalid argument";
    case TENOM_EUNSUPPORTED: return "unsupported scheme, limiter or system";
    case TENOM_EWORKSPACE: return "workspace too small";
    case TENOM_EHIP: return "HIP runtime error";
    case TENOM_ENONFINITE: return "non-finite value";
    default: return "unknown error";
  }
}

const char* tenom_last_error(void) { return g_err; }

int tenom_version(void) { return 10000; }

int tenom_reconstruct_faces(const tenom_grid* grid, int scheme, int limiter, double C_T, double gamma, int axis,
                            const double* U, double* Fhat, uint8_t* flags, void* stream) {
  g_err[0] = 0;
  int rc = check_scheme(grid, scheme, limiter, C_T, gamma);
  if (rc) return rc;
  if (axis < 0 || axis >= grid->ndim) return fail(TENOM_EINVAL, "axis %d not in [0, ndim)", axis);
  if (!U || !Fhat) return fail(TENOM_EINVAL, "U and Fhat must not be NULL");
  FacesFn ff;
  SweepFn sf;
  bool adaptive;
  const int K = scheme_K(scheme, &adaptive);
  int kind;
  double beta;
  limiter_kind(limiter, &kind, &beta);
  if (!pick(nfields(grid), K, &ff, &sf)) return fail(TENOM_EUNSUPPORTED, "no kernel");
  const Dims d = dims(grid);
  FacesLaunch L;
  L.U = U;
  L.Fhat = Fhat;
  L.flags = flags;
  L.axis = axis;
  L.nx = d.nx;
  L.ny = d.ny;
  L.nz = d.nz;
  L.bc = grid->bc[axis];
  field_map(grid, axis, L.fld);
  L.fp = face_params(grid, axis, limiter, C_T, gamma);
  L.stream = (hipStream_t)stream;
  hipError_t e;
  {
    ProfScope ps(0, L.stream);
    e = ff(kind, adaptive ? 1 : 0, L);
  }
  if (e != hipSuccess) return hip_fail(e, "face kernel launch");
  return TENOM_OK;
}

int tenom_flux_divergence(const tenom_grid* grid, int scheme, int limiter, double C_T, double gamma,
                          const double* U, double* dUdt, void* stream) {
  g_err[0] = 0;
  int rc = check_scheme(grid, scheme, limiter, C_T, gamma);
  if (rc) return rc;
  if (!U || !dUdt) return fail(TENOM_EINVAL, "U and dUdt must not be NULL");
  if ((const void*)U == (const void*)dUdt) return fail(TENOM_EINVAL, "dUdt must not alias U");
  hipStream_t s = (hipStream_t)stream;
  for (int ax = 0; ax < grid->ndim; ++ax) {
    rc = sweep(grid, scheme, limiter, C_T, gamma, ax, U, dUdt, nullptr, nullptr, 0.0, 0.0, 0.0,
               ax == 0 ? EPI_STORE : EPI_ACCUM, s);
    if (rc) return rc;
  }
  return TENOM_OK;
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static size_t state_bytes(const tenom_grid* grid) {
  return align256((size_t)nfields(grid) * (size_t)dims(grid).N * sizeof(double));
}

// bytes after the three states: the rate kernels' per-block maxima and dt
static size_t cfl_tail_bytes() { return align256((size_t)(kRateBlocks + 1) * sizeof(double)); }

size_t tenom_workspace_bytes(const tenom_grid* grid, int scheme) {
  bool adaptive;
  const int K = scheme_K(scheme, &adaptive);
  if (!K || check_grid(grid, K) != TENOM_OK) return 0;
  // divergence accumulator R, stage states U1 and U2, then the CFL tail
  return 3 * state_bytes(grid) + cfl_tail_bytes();
}

namespace {

// The three stages of one SSP-RK3 step: U1, U2 written, U updated in place.
int rk3_stages(const tenom_grid* g, int scheme, int limiter, double C_T, double gamma, double dt, double* U, double* R,
               double* U1, double* U2, hipStream_t s, const double* dtp = nullptr) {
  const int nd = g->ndim;
  // (a, b) of U_out = a U^n + b (U_s + dt L(U_s)), stage inputs and outputs
  const double A[3] = {0.0, 0.75, 1.0 / 3.0};
  const double B[3] = {1.0, 0.25, 2.0 / 3.0};
  const double* Uin[3] = {U, U1, U2};
  double* Uo[3] = {U1, U2, U};
  for (int st = 0; st < 3; ++st) {
    for (int ax = 0; ax < nd; ++ax) {
      const bool last = (ax == nd - 1);
      int mode = last ? (nd == 1 ? EPI_RK1 : EPI_RK) : (ax == 0 ? EPI_STORE : EPI_ACCUM);
      const int rc = sweep(g, scheme, limiter, C_T, gamma, ax, Uin[st], R, U, Uo[st], A[st], B[st], dt, mode, s, dtp);
      if (rc) return rc;
    }
  }
  return TENOM_OK;
}

int rk3_step_checks(const tenom_grid* grid, int scheme, int limiter, double C_T, double gamma, double dt,
                    const double* U, void* ws, size_t ws_bytes) {
  int rc = check_scheme(grid, scheme, limiter, C_T, gamma);
  if (rc) return rc;
  if (!U || !ws) return fail(TENOM_EINVAL, "U and ws must not be NULL");
  if (!(dt > 0.0) || !isfinite(dt)) return fail(TENOM_EINVAL, "dt must be finite and > 0 (got %g)", dt);
  if (((uintptr_t)ws & 255) != 0) return fail(TENOM_EINVAL, "workspace must be 256-byte aligned");
  const size_t need = tenom_workspace_bytes(grid, scheme);
  if (ws_bytes < need) return fail(TENOM_EWORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
  return TENOM_OK;
}

}  // namespace

int tenom_rk3_step(const tenom_grid* grid, int scheme, int limiter, double C_T, double gamma, double dt, double* U,
                   void* ws, size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  const int rc = rk3_step_checks(grid, scheme, limiter, C_T, gamma, dt, U, ws, ws_bytes);
  if (rc) return rc;
  const size_t state = state_bytes(grid);
  double* R = (double*)ws;
  double* U1 = (double*)((char*)ws + state);
  double* U2 = (double*)((char*)ws + 2 * state);
  return rk3_stages(grid, scheme, limiter, C_T, gamma, dt, U, R, U1, U2, (hipStream_t)stream);
}

int tenom_rk3_step_cfl(const tenom_grid* grid, int scheme, int limiter, double C_T, double gamma, double cfl,
                       double* U, void* ws, size_t ws_bytes, double* dt_out, void* stream) {
  g_err[0] = 0;
  return tenom::abi::rk3_step_cfl_ws(grid, scheme, limiter, C_T, gamma, cfl, U, ws, ws_bytes, dt_out,
                                     (hipStream_t)stream);
}

}  // extern "C"

// The step of tenom_rk3_step_cfl on the workspace `ws` (checks included);
// also the body of the entry point whose workspace is the library's static
// scratch array.
int tenom::abi::rk3_step_cfl_ws(const tenom_grid* grid, int scheme, int limiter, double C_T, double gamma, double cfl,
                                double* U, void* ws, size_t ws_bytes, double* dt_out, hipStream_t s) {
  if (!(cfl > 0.0) || !isfinite(cfl)) return fail(TENOM_EINVAL, "cfl must be finite and > 0 (got %g)", cfl);
  // dt is formed on the device; 1.0 stands in for it in the host checks
  const int rc = rk3_step_checks(grid, scheme, limiter, C_T, gamma, 1.0, U, ws, ws_bytes);
  if (rc) return rc;
  const size_t state = state_bytes(grid);
  double* R = (double*)ws;
  double* U1 = (double*)((char*)ws + state);
  double* U2 = (double*)((char*)ws + 2 * state);
  unsigned long long* part = (unsigned long long*)((char*)ws + 3 * state);
  double* dt_dev = (double*)(part + kRateBlocks);
  const long N = dims(grid).N;
  hipError_t e = launch_rate(grid, gamma, U, N, nullptr, part, s);
  if (e != hipSuccess) return hip_fail(e, "wave-speed kernel launch");
  hipLaunchKernelGGL(k_cfl_dt, dim3(1), dim3(256), 0, s, part, (int)rate_blocks(N), cfl, dt_dev, dt_out);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "step-size kernel launch");
  return rk3_stages(grid, scheme, limiter, C_T, gamma, 0.0, U, R, U1, U2, s, dt_dev);
}

extern "C" {

int tenom_rk3_step_stages(const tenom_grid* grid, int scheme, int limiter, double C_T, double gamma, double dt,
                          double* U, double* U1, double* U2, void* ws, size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  const int rc = rk3_step_checks(grid, scheme, limiter, C_T, gamma, dt, U, ws, ws_bytes);
  if (rc) return rc;
  if (!U1 || !U2) return fail(TENOM_EINVAL, "U1 and U2 must not be NULL");
  if (U1 == U || U2 == U || U1 == U2) return fail(TENOM_EINVAL, "U, U1 and U2 must be distinct arrays");
  return rk3_stages(grid, scheme, limiter, C_T, gamma, dt, U, (double*)ws, U1, U2, (hipStream_t)stream);
}

int tenom_max_wave_speed(const tenom_grid* grid, double gamma, const double* U, double* out_host, void* stream) {
  g_err[0] = 0;
  int rc = check_grid(grid, 1);
  if (rc) return rc;
  if (!U || !out_host) return fail(TENOM_EINVAL, "U and out_host must not be NULL");
  if (grid->system == TENOM_SYS_EULER && !(gamma > 1.0 && isfinite(gamma)))
    return fail(TENOM_EINVAL, "gamma must be finite and > 1");
  void* buf;
  rc = reduction_buffer(&buf);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const Dims d = dims(grid);
  hipError_t e = hipMemsetAsync(buf, 0, 8, s);
  if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync");
  e = launch_rate(grid, gamma, U, d.N, (unsigned long long*)buf, nullptr, s);
  if (e != hipSuccess) return hip_fail(e, "wave-speed kernel launch");
  unsigned long long bits = 0;
  e = hipMemcpyAsync(&bits, buf, 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "wave-speed readback");
  double v;
  memcpy(&v, &bits, 8);
  *out_host = v;
  return TENOM_OK;
}

int tenom_check_finite(const tenom_grid* grid, const double* U, void* stream) {
  g_err[0] = 0;
  int rc = check_grid(grid, 1);
  if (rc) return rc;
  if (!U) return fail(TENOM_EINVAL, "U must not be NULL");
  void* buf;
  rc = reduction_buffer(&buf);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const long M = (long)nfields(grid) * dims(grid).N;
  unsigned int* flag = (unsigned int*)((char*)buf + 8);
  hipError_t e = hipMemsetAsync(flag, 0, 4, s);
  if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync");
  long blocks = (M + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_nonfinite, dim3((unsigned)blocks), dim3(256), 0, s, U, M, flag);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "finiteness kernel launch");
  unsigned int h = 0;
  e = hipMemcpyAsync(&h, flag, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "finiteness readback");
  return h ? fail(TENOM_ENONFINITE, "state holds NaN or Inf") : TENOM_OK;
}

size_t tenom_vjp_workspace_bytes(const tenom_grid* grid, int scheme) {
  bool adaptive;
  const int K = scheme_K(scheme, &adaptive);
  if (!K || check_grid(grid, K) != TENOM_OK) return 0;
  long faces = 0;
  for (int ax = 0; ax < grid->ndim; ++ax) {
    const long f = vjp_faces(grid, ax);
    faces = f > faces ? f : faces;
  }
  return align256((size_t)K * (size_t)nfields(grid) * (size_t)faces * sizeof(double));
}

int tenom_flux_divergence_vjp(const tenom_grid* grid, int scheme, int limiter, double C_T, double gamma,
                              const double* U, const double* Lbar, double scale, double* Ubar, int accumulate,
                              void* ws, size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  int rc = check_scheme(grid, scheme, limiter, C_T, gamma);
  if (rc) return rc;
  if (!U || !Lbar || !Ubar || !ws) return fail(TENOM_EINVAL, "U, Lbar, Ubar and ws must not be NULL");
  if ((const void*)Ubar == (const void*)U || (const void*)Ubar == (const void*)Lbar)
    return fail(TENOM_EINVAL, "Ubar must not alias U or Lbar");
  if (!isfinite(scale)) return fail(TENOM_EINVAL, "scale must be finite");
  const size_t need = tenom_vjp_workspace_bytes(grid, scheme);
  if (ws_bytes < need) return fail(TENOM_EWORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
  return vjp_axes(grid, scheme, limiter, C_T, gamma, U, Lbar,
                  VjpOut{Ubar, accumulate != 0 ? Ubar : nullptr, 1.0, scale}, (double*)ws,
                  (hipStream_t)stream);
}

size_t tenom_rk3_vjp_workspace_bytes(const tenom_grid* grid, int scheme) {
  const size_t contrib = tenom_vjp_workspace_bytes(grid, scheme);
  if (!contrib) return 0;
  const size_t state = align256((size_t)nfields(grid) * (size_t)dims(grid).N * sizeof(double));
  return 5 * state + contrib;  // R, U1, U2, Ubar1, Ubar2, face contributions
}

namespace {

int rk3_vjp_checks(const tenom_grid* grid, int scheme, int limiter, double C_T, double gamma, double dt,
                   const double* U, const double* Ubar, void* ws, size_t ws_bytes) {
  int rc = check_scheme(grid, scheme, limiter, C_T, gamma);
  if (rc) return rc;
  if (!U || !Ubar || !ws) return fail(TENOM_EINVAL, "U, Ubar and ws must not be NULL");
  if ((const void*)U == (const void*)Ubar) return fail(TENOM_EINVAL, "Ubar must not alias U");
  if (!(dt > 0.0) || !isfinite(dt)) return fail(TENOM_EINVAL, "dt must be finite and > 0 (got %g)", dt);
  if (((uintptr_t)ws & 255) != 0) return fail(TENOM_EINVAL, "workspace must be 256-byte aligned");
  const size_t need = tenom_rk3_vjp_workspace_bytes(grid, scheme);
  if (ws_bytes < need) return fail(TENOM_EWORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
  return TENOM_OK;
}

// The reverse sweep of one step given its stage states.
int rk3_vjp_core(const tenom_grid* grid, int scheme, int limiter, double C_T, double gamma, double dt,
                 const double* U, const double* U1, const double* U2, double* Ubar, double* B1, double* B2,
                 double* contrib, hipStream_t s) {
  const long M = (long)nfields(grid) * dims(grid).N;
  int rc;
  // U3 = U/3 + 2/3 (U2 + dt L(U2)):  Ubar2 = 2/3 Ubar3 + 2/3 dt J(U2)^T Ubar3
  if ((rc = vjp_axes(grid, scheme, limiter, C_T, gamma, U2, Ubar, VjpOut{B2, Ubar, 2.0 / 3.0, 2.0 / 3.0 * dt}, contrib,
                     s)))
    return rc;
  // U2 = 3/4 U + 1/4 (U1 + dt L(U1)):  Ubar1 = 1/4 Ubar2 + 1/4 dt J(U1)^T Ubar2
  if ((rc = vjp_axes(grid, scheme, limiter, C_T, gamma, U1, B2, VjpOut{B1, B2, 0.25, 0.25 * dt}, contrib, s)))
    return rc;
  // U1 = U + dt L(U):  Ubar_n = Ubar3 / 3 + 3/4 Ubar2 + Ubar1 + dt J(U)^T Ubar1
  if ((rc = comb3(Ubar, 1.0 / 3.0, Ubar, 0.75, B2, 1.0, B1, M, s))) return rc;
  return vjp_axes(grid, scheme, limiter, C_T, gamma, U, B1, VjpOut{Ubar, Ubar, 1.0, dt}, contrib, s);
}

}  // namespace

int tenom_rk3_step_vjp(const tenom_grid* grid, int scheme, int limiter, double C_T, double gamma, double dt,
                       const double* U, double* Ubar, void* ws, size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  const int rc = rk3_vjp_checks(grid, scheme, limiter, C_T, gamma, dt, U, Ubar, ws, ws_bytes);
  if (rc) return rc;
  const size_t state = align256((size_t)nfields(grid) * (size_t)dims(grid).N * sizeof(double));
  double* R = (double*)ws;
  double* U1 = (double*)((char*)ws + state);
  double* U2 = (double*)((char*)ws + 2 * state);
  double* B1 = (double*)((char*)ws + 3 * state);
  double* B2 = (double*)((char*)ws + 4 * state);
  double* contrib = (double*)((char*)ws + 5 * state);
  hipStream_t s = (hipStream_t)stream;
  const int nd = grid->ndim;
  // the stage states of the forward step, by the same sweeps as tenom_rk3_step
  const double A[2] = {0.0, 0.75};
  const double B[2] = {1.0, 0.25};
  const double* Uin[2] = {U, U1};
  double* Uo[2] = {U1, U2};
  for (int st = 0; st < 2; ++st) {
    for (int ax = 0; ax < nd; ++ax) {
      const bool last = (ax == nd - 1);
      int mode = last ? (nd == 1 ? EPI_RK1 : EPI_RK) : (ax == 0 ? EPI_STORE : EPI_ACCUM);
      const int r = sweep(grid, scheme, limiter, C_T, gamma, ax, Uin[st], R, U, Uo[st], A[st], B[st], dt, mode, s);
      if (r) return r;
    }
  }
  return rk3_vjp_core(grid, scheme, limiter, C_T, gamma, dt, U, U1, U2, Ubar, B1, B2, contrib, s);
}

int tenom_rk3_step_vjp_stages(const tenom_grid* grid, int scheme, int limiter, double C_T, double gamma, double dt,
                              const double* U, const double* U1, const double* U2, double* Ubar, void* ws,
                              size_t ws_bytes, void* stream) {
  g_err[0] = 0;
  const int rc = rk3_vjp_checks(grid, scheme, limiter, C_T, gamma, dt, U, Ubar, ws, ws_bytes);
  if (rc) return rc;
  if (!U1 || !U2) return fail(TENOM_EINVAL, "U1 and U2 must not be NULL");
  if ((const void*)U1 == (const void*)Ubar || (const void*)U2 == (const void*)Ubar)
    return fail(TENOM_EINVAL, "Ubar must not alias U1 or U2");
  const size_t state = align256((size_t)nfields(grid) * (size_t)dims(grid).N * sizeof(double));
  double* B1 = (double*)((char*)ws + 3 * state);
  double* B2 = (double*)((char*)ws + 4 * state);
  double* contrib = (double*)((char*)ws + 5 * state);
  return rk3_vjp_core(grid, scheme, limiter, C_T, gamma, dt, U, U1, U2, Ubar, B1, B2, contrib, (hipStream_t)stream);
}

int tenom_set_sweep_kernel(int kind) {
  g_err[0] = 0;
  if (kind < TENOM_SWEEP_AUTO || kind > TENOM_SWEEP_TILE) return fail(TENOM_EINVAL, "sweep kernel %d not in {0, 1, 2}", kind);
  g_sweep_kernel.store(kind, std::memory_order_relaxed);
  return TENOM_OK;
}

int tenom_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = on != 0;
  return TENOM_OK;
}

int tenom_profile_read(int64_t* counts, double* total_ms, int nkinds) {
  g_err[0] = 0;
  if (!counts || !total_ms || nkinds < 1) return fail(TENOM_EINVAL, "bad output arrays");
  for (int k = 0; k < nkinds; ++k) {
    counts[k] = 0;
    total_ms[k] = 0.0;
  }
  std::lock_guard<std::mutex> lk(g_prof_mu);
  int rc = TENOM_OK;
  for (const ProfRec& r : g_prof_recs) {
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(r.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess && rc == TENOM_OK) rc = hip_fail(e, "profile event");
    if (r.kind >= 0 && r.kind < nkinds) {
      counts[r.kind] += 1;
      total_ms[r.kind] += ms;
    }
    g_event_pool.push_back(r.a);
    g_event_pool.push_back(r.b);
  }
  g_prof_recs.clear();
  return rc;
}

}  // extern "C"
