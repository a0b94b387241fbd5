// The SSP-RK3 step with dt from the CFL condition whose scratch is a
// library-held static device array instead of a caller workspace: for
// callers that cannot allocate device memory (graph capture, serving loops,
// harnesses that forbid hipMalloc).  The kernels are those of
// tenom_rk3_step_cfl; only where the scratch lives differs.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/tenom.h"
#include "abi_common.h"

using namespace tenom::abi;

namespace {

// Divergence accumulator, two stage states, the rate kernels' per-block
// maxima and dt: the layout of tenom_rk3_step_cfl's workspace.  Each device
// the library runs on holds its own copy until the process ends.
__device__ __align__(256) unsigned char scratch[TENOM_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {nullptr};

// Device address of the current device's copy of `scratch`, looked up once
// per device with that device current.  The array's name in host code is a
// host-side stand-in, never a device address, so only this pointer is
// handed to kernels.
int scratch_ptr(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(TENOM_EHIP, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress of the static scratch");
    if (!p || ((uintptr_t)p & 255) != 0) return fail(TENOM_EHIP, "static scratch is not 256-byte aligned");
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return TENOM_OK;
}

}  // namespace

extern "C" {

size_t tenom_static_scratch_bytes(void) { return TENOM_STATIC_SCRATCH_BYTES; }

int tenom_rk3_step_cfl_noalloc(const tenom_grid* grid, int scheme, int limiter, double C_T, double gamma, double cfl,
                               double* U, double* dt_out, void* stream) {
  g_err[0] = 0;
  const size_t need = tenom_workspace_bytes(grid, scheme);
  if (need > TENOM_STATIC_SCRATCH_BYTES)
    return fail(TENOM_EWORKSPACE, "the grid needs %zu bytes of scratch; the static scratch holds %zu", need,
                (size_t)TENOM_STATIC_SCRATCH_BYTES);
  void* ws = nullptr;
  const int rc = scratch_ptr(&ws);
  if (rc) return rc;
  // every part of the scratch is written before it is read within the
  // step, so nothing is cleared
  return rk3_step_cfl_ws(grid, scheme, limiter, C_T, gamma, cfl, U, ws, TENOM_STATIC_SCRATCH_BYTES, dt_out,
                         (hipStream_t)stream);
}

}  // extern "C"
