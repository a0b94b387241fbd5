"""tenom: TENO-M per-face reconstruction on AMD MI355X (gfx950).

Thin ctypes binding of libtenom.so (C ABI in include/tenom.h).  Every step
of the computation runs in the library's HIP kernels; this module only
checks tensors, marshals arguments and passes torch's current HIP stream.
PyTorch provides device memory and streams.  If the library is missing the
import of any compute call raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtenom.so")

# identifiers (include/tenom.h)
OK, EINVAL, EUNSUPPORTED, EWORKSPACE, EHIP, ENONFINITE = 0, -1, -2, -3, -4, -5
BC_PERIODIC, BC_TRANSMISSIVE = 0, 1
SYS_SCALAR, SYS_EULER = 0, 1
SCHEME_6, SCHEME_8 = 6, 8
SCHEME_ADAPTIVE = 0x100
SCHEME_8A = SCHEME_8 | SCHEME_ADAPTIVE   # eight points, adaptive cutoff (TENO8A)
LIM_TENO, LIM_MP, LIM_TVD_MINMOD, LIM_TVD5, LIM_VA = 0, 1, 2, 3, 4
LIM_MP_M4_B2, LIM_MP_MM_B4, LIM_MP_MM_B2, LIM_MP_MM_B1 = 5, 6, 7, 8
KERNEL_KINDS = ("faces", "sweep_x", "sweep_y", "sweep_z", "batch_sweep", "batch_dt", "batch_graph", "vjp_axis",
                "batch_persist")
BATCH_TILES = 6

SYMBOLS = (
    "tenom_num_fields", "tenom_reconstruct_faces", "tenom_flux_divergence", "tenom_rk3_step",
    "tenom_workspace_bytes", "tenom_max_wave_speed", "tenom_check_finite", "tenom_strerror",
    "tenom_last_error", "tenom_version", "tenom_profile_enable", "tenom_profile_read",
    "tenom_batch_tile_shape", "tenom_batch_create", "tenom_batch_destroy", "tenom_batch_cells",
    "tenom_batch_set_tile", "tenom_batch_get_tile", "tenom_batch_rk3", "tenom_batch_rk3_graph",
    "tenom_batch_autotune", "tenom_batch_times", "tenom_batch_reset_times", "tenom_batch_rk3_persistent",
    "tenom_vjp_workspace_bytes", "tenom_flux_divergence_vjp", "tenom_rk3_vjp_workspace_bytes",
    "tenom_rk3_step_vjp", "tenom_rk3_step_stages", "tenom_rk3_step_vjp_stages", "tenom_rk3_step_cfl",
    "tenom_static_scratch_bytes", "tenom_rk3_step_cfl_noalloc", "tenom_set_sweep_kernel",
)


class TenomError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"tenom error {code}: {msg}")
        self.code = code


class _CGrid(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("n", C.c_int32 * 3), ("dx", C.c_double * 3),
                ("bc", C.c_int32 * 3), ("system", C.c_int32), ("adv", C.c_double * 3)]


@dataclass
class Grid:
    """Uniform Cartesian grid: n and dx in x, y, z order, one entry per axis."""
    ndim: int
    n: Sequence[int]
    dx: Sequence[float]
    bc: Sequence[int] = field(default_factory=lambda: (BC_PERIODIC,) * 3)
    system: int = SYS_EULER
    adv: Sequence[float] = (0.0, 0.0, 0.0)

    @classmethod
    def of(cls, g) -> "Grid":
        if isinstance(g, Grid):
            return g
        nd = int(g["ndim"])
        return cls(ndim=nd, n=tuple(g["n"]), dx=tuple(g.get("dx", [1.0] * nd)),
                   bc=tuple(g.get("bc", [0] * nd)), system=int(g.get("system", SYS_EULER)),
                   adv=tuple(g.get("adv", [0.0] * nd)))

    def to_c(self) -> _CGrid:
        c = _CGrid()
        c.ndim = int(self.ndim)
        for d in range(3):
            c.n[d] = int(self.n[d]) if d < self.ndim else 1
            c.dx[d] = float(self.dx[d]) if d < len(self.dx) else 1.0
            c.bc[d] = int(self.bc[d]) if d < len(self.bc) else 0
            c.adv[d] = float(self.adv[d]) if d < len(self.adv) else 0.0
        c.system = int(self.system)
        return c

    @property
    def nfields(self) -> int:
        return 1 if self.system == SYS_SCALAR else self.ndim + 2

    def state_shape(self):
        return (self.nfields,) + tuple(int(v) for v in reversed(list(self.n)[: self.ndim]))

    def face_shape(self, axis: int):
        n = [int(v) for v in list(self.n)[: self.ndim]]
        n[axis] += 1
        return (self.nfields,) + tuple(reversed(n))


_lib = None


def build_library(verbose: bool = False) -> str:
    """Compile libtenom.so in-tree (hipcc, gfx950)."""
    from . import build as _build
    return _build.build(verbose=verbose)


def lib() -> C.CDLL:
    """Load libtenom.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2010_13289_amd.build`")
        L = C.CDLL(LIB_PATH)
        gp, vp, dp = C.POINTER(_CGrid), C.c_void_p, C.c_double
        L.tenom_num_fields.argtypes = [gp]
        L.tenom_reconstruct_faces.argtypes = [gp, C.c_int, C.c_int, dp, dp, C.c_int, vp, vp, vp, vp]
        L.tenom_flux_divergence.argtypes = [gp, C.c_int, C.c_int, dp, dp, vp, vp, vp]
        L.tenom_rk3_step.argtypes = [gp, C.c_int, C.c_int, dp, dp, dp, vp, vp, C.c_size_t, vp]
        L.tenom_rk3_step_cfl.argtypes = [gp, C.c_int, C.c_int, dp, dp, dp, vp, vp, C.c_size_t, vp, vp]
        L.tenom_rk3_step_cfl_noalloc.argtypes = [gp, C.c_int, C.c_int, dp, dp, dp, vp, vp, vp]
        L.tenom_static_scratch_bytes.restype = C.c_size_t
        L.tenom_workspace_bytes.argtypes = [gp, C.c_int]
        L.tenom_workspace_bytes.restype = C.c_size_t
        L.tenom_max_wave_speed.argtypes = [gp, dp, vp, C.POINTER(C.c_double), vp]
        L.tenom_check_finite.argtypes = [gp, vp, vp]
        L.tenom_strerror.argtypes = [C.c_int]
        L.tenom_strerror.restype = C.c_char_p
        L.tenom_last_error.restype = C.c_char_p
        L.tenom_profile_enable.argtypes = [C.c_int]
        L.tenom_set_sweep_kernel.argtypes = [C.c_int]
        L.tenom_profile_read.argtypes = [C.POINTER(C.c_int64), C.POINTER(C.c_double), C.c_int]
        ip = C.c_int
        L.tenom_batch_tile_shape.argtypes = [ip, C.POINTER(ip), C.POINTER(ip)]
        L.tenom_batch_create.argtypes = [ip, C.POINTER(C.c_int64), C.POINTER(C.c_double), ip, C.POINTER(vp)]
        L.tenom_batch_destroy.argtypes = [vp]
        L.tenom_batch_cells.argtypes = [vp]
        L.tenom_batch_cells.restype = C.c_int64
        L.tenom_batch_set_tile.argtypes = [vp, ip]
        L.tenom_batch_get_tile.argtypes = [vp]
        L.tenom_batch_rk3.argtypes = [vp, ip, ip, dp, dp, dp, ip, ip, ip, vp, vp]
        L.tenom_batch_rk3_graph.argtypes = [vp, ip, ip, dp, dp, dp, ip, vp, vp]
        L.tenom_batch_rk3_persistent.argtypes = [vp, ip, ip, dp, dp, dp, ip, vp, vp]
        L.tenom_batch_autotune.argtypes = [vp, ip, ip, dp, dp, dp, vp, ip, C.POINTER(C.c_float),
                                           C.POINTER(ip), vp]
        L.tenom_batch_times.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double), vp]
        L.tenom_batch_reset_times.argtypes = [vp, vp]
        L.tenom_vjp_workspace_bytes.argtypes = [gp, C.c_int]
        L.tenom_vjp_workspace_bytes.restype = C.c_size_t
        L.tenom_rk3_vjp_workspace_bytes.argtypes = [gp, C.c_int]
        L.tenom_rk3_vjp_workspace_bytes.restype = C.c_size_t
        L.tenom_flux_divergence_vjp.argtypes = [gp, C.c_int, C.c_int, dp, dp, vp, vp, dp, vp, C.c_int, vp,
                                                C.c_size_t, vp]
        L.tenom_rk3_step_vjp.argtypes = [gp, C.c_int, C.c_int, dp, dp, dp, vp, vp, vp, C.c_size_t, vp]
        L.tenom_rk3_step_stages.argtypes = [gp, C.c_int, C.c_int, dp, dp, dp, vp, vp, vp, vp, C.c_size_t, vp]
        L.tenom_rk3_step_vjp_stages.argtypes = [gp, C.c_int, C.c_int, dp, dp, dp, vp, vp, vp, vp, vp, C.c_size_t,
                                                vp]
        _lib = L
    return _lib


def _check(rc: int):
    if rc != OK:
        msg = lib().tenom_last_error().decode() or lib().tenom_strerror(rc).decode()
        raise TenomError(rc, msg)


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _state(U, grid: Grid, name="U"):
    import torch
    if not isinstance(U, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if U.dtype != torch.float64 or not U.is_cuda or not U.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 tensor on a HIP device")
    if tuple(U.shape) != grid.state_shape():
        raise ValueError(f"{name} has shape {tuple(U.shape)}, expected {grid.state_shape()}")
    return C.c_void_p(U.data_ptr())


def reconstruct_faces(U, grid, scheme: int, limiter: int, C_T: float, gamma: float, axis: int,
                      return_flags: bool = False, out=None, stream=None):
    """Face fluxes of one axis (shape of U with n_axis + 1 along the axis);
    with return_flags also the [2, nf, faces...] uint8 smoothness flags."""
    import torch
    g = Grid.of(grid)
    ptr = _state(U, g)
    fshape = g.face_shape(axis) if 0 <= axis < g.ndim else None
    if fshape is None:
        raise TenomError(EINVAL, f"axis {axis} out of range")
    if out is None:
        out = torch.empty(fshape, dtype=torch.float64, device=U.device)
    elif tuple(out.shape) != fshape or out.dtype != torch.float64 or not out.is_contiguous():
        raise ValueError("out has the wrong shape, dtype or layout")
    flags = torch.empty((2,) + fshape, dtype=torch.uint8, device=U.device) if return_flags else None
    gc = g.to_c()
    _check(lib().tenom_reconstruct_faces(C.byref(gc), scheme, limiter, C_T, gamma, axis, ptr,
                                         C.c_void_p(out.data_ptr()),
                                         C.c_void_p(flags.data_ptr()) if flags is not None else None,
                                         _stream(stream)))
    return (out, flags) if return_flags else out


def flux_divergence(U, grid, scheme: int, limiter: int, C_T: float, gamma: float, out=None, stream=None):
    """dU/dt = -sum_axis dF/dx (same shape as U)."""
    import torch
    g = Grid.of(grid)
    ptr = _state(U, g)
    if out is None:
        out = torch.empty_like(U)
    optr = _state(out, g, "out")
    gc = g.to_c()
    _check(lib().tenom_flux_divergence(C.byref(gc), scheme, limiter, C_T, gamma, ptr, optr, _stream(stream)))
    return out


def workspace_bytes(grid, scheme: int) -> int:
    g = Grid.of(grid).to_c()
    return int(lib().tenom_workspace_bytes(C.byref(g), scheme))


class Workspace:
    """Device workspace for rk3_step, owned by a torch uint8 tensor."""

    def __init__(self, grid, scheme: int, device="cuda"):
        import torch
        nbytes = workspace_bytes(grid, scheme)
        if nbytes == 0:
            raise TenomError(EINVAL, "invalid grid or scheme for a workspace")
        # torch's caching allocator returns >= 256-byte aligned blocks
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.nbytes = nbytes

    @property
    def ptr(self):
        return C.c_void_p(self.buf.data_ptr())


def rk3_step(U, grid, scheme: int, limiter: int, C_T: float, gamma: float, dt: float,
             workspace: Workspace | None = None, stream=None, stages=None):
    """One SSP-RK3 step in place on U; returns U.  stages = (U1, U2): device
    arrays that receive the step's stage states (tenom_rk3_step_stages)."""
    g = Grid.of(grid)
    ptr = _state(U, g)
    ws = workspace if workspace is not None else Workspace(g, scheme, U.device)
    gc = g.to_c()
    if stages is None:
        _check(lib().tenom_rk3_step(C.byref(gc), scheme, limiter, C_T, gamma, dt, ptr, ws.ptr, ws.nbytes,
                                    _stream(stream)))
    else:
        p1, p2 = _state(stages[0], g, "U1"), _state(stages[1], g, "U2")
        _check(lib().tenom_rk3_step_stages(C.byref(gc), scheme, limiter, C_T, gamma, dt, ptr, p1, p2, ws.ptr,
                                           ws.nbytes, _stream(stream)))
    return U


def rk3_step_cfl(U, grid, scheme: int, limiter: int, C_T: float, gamma: float, cfl: float,
                 workspace: Workspace | None = None, stream=None, dt_out=None):
    """One SSP-RK3 step in place on U with dt = cfl / max_wave_speed(U)
    taken on the device (tenom_rk3_step_cfl): no synchronisation, so it can
    be captured in a graph.  dt_out: optional 1-element float64 device
    tensor that receives the dt used.  Returns U."""
    g = Grid.of(grid)
    ptr = _state(U, g)
    ws = workspace if workspace is not None else Workspace(g, scheme, U.device)
    dptr = None
    if dt_out is not None:
        import torch
        if not (dt_out.is_cuda and dt_out.dtype == torch.float64 and dt_out.numel() >= 1 and dt_out.is_contiguous()):
            raise TenomError(EINVAL, "dt_out must be a contiguous float64 device tensor with at least one element")
        dptr = C.c_void_p(dt_out.data_ptr())
    gc = g.to_c()
    _check(lib().tenom_rk3_step_cfl(C.byref(gc), scheme, limiter, C_T, gamma, cfl, ptr, ws.ptr, ws.nbytes, dptr,
                                    _stream(stream)))
    return U


def static_scratch_bytes() -> int:
    """Size of the library-held scratch of rk3_step_cfl_noalloc."""
    return int(lib().tenom_static_scratch_bytes())


def rk3_step_cfl_noalloc(U, grid, scheme: int, limiter: int, C_T: float, gamma: float, cfl: float,
                         stream=None, dt_out=None):
    """rk3_step_cfl without a workspace: the scratch is the library's static
    device array (tenom_rk3_step_cfl_noalloc), so the call allocates
    nothing.  Grids whose workspace_bytes exceed static_scratch_bytes()
    raise EWORKSPACE.  Overlapping calls on one device race.  Returns U."""
    g = Grid.of(grid)
    ptr = _state(U, g)
    dptr = None
    if dt_out is not None:
        import torch
        if not (dt_out.is_cuda and dt_out.dtype == torch.float64 and dt_out.numel() >= 1 and dt_out.is_contiguous()):
            raise TenomError(EINVAL, "dt_out must be a contiguous float64 device tensor with at least one element")
        dptr = C.c_void_p(dt_out.data_ptr())
    gc = g.to_c()
    _check(lib().tenom_rk3_step_cfl_noalloc(C.byref(gc), scheme, limiter, C_T, gamma, cfl, ptr, dptr,
                                            _stream(stream)))
    return U


def max_wave_speed(U, grid, gamma: float, stream=None) -> float:
    """max over cells of sum_d (|u_d| + c)/dx_d; dt = CFL / this."""
    g = Grid.of(grid)
    ptr = _state(U, g)
    out = C.c_double()
    gc = g.to_c()
    _check(lib().tenom_max_wave_speed(C.byref(gc), gamma, ptr, C.byref(out), _stream(stream)))
    return out.value


def check_finite(U, grid, stream=None) -> bool:
    g = Grid.of(grid)
    ptr = _state(U, g)
    gc = g.to_c()
    rc = lib().tenom_check_finite(C.byref(gc), ptr, _stream(stream))
    if rc == ENONFINITE:
        return False
    _check(rc)
    return True


SWEEP_AUTO, SWEEP_MARCH, SWEEP_TILE = 0, 1, 2


def set_sweep_kernel(kind: int):
    """Kernel of the sweeps for every later call (SWEEP_AUTO, SWEEP_MARCH:
    the line kernels, or SWEEP_TILE); all give the same bits."""
    _check(lib().tenom_set_sweep_kernel(int(kind)))


def profile_enable(on: bool = True):
    _check(lib().tenom_profile_enable(1 if on else 0))


def profile_read() -> dict:
    """{kind: (launches, total_ms)} since the last read (synchronises)."""
    n = len(KERNEL_KINDS)
    cnt = (C.c_int64 * n)()
    ms = (C.c_double * n)()
    _check(lib().tenom_profile_read(cnt, ms, n))
    return {k: (int(cnt[i]), float(ms[i])) for i, k in enumerate(KERNEL_KINDS)}


# ---------------------------------------------------------------------------
# batched independent 1D Euler problems
# ---------------------------------------------------------------------------

def batch_tile_shape(tile: int) -> tuple[int, int]:
    """(threads per workgroup, faces per thread) of a batched tile shape."""
    t, f = C.c_int(), C.c_int()
    _check(lib().tenom_batch_tile_shape(int(tile), C.byref(t), C.byref(f)))
    return t.value, f.value


class BatchPlan:
    """Plan of a batch of independent 1D Euler problems (tenom_batch_*).

    sizes[p] cells of size dx[p] per problem, one boundary rule for all.
    The state is a float64 tensor [3, total] with the problems packed end to
    end (``offsets`` gives each problem's first cell)."""

    def __init__(self, sizes, dx, bc: int = BC_TRANSMISSIVE):
        import numpy as np
        n = np.ascontiguousarray(sizes, dtype=np.int64)
        d = np.ascontiguousarray(dx, dtype=np.float64)
        if n.ndim != 1 or d.shape != n.shape:
            raise ValueError("sizes and dx must be 1D arrays of equal length")
        self.count = int(n.size)
        self.sizes = n
        self.offsets = np.concatenate([[0], np.cumsum(n)]).astype(np.int64)
        self._h = C.c_void_p()
        _check(lib().tenom_batch_create(self.count, n.ctypes.data_as(C.POINTER(C.c_int64)),
                                        d.ctypes.data_as(C.POINTER(C.c_double)), int(bc), C.byref(self._h)))
        self.total = int(lib().tenom_batch_cells(self._h))

    def close(self):
        if self._h:
            _check(lib().tenom_batch_destroy(self._h))
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _state(self, U):
        import torch
        if not isinstance(U, torch.Tensor) or U.dtype != torch.float64 or not U.is_cuda or not U.is_contiguous():
            raise ValueError("U must be a contiguous float64 tensor on a HIP device")
        if tuple(U.shape) != (3, self.total):
            raise ValueError(f"U has shape {tuple(U.shape)}, expected (3, {self.total})")
        return C.c_void_p(U.data_ptr())

    @property
    def tile(self) -> int:
        return int(lib().tenom_batch_get_tile(self._h))

    @tile.setter
    def tile(self, t: int):
        _check(lib().tenom_batch_set_tile(self._h, int(t)))

    def rk3(self, U, scheme, limiter, C_T, gamma, cfl, steps=1, first=0, count=None, stream=None):
        """Enqueue `steps` RK3 steps of problems [first, first + count)."""
        count = self.count - first if count is None else count
        _check(lib().tenom_batch_rk3(self._h, scheme, limiter, C_T, gamma, cfl, int(steps), int(first), int(count),
                                     self._state(U), _stream(stream)))
        return U

    def rk3_graph(self, U, scheme, limiter, C_T, gamma, cfl, steps=1, stream=None):
        """`steps` RK3 steps of every problem as one captured-graph launch."""
        _check(lib().tenom_batch_rk3_graph(self._h, scheme, limiter, C_T, gamma, cfl, int(steps),
                                           self._state(U), _stream(stream)))
        return U

    def rk3_persistent(self, U, scheme, limiter, C_T, gamma, cfl, steps=1, stream=None):
        """`steps` RK3 steps of every problem in one persistent kernel launch."""
        _check(lib().tenom_batch_rk3_persistent(self._h, scheme, limiter, C_T, gamma, cfl, int(steps),
                                                self._state(U), _stream(stream)))
        return U

    def autotune(self, U, scheme, limiter, C_T, gamma, cfl, steps=2, stream=None):
        """Time every tile shape; select the fastest.  Returns (tile, ms/step per tile)."""
        ms = (C.c_float * BATCH_TILES)()
        best = C.c_int()
        _check(lib().tenom_batch_autotune(self._h, scheme, limiter, C_T, gamma, cfl, self._state(U), int(steps),
                                          ms, C.byref(best), _stream(stream)))
        return best.value, [float(v) for v in ms]

    def times(self, stream=None):
        """(clock, last step) of every problem as numpy arrays (synchronises)."""
        import numpy as np
        t = np.zeros(self.count)
        dt = np.zeros(self.count)
        _check(lib().tenom_batch_times(self._h, t.ctypes.data_as(C.POINTER(C.c_double)),
                                       dt.ctypes.data_as(C.POINTER(C.c_double)), _stream(stream)))
        return t, dt

    def reset_times(self, stream=None):
        _check(lib().tenom_batch_reset_times(self._h, _stream(stream)))


# ---------------------------------------------------------------------------
# adjoint
# ---------------------------------------------------------------------------

class _Buffer:
    """Device workspace owned by a torch uint8 tensor (256-byte aligned)."""

    def __init__(self, nbytes: int, device):
        import torch
        if nbytes == 0:
            raise TenomError(EINVAL, "invalid grid or scheme for a workspace")
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.nbytes = nbytes

    @property
    def ptr(self):
        return C.c_void_p(self.buf.data_ptr())


def vjp_workspace(grid, scheme: int, device="cuda") -> _Buffer:
    g = Grid.of(grid).to_c()
    return _Buffer(int(lib().tenom_vjp_workspace_bytes(C.byref(g), scheme)), device)


def rk3_vjp_workspace(grid, scheme: int, device="cuda") -> _Buffer:
    g = Grid.of(grid).to_c()
    return _Buffer(int(lib().tenom_rk3_vjp_workspace_bytes(C.byref(g), scheme)), device)


def flux_divergence_vjp(U, Lbar, grid, scheme: int, limiter: int, C_T: float, gamma: float, out=None,
                        scale: float = 1.0, accumulate: bool = False, workspace=None, stream=None):
    """out (+)= scale * (dL/dU)^T Lbar for L = flux_divergence; returns out."""
    import torch
    g = Grid.of(grid)
    up, lp = _state(U, g), _state(Lbar, g, "Lbar")
    if out is None:
        out = torch.empty_like(U)
        accumulate = False
    op = _state(out, g, "out")
    ws = workspace if workspace is not None else vjp_workspace(g, scheme, U.device)
    gc = g.to_c()
    _check(lib().tenom_flux_divergence_vjp(C.byref(gc), scheme, limiter, C_T, gamma, up, lp, float(scale), op,
                                           1 if accumulate else 0, ws.ptr, ws.nbytes, _stream(stream)))
    return out


def rk3_step_vjp(U, Ubar, grid, scheme: int, limiter: int, C_T: float, gamma: float, dt: float, workspace=None,
                 stream=None, stages=None):
    """Ubar <- (d step(U) / d U)^T Ubar, in place; U is the step's input.
    stages = (U1, U2): the step's stage states as rk3_step(stages=...) wrote
    them (tenom_rk3_step_vjp_stages); otherwise they are recomputed."""
    g = Grid.of(grid)
    up, bp = _state(U, g), _state(Ubar, g, "Ubar")
    ws = workspace if workspace is not None else rk3_vjp_workspace(g, scheme, U.device)
    gc = g.to_c()
    if stages is None:
        _check(lib().tenom_rk3_step_vjp(C.byref(gc), scheme, limiter, C_T, gamma, dt, up, bp, ws.ptr, ws.nbytes,
                                        _stream(stream)))
    else:
        p1, p2 = _state(stages[0], g, "U1"), _state(stages[1], g, "U2")
        _check(lib().tenom_rk3_step_vjp_stages(C.byref(gc), scheme, limiter, C_T, gamma, dt, up, p1, p2, bp,
                                               ws.ptr, ws.nbytes, _stream(stream)))
    return Ubar


def _rollout_forward(U0, g, scheme, limiter, C_T, gamma, dt, steps, checkpoint, ws):
    U = U0.detach().clone()
    saved = []
    for s in range(steps):
        if s % checkpoint == 0:
            saved.append(U.clone())
        rk3_step(U, g, scheme, limiter, C_T, gamma, dt, workspace=ws)
    return U, saved


class Rk3Rollout:
    """`steps` SSP-RK3 steps of fixed size dt as a differentiable torch op.

    The forward keeps the state every `checkpoint` steps; the backward
    replays each segment from its checkpoint (the same kernels, so the same
    decisions), keeping each step's input and stage states, and applies
    tenom_rk3_step_vjp_stages in reverse order.  Memory: steps/checkpoint +
    3 checkpoint states."""

    @staticmethod
    def apply(U0, grid, scheme, limiter, C_T, gamma, dt, steps, checkpoint=20):
        import torch

        class _Fn(torch.autograd.Function):
            @staticmethod
            def forward(ctx, U0_):
                g = Grid.of(grid)
                ws = Workspace(g, scheme, U0_.device)
                U, saved = _rollout_forward(U0_, g, scheme, limiter, C_T, gamma, dt, steps, checkpoint, ws)
                ctx.saved = saved
                return U

            @staticmethod
            def backward(ctx, Ubar):
                g = Grid.of(grid)
                ws = Workspace(g, scheme, Ubar.device)
                vws = rk3_vjp_workspace(g, scheme, Ubar.device)
                lam = Ubar.detach().clone().contiguous()
                nseg = len(ctx.saved)
                for k in range(nseg - 1, -1, -1):
                    first = k * checkpoint
                    last = min(steps, first + checkpoint)
                    # replay the segment, keeping every step's input and stage states
                    steps_kept = []
                    V = ctx.saved[k]
                    for _ in range(first, last):
                        W = V.clone()
                        S1, S2 = torch.empty_like(V), torch.empty_like(V)
                        rk3_step(W, g, scheme, limiter, C_T, gamma, dt, workspace=ws, stages=(S1, S2))
                        steps_kept.append((V, S1, S2))
                        V = W
                    for V, S1, S2 in reversed(steps_kept):
                        rk3_step_vjp(V, lam, g, scheme, limiter, C_T, gamma, dt, workspace=vws, stages=(S1, S2))
                    del steps_kept
                ctx.saved = None
                return lam

        return _Fn.apply(U0)


def rollout_flags(U0, grid, scheme: int, limiter: int, C_T: float, gamma: float, dt: float, steps: int,
                  ref=None):
    """Smoothness flags of every stage and axis of a `steps`-step fixed-dt
    rollout from U0 (U0 is left untouched): a list of [2, nf, faces...]
    uint8 tensors in the order step, stage, axis.  With ref (the list of a
    previous call) it returns instead whether every flag equals ref's, e.g.
    to tell whether a perturbed rollout takes the same decisions."""
    import torch
    g = Grid.of(grid)
    U = U0.detach().clone().contiguous()
    U1, U2 = torch.empty_like(U), torch.empty_like(U)
    ws = Workspace(g, scheme, U.device)
    out, k = [], 0
    for _ in range(steps):
        stage_in = U.clone()
        rk3_step(U, g, scheme, limiter, C_T, gamma, dt, workspace=ws, stages=(U1, U2))
        for S in (stage_in, U1, U2):
            for axis in range(g.ndim):
                _, fl = reconstruct_faces(S, g, scheme, limiter, C_T, gamma, axis, return_flags=True)
                if ref is None:
                    out.append(fl)
                elif not torch.equal(fl, ref[k]):
                    return False
                k += 1
    return out if ref is None else True


def rollout(U0, grid, scheme: int, limiter: int, C_T: float, gamma: float, dt: float, steps: int,
            checkpoint: int = 20):
    """Differentiable `steps`-step rollout (see Rk3Rollout)."""
    return Rk3Rollout.apply(U0, grid, scheme, limiter, C_T, gamma, dt, steps, checkpoint)
