"""CPU oracle of the TENO-M reconstruction path (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  It wraps ``libtenom_oracle.so``, built
from ``tenom_oracle.c`` by :func:`build`, with ctypes, and adds the exact
Riemann solver used to check shock-tube runs (``oracle.exact_riemann``).
It shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tenom_oracle.c")
_LIB = os.path.join(_HERE, "libtenom_oracle.so")

# limiter numbering of the oracle (its own; equal to the C-ABI's by design of
# the tests, which pass the same integers to both sides)
LIM_TENO, LIM_MP, LIM_TVD_MINMOD, LIM_TVD5, LIM_VA = 0, 1, 2, 3, 4
LIM_MP_M4_B2, LIM_MP_MM_B4, LIM_MP_MM_B2, LIM_MP_MM_B1 = 5, 6, 7, 8
SCHEME_ADAPTIVE = 0x100           # or-ed into K = 8: the adaptive cutoff (TENO8A)
SCHEME_8A = 8 | SCHEME_ADAPTIVE


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
               "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Grid(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("n", C.c_int32 * 3), ("dx", C.c_double * 3),
                ("bc", C.c_int32 * 3), ("system", C.c_int32), ("adv", C.c_double * 3)]


class Trace(C.Structure):
    _fields_ = [("cand", C.c_double * 6), ("beta", C.c_double * 6), ("betaK", C.c_double),
                ("tau", C.c_double), ("gam", C.c_double * 6), ("chi", C.c_double * 6),
                ("delta", C.c_int * 6), ("band", C.c_int * 6), ("fmin", C.c_double),
                ("fmax", C.c_double), ("ftvd", C.c_double), ("fM", C.c_double * 6),
                ("out", C.c_double), ("eta", C.c_double), ("m", C.c_double), ("ct", C.c_double),
                ("ct_band", C.c_int), ("status", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        dp, u8p, lp = C.POINTER(C.c_double), C.POINTER(C.c_uint8), C.POINTER(C.c_long)
        gp = C.POINTER(_Grid)
        L.or_init.restype = C.c_int
        L.or_param.argtypes = [C.c_char_p]
        L.or_param.restype = C.c_double
        L.or_get_weights.argtypes = [C.c_int, dp]
        L.or_get_poly_face.argtypes = [C.c_int, C.c_int, dp]
        L.or_beta_stencil.argtypes = [C.c_int, C.c_int, dp]
        L.or_beta_stencil.restype = C.c_double
        for name in ("or_minmod2",):
            getattr(L, name).argtypes = [C.c_double] * 2
            getattr(L, name).restype = C.c_double
        L.or_minmod4.argtypes = [C.c_double] * 4
        L.or_minmod4.restype = C.c_double
        L.or_median.argtypes = [C.c_double] * 3
        L.or_median.restype = C.c_double
        L.or_mp_bounds.argtypes = [C.c_double] * 5 + [C.c_int, C.c_double, dp, dp]
        L.or_tvd_minmod.argtypes = [C.c_double] * 3
        L.or_tvd_minmod.restype = C.c_double
        L.or_tvd5.argtypes = [C.c_double] * 5
        L.or_tvd5.restype = C.c_double
        L.or_van_albada.argtypes = [C.c_double] * 3
        L.or_van_albada.restype = C.c_double
        L.or_teno_m.argtypes = [C.c_int, C.c_int, C.c_double, dp, C.POINTER(Trace)]
        L.or_teno_m.restype = C.c_double
        L.or_trace_size.restype = C.c_int
        L.or_roe_eigenvectors.argtypes = [C.c_int, C.c_double, C.c_int, dp, dp, dp, dp]
        L.or_reconstruct_faces.argtypes = [gp, C.c_int, C.c_int, C.c_double, C.c_double, C.c_int,
                                           dp, dp, u8p, u8p]
        L.or_flux_divergence.argtypes = [gp, C.c_int, C.c_int, C.c_double, C.c_double, dp, dp]
        L.or_rk3_step.argtypes = [gp, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, dp]
        L.or_faces_points.argtypes = [gp, C.c_int, C.c_int, C.c_double, C.c_double, C.c_int, dp,
                                      C.c_long, lp, dp, u8p, u8p]
        L.or_dudt_points.argtypes = [gp, C.c_int, C.c_int, C.c_double, C.c_double, dp, C.c_long,
                                     lp, dp, lp]
        L.or_rk3_points.argtypes = [gp, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, dp,
                                    C.c_long, lp, dp, lp]
        L.or_max_wave_speed.argtypes = [gp, C.c_double, dp]
        L.or_max_wave_speed.restype = C.c_double
        L.or_num_threads.restype = C.c_int
        L.or_set_num_threads.argtypes = [C.c_int]
        if C.sizeof(Trace) != L.or_trace_size():
            raise RuntimeError("oracle trace layout mismatch")
        if L.or_init() != 0:
            raise RuntimeError("oracle initialisation failed")
        _lib = L
    return _lib


# ---------------------------------------------------------------------------
# helpers
# ---------------------------------------------------------------------------

def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _u8p(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_uint8))


def _lp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_long))


def _grid(grid) -> _Grid:
    """grid: dict with ndim, n (x, y, z order), dx, bc, system, adv."""
    g = _Grid()
    nd = int(grid["ndim"])
    g.ndim = nd
    n = list(grid["n"]) + [1] * (3 - len(grid["n"]))
    dx = list(grid.get("dx", [1.0] * nd)) + [1.0] * (3 - len(grid.get("dx", [1.0] * nd)))
    bc = list(grid.get("bc", [0] * nd)) + [0] * (3 - len(grid.get("bc", [0] * nd)))
    adv = list(grid.get("adv", [0.0] * nd)) + [0.0] * (3 - len(grid.get("adv", [0.0] * nd)))
    for d in range(3):
        g.n[d] = int(n[d]) if d < nd else 1
        g.dx[d] = float(dx[d])
        g.bc[d] = int(bc[d])
        g.adv[d] = float(adv[d])
    g.system = int(grid.get("system", 1))
    return g


def nfields(grid) -> int:
    return 1 if int(grid.get("system", 1)) == 0 else int(grid["ndim"]) + 2


def face_shape(grid, axis):
    """Array shape (z, y, x order) of the faces of `axis` (x = 0)."""
    nd = int(grid["ndim"])
    n = [int(v) for v in grid["n"][:nd]]
    n[axis] += 1
    return tuple(reversed(n))


def _state(U, grid):
    U = np.ascontiguousarray(U, dtype=np.float64)
    nd = int(grid["ndim"])
    expect = (nfields(grid),) + tuple(reversed([int(v) for v in grid["n"][:nd]]))
    if U.shape != expect:
        raise ValueError(f"state shape {U.shape} != {expect}")
    return U


ENONFINITE = -5  # a sum of gamma_k overflowed (Eq. normalize undefined)


class NonFiniteIndicator(RuntimeError):
    """The literal gamma_k of Eq. measureTENO overflowed somewhere."""


def _chk(rc, what):
    if rc == ENONFINITE:
        raise NonFiniteIndicator(f"oracle {what}: the sum of gamma_k is not finite")
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with {rc}")


def param(name: str) -> float:
    """A constant the oracle uses, by the name of the paper's parameter
    (C, q, epsilon, mp_alpha, mp_beta, tvd5_alpha, va_kappa, ren_xi, ren_cr,
    adapt_alpha1, adapt_alpha2); NaN for an unknown name."""
    return lib().or_param(name.encode())


# ---------------------------------------------------------------------------
# per-face scalar reconstruction and its building blocks
# ---------------------------------------------------------------------------

def teno_m(K: int, lim: int, C_T: float, v) -> tuple[float, Trace]:
    """One TENO-M reconstruction at x_{i+1/2} from v = f_{i-K/2+1..i+K/2}.
    K may carry SCHEME_ADAPTIVE (TENO8A: C_T from Sec. 2.4, argument ignored)."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    assert v.shape == (K & 0xFF,)
    tr = Trace()
    out = lib().or_teno_m(K, lim, C_T, _dp(v), C.byref(tr))
    return out, tr


def weights(K: int) -> np.ndarray:
    d = np.zeros(K - 2)
    _chk(lib().or_get_weights(K, _dp(d)), "weights")
    return d


def poly_face(lo: int, hi: int) -> np.ndarray:
    c = np.zeros(hi - lo + 1)
    _chk(lib().or_get_poly_face(lo, hi, _dp(c)), "poly_face")
    return c


def beta(lo: int, hi: int, vs) -> float:
    vs = np.ascontiguousarray(vs, dtype=np.float64)
    return lib().or_beta_stencil(lo, hi, _dp(vs))


def minmod2(x, y):
    return lib().or_minmod2(float(x), float(y))


def minmod4(a, b, c, d):
    return lib().or_minmod4(float(a), float(b), float(c), float(d))


def median(x, y, z):
    return lib().or_median(float(x), float(y), float(z))


def mp_bounds(f, curv: int = 0, bet: float = 4.0):
    lo, hi = C.c_double(), C.c_double()
    lib().or_mp_bounds(*[float(t) for t in f], curv, bet, C.byref(lo), C.byref(hi))
    return lo.value, hi.value


def tvd_minmod(fm1, f0, fp1):
    return lib().or_tvd_minmod(float(fm1), float(f0), float(fp1))


def tvd5(f):
    return lib().or_tvd5(*[float(t) for t in f])


def van_albada(fm1, f0, fp1):
    return lib().or_van_albada(float(fm1), float(f0), float(fp1))


def roe_eigenvectors(ndim, gamma, axis, UL, UR):
    nf = ndim + 2
    UL = np.ascontiguousarray(UL, dtype=np.float64)
    UR = np.ascontiguousarray(UR, dtype=np.float64)
    R = np.zeros((nf, nf))
    L = np.zeros((nf, nf))
    _chk(lib().or_roe_eigenvectors(ndim, gamma, axis, _dp(UL), _dp(UR), _dp(R), _dp(L)), "roe")
    return R, L


# ---------------------------------------------------------------------------
# whole-grid and sampled entry points
# ---------------------------------------------------------------------------

def reconstruct_faces(U, grid, scheme, limiter, C_T, gamma, axis, with_flags=True):
    """Returns (Fhat, flags, band); flags/band are [2][nf][faces] uint8."""
    U = _state(U, grid)
    nf = nfields(grid)
    fs = face_shape(grid, axis)
    F = np.zeros((nf,) + fs)
    fl = np.zeros((2, nf) + fs, dtype=np.uint8) if with_flags else None
    bd = np.zeros((2, nf) + fs, dtype=np.uint8) if with_flags else None
    g = _grid(grid)
    _chk(lib().or_reconstruct_faces(C.byref(g), scheme, limiter, C_T, gamma, axis, _dp(U), _dp(F),
                                    _u8p(fl), _u8p(bd)), "reconstruct_faces")
    return F, fl, bd


def flux_divergence(U, grid, scheme, limiter, C_T, gamma):
    U = _state(U, grid)
    out = np.zeros_like(U)
    g = _grid(grid)
    _chk(lib().or_flux_divergence(C.byref(g), scheme, limiter, C_T, gamma, _dp(U), _dp(out)),
         "flux_divergence")
    return out


def rk3_step(U, grid, scheme, limiter, C_T, gamma, dt):
    """Returns the state after one SSP-RK3 step (input left untouched)."""
    out = _state(U, grid).copy()
    g = _grid(grid)
    _chk(lib().or_rk3_step(C.byref(g), scheme, limiter, C_T, gamma, dt, _dp(out)), "rk3_step")
    return out


def faces_points(U, grid, scheme, limiter, C_T, gamma, axis, face_idx):
    """Face fluxes at flat face indices: (F[npts][nf], flags[npts][2nf], band[npts][2nf])."""
    U = _state(U, grid)
    idx = np.ascontiguousarray(face_idx, dtype=np.int64)
    nf = nfields(grid)
    out = np.zeros((len(idx), nf))
    fl = np.zeros((len(idx), 2 * nf), dtype=np.uint8)
    bd = np.zeros((len(idx), 2 * nf), dtype=np.uint8)
    g = _grid(grid)
    _chk(lib().or_faces_points(C.byref(g), scheme, limiter, C_T, gamma, axis, _dp(U), len(idx),
                               _lp(idx), _dp(out), _u8p(fl), _u8p(bd)), "faces_points")
    return out, fl, bd


def dudt_points(U, grid, scheme, limiter, C_T, gamma, cell_idx):
    U = _state(U, grid)
    idx = np.ascontiguousarray(cell_idx, dtype=np.int64)
    out = np.zeros((len(idx), nfields(grid)))
    bh = np.zeros(len(idx), dtype=np.int64)
    g = _grid(grid)
    _chk(lib().or_dudt_points(C.byref(g), scheme, limiter, C_T, gamma, _dp(U), len(idx), _lp(idx),
                              _dp(out), _lp(bh)), "dudt_points")
    return out, bh


def rk3_points(U, grid, scheme, limiter, C_T, gamma, dt, cell_idx):
    """One RK3 step at flat cell indices: (U_new[npts][nf], bandhits[npts])."""
    U = _state(U, grid)
    idx = np.ascontiguousarray(cell_idx, dtype=np.int64)
    out = np.zeros((len(idx), nfields(grid)))
    bh = np.zeros(len(idx), dtype=np.int64)
    g = _grid(grid)
    _chk(lib().or_rk3_points(C.byref(g), scheme, limiter, C_T, gamma, dt, _dp(U), len(idx), _lp(idx),
                             _dp(out), _lp(bh)), "rk3_points")
    return out, bh


def max_wave_speed(U, grid, gamma):
    U = _state(U, grid)
    g = _grid(grid)
    return lib().or_max_wave_speed(C.byref(g), gamma, _dp(U))


def num_threads() -> int:
    return lib().or_num_threads()


def set_num_threads(n: int) -> None:
    """OpenMP threads of the oracle's parallel loops from now on."""
    lib().or_set_num_threads(int(n))
