"""The C-ABI library without a GPU: it loads, exports every symbol the
header declares, and rejects bad arguments before touching the device."""
import ctypes as C
import os
import re

import pytest

import paper_2010_13289_amd as T

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tenom.h")


def declared_symbols():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tenom_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(T.LIB_PATH):
        T.build_library()
    return T.lib()


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ("tenom_reconstruct_faces", "tenom_flux_divergence", "tenom_rk3_step"):
        assert name in syms
    assert set(syms) == set(T.SYMBOLS)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_symbols():
        assert hasattr(lib, name), name
    assert lib.tenom_version() == 10000


def grid(**kw):
    g = dict(ndim=3, n=[16, 16, 16], dx=[0.1, 0.1, 0.1], bc=[0, 0, 0], system=1, adv=[0, 0, 0])
    g.update(kw)
    return T.Grid.of(g).to_c()


DUMMY = C.c_void_p(0x1000)  # never dereferenced: every call below fails validation


@pytest.mark.parametrize("kw,scheme,lim,ct,gam,code", [
    (dict(ndim=0), 6, 1, 1e-5, 1.4, T.EINVAL),
    (dict(ndim=4), 6, 1, 1e-5, 1.4, T.EINVAL),
    (dict(n=[5, 16, 16]), 6, 1, 1e-5, 1.4, T.EINVAL),   # fewer than K cells
    (dict(n=[16, 7, 16]), 8, 1, 1e-5, 1.4, T.EINVAL),
    (dict(dx=[0.1, -1.0, 0.1]), 6, 1, 1e-5, 1.4, T.EINVAL),
    (dict(bc=[0, 2, 0]), 6, 1, 1e-5, 1.4, T.EINVAL),
    (dict(system=7), 6, 1, 1e-5, 1.4, T.EUNSUPPORTED),
    ({}, 7, 1, 1e-5, 1.4, T.EUNSUPPORTED),
    ({}, 6, 99, 1e-5, 1.4, T.EUNSUPPORTED),
    ({}, 6, 1, -1e-5, 1.4, T.EINVAL),
    ({}, 6, 1, float("nan"), 1.4, T.EINVAL),
    ({}, 6, 1, 1e-5, 1.0, T.EINVAL),
    ({}, 6, 1, 1e-5, float("inf"), T.EINVAL),
])
def test_argument_errors(lib, kw, scheme, lim, ct, gam, code):
    g = grid(**kw)
    rc = lib.tenom_reconstruct_faces(C.byref(g), scheme, lim, ct, gam, 0, DUMMY, DUMMY, None, None)
    assert rc == code
    assert lib.tenom_last_error().decode()
    rc = lib.tenom_flux_divergence(C.byref(g), scheme, lim, ct, gam, DUMMY, C.c_void_p(0x2000), None)
    assert rc == code


def test_pointer_and_axis_errors(lib):
    g = grid()
    assert lib.tenom_reconstruct_faces(C.byref(g), 6, 1, 1e-5, 1.4, 0, None, DUMMY, None, None) == T.EINVAL
    assert lib.tenom_reconstruct_faces(C.byref(g), 6, 1, 1e-5, 1.4, 3, DUMMY, DUMMY, None, None) == T.EINVAL
    assert lib.tenom_reconstruct_faces(None, 6, 1, 1e-5, 1.4, 0, DUMMY, DUMMY, None, None) == T.EINVAL
    assert lib.tenom_flux_divergence(C.byref(g), 6, 1, 1e-5, 1.4, DUMMY, DUMMY, None) == T.EINVAL  # alias


def test_rk3_workspace_and_dt_errors(lib):
    g = grid()
    need = lib.tenom_workspace_bytes(C.byref(g), 6)
    # three states, then the step-size tail: 4096 per-block maxima and dt, 256-byte aligned
    assert need == 3 * 5 * 16 ** 3 * 8 + 33024
    ws = C.c_void_p(0x10000)
    assert lib.tenom_rk3_step(C.byref(g), 6, 1, 1e-5, 1.4, 0.01, DUMMY, ws, need - 1, None) == T.EWORKSPACE
    assert lib.tenom_rk3_step(C.byref(g), 6, 1, 1e-5, 1.4, 0.0, DUMMY, ws, need, None) == T.EINVAL
    assert lib.tenom_rk3_step(C.byref(g), 6, 1, 1e-5, 1.4, float("nan"), DUMMY, ws, need, None) == T.EINVAL
    assert lib.tenom_rk3_step(C.byref(g), 6, 1, 1e-5, 1.4, 0.01, DUMMY, C.c_void_p(0x10008), need, None) == T.EINVAL
    assert lib.tenom_rk3_step(C.byref(g), 6, 1, 1e-5, 1.4, 0.01, DUMMY, None, need, None) == T.EINVAL
    assert lib.tenom_workspace_bytes(C.byref(grid(ndim=0)), 6) == 0


def test_stage_entry_errors(lib):
    """tenom_rk3_step_stages / tenom_rk3_step_vjp_stages reject missing or
    aliased stage arrays before touching memory."""
    g = grid()
    need = lib.tenom_workspace_bytes(C.byref(g), 6)
    ws = C.c_void_p(0x10000)
    U1, U2 = C.c_void_p(0x3000), C.c_void_p(0x4000)
    step = lib.tenom_rk3_step_stages
    assert step(C.byref(g), 6, 1, 1e-5, 1.4, 0.01, DUMMY, None, U2, ws, need, None) == T.EINVAL
    assert step(C.byref(g), 6, 1, 1e-5, 1.4, 0.01, DUMMY, DUMMY, U2, ws, need, None) == T.EINVAL
    assert step(C.byref(g), 6, 1, 1e-5, 1.4, 0.01, DUMMY, U1, U1, ws, need, None) == T.EINVAL
    assert step(C.byref(g), 6, 1, 1e-5, 1.4, 0.01, DUMMY, U1, U2, ws, need - 1, None) == T.EWORKSPACE
    vneed = lib.tenom_rk3_vjp_workspace_bytes(C.byref(g), 6)
    vjp = lib.tenom_rk3_step_vjp_stages
    Ub = C.c_void_p(0x5000)
    assert vjp(C.byref(g), 6, 1, 1e-5, 1.4, 0.01, DUMMY, None, U2, Ub, ws, vneed, None) == T.EINVAL
    assert vjp(C.byref(g), 6, 1, 1e-5, 1.4, 0.01, DUMMY, U1, U2, U1, ws, vneed, None) == T.EINVAL
    assert vjp(C.byref(g), 6, 1, 1e-5, 1.4, 0.01, DUMMY, U1, U2, DUMMY, ws, vneed, None) == T.EINVAL
    assert vjp(C.byref(g), 6, 1, 1e-5, 1.4, 0.01, DUMMY, U1, U2, Ub, ws, vneed - 1, None) == T.EWORKSPACE


def test_cfl_step_errors(lib):
    """tenom_rk3_step_cfl rejects a bad CFL number, missing pointers and a
    short workspace before any launch; its workspace is tenom_rk3_step's,
    which holds three states and the step-size tail."""
    g = grid()
    need = lib.tenom_workspace_bytes(C.byref(g), 6)
    ws = C.c_void_p(0x10000)
    step = lib.tenom_rk3_step_cfl
    for cfl in (0.0, -0.4, float("nan"), float("inf")):
        assert step(C.byref(g), 6, 1, 1e-5, 1.4, cfl, DUMMY, ws, need, None, None) == T.EINVAL, cfl
    assert step(C.byref(g), 6, 1, 1e-5, 1.4, 0.4, None, ws, need, None, None) == T.EINVAL
    assert step(C.byref(g), 6, 1, 1e-5, 1.4, 0.4, DUMMY, None, need, None, None) == T.EINVAL
    assert step(C.byref(g), 6, 1, 1e-5, 1.4, 0.4, DUMMY, C.c_void_p(0x10008), need, None, None) == T.EINVAL
    assert step(C.byref(g), 6, 1, 1e-5, 1.4, 0.4, DUMMY, ws, need - 1, None, None) == T.EWORKSPACE
    assert step(C.byref(g), 6, 9, 1e-5, 1.4, 0.4, DUMMY, ws, need, None, None) == T.EUNSUPPORTED


def test_noalloc_step_rejects_oversized_grids_before_touching_the_device(lib):
    """The allocation-free step checks the grid's scratch need against its
    static array first: a 128^3 Euler grid needs 3 states (252 MB) and is
    refused without any HIP call."""
    assert lib.tenom_static_scratch_bytes() == 128 << 20
    g = grid(n=[128, 128, 128])
    assert lib.tenom_workspace_bytes(C.byref(g), 6) > lib.tenom_static_scratch_bytes()
    rc = lib.tenom_rk3_step_cfl_noalloc(C.byref(g), 6, 1, 1e-5, 1.4, 0.4, DUMMY, None, None)
    assert rc == T.EWORKSPACE
    assert b"static scratch" in lib.tenom_last_error()


def test_scheme_and_limiter_ids(lib):
    g = grid()
    bad = C.c_void_p(0x2000)
    # unknown scheme bits, adaptive with K = 6, unknown limiter
    for scheme, lim in ((6 | 0x200, 1), (6 | 0x100, 1), (8, 9), (8, -1)):
        rc = lib.tenom_reconstruct_faces(C.byref(g), scheme, lim, 1e-5, 1.4, 0, DUMMY, bad, None, None)
        assert rc == T.EUNSUPPORTED, (scheme, lim)
    # classic TENO keeps a candidate only for C_T <= 1/(K-2)
    # (scheme and limiter arguments are checked before the pointers)
    rc = lib.tenom_flux_divergence(C.byref(g), 6, T.LIM_TENO, 0.3, 1.4, None, bad, None)
    assert rc == T.EINVAL and "C_T" in lib.tenom_last_error().decode()
    # the adaptive scheme ignores C_T, so even a negative one is accepted (NULL U fails later)
    rc = lib.tenom_flux_divergence(C.byref(g), T.SCHEME_8A, T.LIM_MP, -1.0, 1.4, None, bad, None)
    assert rc == T.EINVAL and "NULL" in lib.tenom_last_error().decode()
    assert lib.tenom_workspace_bytes(C.byref(g), T.SCHEME_8A) == lib.tenom_workspace_bytes(C.byref(g), 8)
    assert lib.tenom_workspace_bytes(C.byref(g), 6 | 0x100) == 0


def test_sweep_kernel_choice(lib):
    """0 automatic, 1 march, 2 tile; anything else is rejected and leaves
    the setting as it was (no device is touched)."""
    for bad in (-1, 3, 99):
        assert lib.tenom_set_sweep_kernel(bad) == -1
    for ok in (1, 2, 0):
        assert lib.tenom_set_sweep_kernel(ok) == 0


def test_strerror_and_fields(lib):
    for code in (0, -1, -2, -3, -4, -5, -77):
        assert lib.tenom_strerror(code)
    assert lib.tenom_num_fields(C.byref(grid())) == 5
    assert lib.tenom_num_fields(C.byref(grid(ndim=2))) == 4
    assert lib.tenom_num_fields(C.byref(grid(system=0))) == 1


def test_batch_arguments_fail_before_allocation(lib):
    """tenom_batch_create checks its arguments before touching the device."""
    plan = C.c_void_p()
    n = (C.c_int64 * 3)(64, 5, 64)
    dx = (C.c_double * 3)(0.1, 0.1, 0.1)
    assert lib.tenom_batch_create(3, n, dx, 1, C.byref(plan)) == T.EINVAL  # 5 < 6 cells
    assert "fewer than 6" in lib.tenom_last_error().decode()
    n[1] = 64
    dx[2] = 0.0
    assert lib.tenom_batch_create(3, n, dx, 1, C.byref(plan)) == T.EINVAL
    dx[2] = float("inf")
    assert lib.tenom_batch_create(3, n, dx, 1, C.byref(plan)) == T.EINVAL
    dx[2] = 0.1
    assert lib.tenom_batch_create(3, n, dx, 2, C.byref(plan)) == T.EINVAL  # boundary rule
    assert lib.tenom_batch_create(-1, n, dx, 1, C.byref(plan)) == T.EINVAL
    assert lib.tenom_batch_create(3, None, dx, 1, C.byref(plan)) == T.EINVAL
    assert lib.tenom_batch_create(3, n, dx, 1, None) == T.EINVAL
    assert plan.value is None
    # calls on a NULL plan
    assert lib.tenom_batch_rk3(None, 8, 1, 1e-7, 1.4, 0.4, 1, 0, 1, DUMMY, None) == T.EINVAL
    assert lib.tenom_batch_rk3_graph(None, 8, 1, 1e-7, 1.4, 0.4, 1, DUMMY, None) == T.EINVAL
    assert lib.tenom_batch_cells(None) == -1
    assert lib.tenom_batch_get_tile(None) == -1
    assert lib.tenom_batch_destroy(None) == T.OK


def test_batch_tile_shapes(lib):
    shapes = [T.batch_tile_shape(t) for t in range(T.BATCH_TILES)]
    assert len(set(shapes)) == T.BATCH_TILES
    for threads, fpt in shapes:
        assert threads % 64 == 0 and fpt >= 1  # whole wavefronts
    with pytest.raises(T.TenomError):
        T.batch_tile_shape(T.BATCH_TILES)


def test_missing_library_raises(monkeypatch):
    """Without libtenom.so the binding raises instead of computing anything
    another way (there is no fallback path)."""
    monkeypatch.setattr(T, "_lib", None)
    monkeypatch.setattr(T, "LIB_PATH", os.path.join(os.path.dirname(T.LIB_PATH), "no_such_libtenom.so"))
    with pytest.raises(ImportError, match="missing"):
        T.lib()
