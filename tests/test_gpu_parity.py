"""GPU parity: the HIP path through the C ABI against the oracle, element by
element, on seeded inputs that span several workgroup tiles and ragged
tails, every system, both schemes, every limiter and both boundary rules.
Bar: 1e-12 of the field's largest magnitude, flags bit-identical, both
outside the cutoff band (see tests/parity.py)."""
import numpy as np
import pytest

import workloads as W
from parity import (assert_close_fields, band_faces, faces_to_cells, require_gpu, to_dev, to_host)

pytestmark = pytest.mark.gpu

GAMMA = 1.4

# name, shape (z, y, x order), system, bc (x, y, z order), K, limiter, C_T, adv
CASES = [
    ("scalar1d_mp6", (200,), 0, [0], 6, 1, 1e-5, [1.0]),
    ("scalar1d_neg_tvd8", (301,), 0, [1], 8, 2, 1e-7, [-0.7]),
    ("scalar2d_tvd5", (20, 70), 0, [0, 1], 6, 3, 1e-5, [0.5, -1.2]),
    ("scalar3d_mp8", (9, 12, 40), 0, [0, 0, 1], 8, 1, 1e-6, [0.3, 1.0, -0.4]),
    ("euler1d_mp6_per", (300,), 1, [0], 6, 1, 1e-5, None),
    ("euler1d_tvd8_trans", (257,), 1, [1], 8, 2, 1e-7, None),
    ("euler1d_tvd5_8", (600,), 1, [0], 8, 3, 1e-7, None),
    ("euler1d_mp8_trans256", (256,), 1, [1], 8, 1, 1e-7, None),
    ("euler2d_mp6", (37, 70), 1, [0, 1], 6, 1, 1e-5, None),
    ("euler2d_tvd5_8", (33, 65), 1, [1, 0], 8, 3, 1e-6, None),
    ("euler2d_tvdmm_6", (40, 129), 1, [0, 0], 6, 2, 1e-5, None),
    ("euler3d_mp6", (18, 20, 33), 1, [0, 0, 0], 6, 1, 1e-5, None),
    ("euler3d_tvd8", (12, 17, 70), 1, [1, 0, 1], 8, 2, 1e-7, None),
    ("euler3d_tvd5_6", (9, 10, 66), 1, [0, 1, 0], 6, 3, 1e-4, None),
    ("euler3d_mp8_long_z", (80, 8, 16), 1, [0, 0, 0], 8, 1, 1e-7, None),
    ("min_size_6", (6,), 1, [0], 6, 1, 1e-5, None),
    ("min_size_8_trans", (8,), 1, [1], 8, 1, 1e-7, None),
    ("min_size_3d_6", (6, 6, 6), 1, [0, 0, 0], 6, 1, 1e-5, None),
    ("min_size_3d_8_mixed", (8, 8, 8), 1, [1, 0, 1], 8, 1, 1e-7, None),
    # limiter variants (Secs. 3.2.1, 4.2.5, 4.4) and classic renormalised TENO
    ("euler1d_va6", (300,), 1, [1], 6, 4, 1e-5, None),
    ("euler2d_va8", (21, 40), 1, [0, 1], 8, 4, 1e-6, None),
    ("euler1d_mp_m4_b2", (260,), 1, [0], 6, 5, 1e-5, None),
    ("euler2d_mp_mm_b4", (19, 44), 1, [1, 0], 8, 6, 1e-6, None),
    ("euler3d_mp_mm_b2", (10, 12, 36), 1, [0, 0, 1], 6, 7, 1e-5, None),
    ("scalar1d_mp_mm_b1", (150,), 0, [0], 8, 8, 1e-6, [1.0]),
    ("euler1d_teno6", (300,), 1, [1], 6, 0, 1e-5, None),
    ("euler3d_teno8", (9, 11, 40), 1, [0, 0, 0], 8, 0, 1e-6, None),
    # eight points with the adaptive cutoff (TENO8A-M, Sec. 2.4)
    ("euler1d_8a_mp", (400,), 1, [1], 8 | 0x100, 1, 0.0, None),
    ("euler2d_8a_tvd5", (25, 48), 1, [0, 0], 8 | 0x100, 3, 0.0, None),
    ("euler3d_8a_va", (9, 10, 33), 1, [0, 1, 0], 8 | 0x100, 4, 0.0, None),
    ("euler2d_8a_teno", (20, 36), 1, [1, 1], 8 | 0x100, 0, 0.0, None),
    ("scalar1d_8a_mp_mm_b2", (257,), 0, [1], 8 | 0x100, 7, 0.0, [-1.3]),
]
IDS = [c[0] for c in CASES]


def make(case, seed=0):
    name, shape, system, bc, K, lim, C_T, adv = case
    nd = len(shape)
    n = list(reversed(shape))
    dx = [0.05, 0.07, 0.06][:nd]
    grid = dict(ndim=nd, n=n, dx=dx, bc=bc, system=system, adv=adv or [0.0] * nd)
    if system == 0:
        U = W.random_scalar_lines(shape, seed=seed + 100, kind="mixed")
    else:
        U = W.random_euler_state(shape, seed=seed + 200, kind="mixed")
    return grid, U, K, lim, C_T


@pytest.fixture(scope="module")
def T():
    require_gpu()
    import paper_2010_13289_amd as T
    return T


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_reconstruct_faces(T, orc, case):
    grid, U, K, lim, C_T = make(case)
    Ud = to_dev(U)
    nd = grid["ndim"]
    for axis in range(nd):
        print(f"[reconstruct_faces] {case[0]} axis={axis}", flush=True)
        Fo, flo, bdo = orc.reconstruct_faces(U, grid, K, lim, C_T, GAMMA, axis)
        Fg, flg = T.reconstruct_faces(Ud, grid, K, lim, C_T, GAMMA, axis, return_flags=True)
        Fg, flg = to_host(Fg), to_host(flg)
        band = band_faces(bdo)
        assert band.sum() <= max(2, band.size // 1000), f"{band.sum()} band faces"
        assert_close_fields(Fg, Fo, exclude=band, what=f"{case[0]} axis {axis} Fhat")
        mism = (flg != flo) & ~band[None, None]
        assert not mism.any(), f"{int(mism.sum())} flag mismatches outside the band"


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_flux_divergence(T, orc, case):
    grid, U, K, lim, C_T = make(case, seed=1)
    print(f"[flux_divergence] {case[0]}", flush=True)
    nd = grid["ndim"]
    do = orc.flux_divergence(U, grid, K, lim, C_T, GAMMA)
    dg = to_host(T.flux_divergence(to_dev(U), grid, K, lim, C_T, GAMMA))
    excl = np.zeros(U.shape[1:], dtype=bool)
    for axis in range(nd):
        _, _, bd = orc.reconstruct_faces(U, grid, K, lim, C_T, GAMMA, axis)
        excl |= faces_to_cells(band_faces(bd), nd - 1 - axis, grid["n"][axis], grid["bc"][axis] == 0, 1)
    assert_close_fields(dg, do, exclude=excl, what=f"{case[0]} dU/dt")


def rk3_band_cells(orc, U, grid, K, lim, C_T, dt):
    """Cells whose one-step result depends on a face in the cutoff band at
    any of the three stages (dependency cone of 3 K/2 cells per axis)."""
    nd = grid["ndim"]
    L0 = orc.flux_divergence(U, grid, K, lim, C_T, GAMMA)
    U1 = U + dt * L0
    L1 = orc.flux_divergence(U1, grid, K, lim, C_T, GAMMA)
    U2 = 0.75 * U + 0.25 * (U1 + dt * L1)
    excl = np.zeros(U.shape[1:], dtype=bool)
    for S in (U, U1, U2):
        for axis in range(nd):
            _, _, bd = orc.reconstruct_faces(S, grid, K, lim, C_T, GAMMA, axis)
            excl |= faces_to_cells(band_faces(bd), nd - 1 - axis, grid["n"][axis], grid["bc"][axis] == 0,
                                   3 * (K & 0xFF) // 2)
    return excl


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_rk3_step(T, orc, case):
    grid, U, K, lim, C_T = make(case, seed=2)
    print(f"[rk3_step] {case[0]}", flush=True)
    dt = 0.4 / orc.max_wave_speed(U, grid, GAMMA)
    Uo = orc.rk3_step(U, grid, K, lim, C_T, GAMMA, dt)
    Ud = to_dev(U)
    ws = T.Workspace(grid, K)
    T.rk3_step(Ud, grid, K, lim, C_T, GAMMA, dt, workspace=ws)
    Ug = to_host(Ud)
    excl = rk3_band_cells(orc, U, grid, K, lim, C_T, dt)
    assert_close_fields(Ug, Uo, exclude=excl, what=f"{case[0]} RK3 step")
    # bitwise determinism of a second run on the same input
    Ud2 = to_dev(U)
    T.rk3_step(Ud2, grid, K, lim, C_T, GAMMA, dt, workspace=ws)
    assert np.array_equal(to_host(Ud2), Ug)


@pytest.mark.parametrize("case", CASES[:6] + CASES[11:13], ids=IDS[:6] + IDS[11:13])
def test_max_wave_speed(T, orc, case):
    grid, U, K, lim, C_T = make(case, seed=3)
    so = orc.max_wave_speed(U, grid, GAMMA)
    sg = T.max_wave_speed(to_dev(U), grid, GAMMA)
    assert sg == pytest.approx(so, rel=1e-13)


@pytest.mark.parametrize("C_T,expect", [(0.0, "all"), (2.0, "none")])
@pytest.mark.parametrize("K", [6, 8])
def test_cutoff_extremes(T, orc, C_T, expect, K):
    """C_T = 0 marks every candidate smooth (linear scheme); C_T > 1 marks
    every candidate nonsmooth (limiter everywhere)."""
    grid = dict(ndim=2, n=[45, 23], dx=[0.1, 0.1], bc=[0, 1], system=1)
    U = W.random_euler_state((23, 45), seed=9, kind="jumps")
    for axis in range(2):
        Fo, flo, _ = orc.reconstruct_faces(U, grid, K, 1, C_T, GAMMA, axis)
        Fg, flg = T.reconstruct_faces(to_dev(U), grid, K, 1, C_T, GAMMA, axis, return_flags=True)
        flg = to_host(flg)
        full = (1 << (K - 2)) - 1
        assert np.all(flg == (full if expect == "all" else 0))
        assert np.array_equal(flg, flo)
        assert_close_fields(to_host(Fg), Fo, what=f"C_T={C_T}")


@pytest.mark.parametrize("scheme", [6, 8, 8 | 0x100])
def test_flags_do_not_depend_on_the_limiter(T, orc, scheme):
    """The cutoff is taken before any limiter (Sec. 3.1), so every limiter
    kind gives the same flags on the same input.  Transmissive axes put runs
    of equal ghost values in the boundary stencils: their differences, and
    so beta_k, must be exactly zero in every kernel instantiation."""
    grid = dict(ndim=2, n=[37, 23], dx=[0.05, 0.07], bc=[1, 1], system=1)
    U = W.random_euler_state((23, 37), seed=211, kind="mixed")
    C_T = 1e-6
    Ud = to_dev(U)
    for axis in range(2):
        print(f"[flags_vs_limiter] scheme={scheme} axis={axis}", flush=True)
        _, flo, bdo = orc.reconstruct_faces(U, grid, scheme, 1, C_T, GAMMA, axis)
        band = band_faces(bdo)
        ref = None
        for lim in range(9):
            _, flg = T.reconstruct_faces(Ud, grid, scheme, lim, C_T, GAMMA, axis, return_flags=True)
            flg = to_host(flg)
            if ref is None:
                ref = flg
            assert np.array_equal(flg, ref), f"limiter {lim}: flags differ from limiter 0"
        mism = (ref != flo) & ~band[None, None]
        assert not mism.any(), f"{int(mism.sum())} flag mismatches outside the band"


@pytest.mark.parametrize("scale", [1e60, -1e60, 1e72, -1e72, 1e-15])
@pytest.mark.parametrize("K", [6, 8])
def test_scalar_faces_at_extreme_magnitudes(T, orc, scale, K):
    """Scalar data scaled far from O(1): the indicators scale with the data
    squared (about 1e120 at 1e60, where the GPU's paired reciprocals of the
    indicator denominators, products of two of them, reach about 1e240).
    At 1e72 the doubled split values reach about 1e73 and the products about
    1e296, close to the documented range of the paired reciprocals (each
    denominator below 2^500, about 3e150).  The cutoff decisions are
    scale-invariant while beta stays far above eps.
    Faces against the oracle to 1e-12 of the largest magnitude, flags equal
    outside the band."""
    grid = dict(ndim=1, n=[300], dx=[0.05], bc=[0], system=0, adv=[1.0])
    U = W.random_scalar_lines((300,), seed=17, kind="mixed") * scale
    print(f"[extreme magnitudes] K={K} scale={scale:g}", flush=True)
    Fo, flo, bdo = orc.reconstruct_faces(U, grid, K, 1, 1e-5, GAMMA, 0)
    Fg, flg = T.reconstruct_faces(to_dev(U), grid, K, 1, 1e-5, GAMMA, 0, return_flags=True)
    Fg, flg = to_host(Fg), to_host(flg)
    assert np.all(np.isfinite(Fg))
    band = band_faces(bdo)
    assert_close_fields(Fg, Fo, exclude=band, what=f"scale {scale:g} Fhat")
    mism = (flg != flo) & ~band[None, None]
    assert not mism.any(), f"{int(mism.sum())} flag mismatches outside the band"
    if abs(scale) > 1.0:
        # the same decisions as on the unscaled data (scale invariance; at
        # small scales eps is no longer negligible against smooth betas)
        _, fl1, bd1 = orc.reconstruct_faces(U / scale, grid, K, 1, 1e-5, GAMMA, 0)
        both = band | band_faces(bd1)
        assert not ((flg != fl1) & ~both[None, None]).any()


def test_constant_state_is_steady(T):
    """A uniform state has zero divergence exactly (every face flux equal)."""
    grid = dict(ndim=3, n=[20, 9, 8], dx=[0.1, 0.1, 0.1], bc=[0, 1, 0], system=1)
    U0 = np.array([0.8, 0.1, -0.3, 0.2, 2.5])
    U = np.broadcast_to(U0[:, None, None, None], (5, 8, 9, 20)).copy()
    d = to_host(T.flux_divergence(to_dev(U), grid, 6, 1, 1e-5, GAMMA))
    assert np.all(d == 0.0)


def test_errors_on_gpu(T):
    import torch
    grid = dict(ndim=1, n=[64], dx=[0.1], bc=[0], system=1)
    U = to_dev(W.random_euler_state((64,), 1))
    with pytest.raises(T.TenomError) as e:
        T.reconstruct_faces(U, grid, 7, 1, 1e-5, GAMMA, 0)
    assert e.value.code == T.EUNSUPPORTED
    with pytest.raises(T.TenomError) as e:
        T.rk3_step(U, grid, 6, 1, 1e-5, GAMMA, -1.0)
    assert e.value.code == T.EINVAL
    small = T.Workspace(dict(ndim=1, n=[32], dx=[0.1], bc=[0], system=1), 6)
    with pytest.raises(T.TenomError) as e:
        T.rk3_step(U, grid, 6, 1, 1e-5, GAMMA, 0.01, workspace=small)
    assert e.value.code == T.EWORKSPACE
    assert T.check_finite(U, grid)
    U[1, 10] = float("nan")
    assert not T.check_finite(U, grid)
    assert np.isnan(T.max_wave_speed(U, grid, GAMMA))
    torch.cuda.synchronize()
