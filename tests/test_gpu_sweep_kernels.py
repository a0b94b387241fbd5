"""The tile sweep against the line sweeps and the oracle, on every axis.

The tile sweep (a workgroup stages tiles of 8 adjacent lines by a chunk of
the line in LDS and walks the lines whole, handing each chunk's last face to
the next; the lines are x columns for y and z, y rows for x) and the line
kernels (the row sweep for x; for y and z the march, one lane per x column
with its stencil in an LDS ring) evaluate the same face fluxes and cell
updates operation for operation, so their results must agree bit for bit.
The shapes put line lengths below, at and just above one chunk (32 faces)
and several chunks with a ragged last one, on every axis, extents across
the lines that leave part of the last group of 8 outside the grid, and both
boundary rules on every axis; the automatic choice takes the line kernels
for all of them, so each kernel is forced through tenom_set_sweep_kernel.
One case per scheme also goes to the oracle on the tile path directly
(1e-12 of each field's largest magnitude outside the cutoff band, as in the
other parity tests).
"""
import numpy as np
import pytest

import workloads as W
from parity import assert_close_fields, require_gpu, to_dev, to_host
from test_gpu_parity import CASES, make, rk3_band_cells

pytestmark = pytest.mark.gpu

GAMMA = 1.4

# name, shape (z, y, x order), bc (x, y, z order), scheme, limiter, C_T
SHAPES = [
    ("chunk_below", (20, 31, 13), [0, 0, 1], 6, 1, 1e-5),
    ("chunk_exact", (32, 32, 16), [1, 0, 0], 6, 1, 1e-5),
    ("chunk_above", (33, 33, 9), [0, 1, 0], 8, 1, 1e-7),
    ("chunks_ragged", (70, 12, 24), [0, 0, 0], 6, 3, 1e-5),
    ("chunks_ragged_trans", (12, 97, 17), [1, 1, 1], 8, 2, 1e-7),
    ("two_chunks_exact", (64, 9, 8), [0, 1, 1], 8 | 0x100, 1, 0.0),
    ("narrow_x", (40, 36, 6), [0, 0, 1], 6, 7, 1e-5),
    ("teno8_long_y", (9, 129, 11), [1, 0, 0], 8, 0, 1e-6),
    ("x_chunks_ragged", (6, 13, 70), [0, 1, 0], 6, 1, 1e-5),
    ("x_two_chunks_exact", (8, 17, 64), [1, 0, 0], 8, 1, 1e-7),
    ("x_chunk_above", (8, 8, 33), [0, 0, 1], 8 | 0x100, 1, 0.0),
]
SHAPE_IDS = [s[0] for s in SHAPES]
MULTI_D = [c for c in CASES if len(c[1]) >= 2]


@pytest.fixture(scope="module")
def T():
    require_gpu()
    import paper_2010_13289_amd as T
    yield T
    T.set_sweep_kernel(T.SWEEP_AUTO)


def both_kernels(T, fn):
    out = []
    for kind in (T.SWEEP_TILE, T.SWEEP_MARCH):
        T.set_sweep_kernel(kind)
        out.append(fn())
    T.set_sweep_kernel(T.SWEEP_AUTO)
    return out


def shape_case(spec, seed):
    name, shape, bc, K, lim, C_T = spec
    n = list(reversed(shape))
    grid = dict(ndim=3, n=n, dx=[0.05, 0.07, 0.06], bc=bc, system=1)
    U = W.random_euler_state(shape, seed=seed, kind="mixed")
    return grid, U, K, lim, C_T


def check_identical(T, grid, U, K, lim, C_T, what):
    dt = 0.4 / T.max_wave_speed(to_dev(U), grid, GAMMA)

    def div():
        return to_host(T.flux_divergence(to_dev(U), grid, K, lim, C_T, GAMMA))

    def step():
        Ud = to_dev(U)
        T.rk3_step(Ud, grid, K, lim, C_T, GAMMA, dt)
        return to_host(Ud)

    d_tile, d_march = both_kernels(T, div)
    assert np.array_equal(d_tile, d_march), f"{what}: divergence differs between the sweep kernels"
    s_tile, s_march = both_kernels(T, step)
    assert np.array_equal(s_tile, s_march), f"{what}: RK3 step differs between the sweep kernels"
    return d_tile, s_tile, dt


@pytest.mark.parametrize("spec", SHAPES, ids=SHAPE_IDS)
def test_tile_and_march_agree_on_chunk_shapes(T, spec):
    grid, U, K, lim, C_T = shape_case(spec, seed=31)
    print(f"[sweep kernels] {spec[0]} n={grid['n']} bc={grid['bc']}", flush=True)
    check_identical(T, grid, U, K, lim, C_T, spec[0])


@pytest.mark.parametrize("case", MULTI_D, ids=[c[0] for c in MULTI_D])
def test_tile_and_march_agree_on_parity_cases(T, case):
    grid, U, K, lim, C_T = make(case, seed=5)
    print(f"[sweep kernels] {case[0]}", flush=True)
    check_identical(T, grid, U, K, lim, C_T, case[0])


ORACLE_SHAPES = [SHAPES[i] for i in (1, 4, 5, 8)]


@pytest.mark.parametrize("spec", ORACLE_SHAPES, ids=[s[0] for s in ORACLE_SHAPES])
def test_tile_against_the_oracle(T, orc, spec):
    grid, U, K, lim, C_T = shape_case(spec, seed=43)
    print(f"[tile vs oracle] {spec[0]}", flush=True)
    T.set_sweep_kernel(T.SWEEP_TILE)
    try:
        dt = 0.4 / orc.max_wave_speed(U, grid, GAMMA)
        Ud = to_dev(U)
        T.rk3_step(Ud, grid, K, lim, C_T, GAMMA, dt)
        Ug = to_host(Ud)
    finally:
        T.set_sweep_kernel(T.SWEEP_AUTO)
    Uo = orc.rk3_step(U, grid, K, lim, C_T, GAMMA, dt)
    excl = rk3_band_cells(orc, U, grid, K, lim, C_T, dt)
    assert_close_fields(Ug, Uo, exclude=excl, what=f"{spec[0]} RK3 step, tile sweeps")


def test_automatic_choice_at_64_cubed_against_the_oracle(T, orc):
    """At 64^3 the lines of every axis give 512 tile workgroups, so the
    automatic choice runs the tile sweeps: the divergence of a seeded state against
    the oracle over every cell outside the cutoff band (1e-12 of each field's
    largest magnitude)."""
    from parity import band_faces, faces_to_cells
    shape = (64, 64, 64)
    grid = dict(ndim=3, n=[64, 64, 64], dx=[0.05, 0.07, 0.06], bc=[0, 1, 0], system=1)
    U = W.random_euler_state(shape, seed=57, kind="mixed")
    K, lim, C_T = 6, 1, 1e-5
    print("[automatic choice] 64^3 divergence", flush=True)
    T.set_sweep_kernel(T.SWEEP_AUTO)
    dg = to_host(T.flux_divergence(to_dev(U), grid, K, lim, C_T, GAMMA))
    do = orc.flux_divergence(U, grid, K, lim, C_T, GAMMA)
    excl = np.zeros(shape, dtype=bool)
    for axis in range(3):
        _, _, bd = orc.reconstruct_faces(U, grid, K, lim, C_T, GAMMA, axis)
        excl |= faces_to_cells(band_faces(bd), 2 - axis, 64, grid["bc"][axis] == 0, 1)
    assert excl.mean() < 0.01
    assert_close_fields(dg, do, exclude=excl, what="64^3 dU/dt, automatic sweep kernels")
