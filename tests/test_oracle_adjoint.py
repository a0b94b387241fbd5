"""Pins of the reference adjoint (oracle/reference_adjoint.py), the CPU
check of the GPU adjoint: its forward map equals the C oracle's, and its
vector-Jacobian products equal central differences of the C oracle's flux
divergence and RK3 step along random directions (with the oracle's
smoothness flags unchanged between U - hV and U + hV)."""
import numpy as np
import pytest

import workloads as W
from oracle import reference_adjoint as RA

GAMMA = 1.4

# name, shape (z, y, x), grid, scheme, limiter, C_T
CASES = [
    ("euler1d_mp6_trans", (40,), dict(ndim=1, n=[40], dx=[0.05], bc=[1], system=1), 6, 1, 1e-5),
    ("euler2d_tvd5_8", (14, 12), dict(ndim=2, n=[12, 14], dx=[0.05, 0.07], bc=[0, 1], system=1), 8, 3, 1e-7),
    ("euler2d_8a_va", (14, 12), dict(ndim=2, n=[12, 14], dx=[0.05, 0.07], bc=[1, 0], system=1), 8 | 0x100, 4, 0.0),
    ("euler2d_mpmm6", (12, 13), dict(ndim=2, n=[13, 12], dx=[0.06, 0.05], bc=[0, 0], system=1), 6, 6, 1e-5),
    ("euler1d_tvdmm8", (36,), dict(ndim=1, n=[36], dx=[0.05], bc=[0], system=1), 8, 2, 1e-7),
    ("euler1d_teno6", (30,), dict(ndim=1, n=[30], dx=[0.05], bc=[1], system=1), 6, 0, 1e-5),
    ("scalar1d_mp8", (34,), dict(ndim=1, n=[34], dx=[0.05], bc=[0], system=0, adv=[-0.7]), 8, 1, 1e-7),
    ("euler3d_mp6", (7, 8, 9), dict(ndim=3, n=[9, 8, 7], dx=[0.05, 0.06, 0.07], bc=[0, 1, 0], system=1), 6, 1, 1e-5),
]
IDS = [c[0] for c in CASES]


def state(case, seed):
    """Mixed smooth and discontinuous data, every value moved by a 0.1 %
    random factor: no characteristic field is identically zero (a field that
    is zero up to rounding, e.g. a shear wave of a velocity component that is
    constant along the axis, has smoothness decisions set by rounding noise
    on any implementation)."""
    shape, grid = case[1], case[2]
    if grid["system"] == 0:
        U = W.random_scalar_lines(shape, seed=seed, kind="mixed")
    else:
        U = W.random_euler_state(shape, seed=seed, kind="mixed")
    return U * (1.0 + 1e-3 * np.random.default_rng(seed + 1000).standard_normal(U.shape))


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_reference_forward_is_the_oracle(orc, case):
    """Same values (1e-12 of each field's scale) and the same smoothness
    flags outside the cutoff band."""
    name, shape, grid, K, lim, C_T = case
    U = state(case, 1)
    Lr, flags = RA.flux_divergence(RA._t(U), grid, K, lim, C_T, GAMMA, return_flags=True)
    Lo = orc.flux_divergence(U, grid, K, lim, C_T, GAMMA)
    ax = tuple(range(1, U.ndim))
    assert np.all(np.abs(Lr.numpy() - Lo).max(axis=ax) <= 1e-12 * np.abs(Lo).max(axis=ax))
    for axis in range(grid["ndim"]):
        _, flo, bdo = orc.reconstruct_faces(U, grid, K, lim, C_T, GAMMA, axis)
        d = flags[axis].numpy()                       # [2, nf, ..., faces, K-2] along the axis
        bits = (d * (1 << np.arange(d.shape[-1]))).sum(-1).astype(np.uint8)
        bits = np.moveaxis(bits, -1, bits.ndim - 1 - axis)
        band = np.any(bdo.reshape((-1,) + bdo.shape[2:]) != 0, axis=0)
        assert np.array_equal(np.where(band, 0, bits), np.where(band, 0, flo))


def _fd_check(f_oracle, flags_oracle, vjp, U, rng, ndir=6, rtol=1e-6):
    """<Lbar, (f(U + hV) - f(U - hV)) / 2h> against <V, vjp(Lbar)>.

    A direction is usable when the oracle's smoothness flags are those of U
    at U -+ hV and the central differences at h = 1e-7 and 1e-8 (relative to
    each field's scale) agree to 1e-6: no limiter branch changes within the
    interval, so the map is smooth there and its derivative is the one with
    every choice frozen.  (On these data ties sit ~1e-6 apart, so h = 1e-6
    can cross one.)"""
    ax = tuple(range(1, U.ndim))
    scale = np.abs(U).max(axis=ax, keepdims=True)
    base = flags_oracle(U)
    checked = 0
    for _ in range(ndir):
        V = rng.standard_normal(U.shape) * scale
        Lbar = rng.standard_normal(U.shape)
        fd = []
        for h in (1e-7, 1e-8):
            if not (np.array_equal(flags_oracle(U + h * V), base) and np.array_equal(flags_oracle(U - h * V), base)):
                break
            fd.append(np.sum(Lbar * (f_oracle(U + h * V) - f_oracle(U - h * V))) / (2 * h))
        if len(fd) < 2 or abs(fd[0] - fd[1]) > 1e-6 * abs(fd[0]):
            continue
        ad = np.sum(V * vjp(Lbar))
        assert abs(fd[0] - ad) <= rtol * abs(ad) + 1e-9 * np.sum(np.abs(Lbar)), (fd, ad)
        checked += 1
    assert checked >= max(2, ndir // 2), f"only {checked} of {ndir} directions usable"


def _flags(orc, grid, K, lim, C_T):
    def f(U):
        return np.concatenate([orc.reconstruct_faces(U, grid, K, lim, C_T, GAMMA, a)[1].ravel()
                               for a in range(grid["ndim"])])
    return f


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_reference_vjp_matches_oracle_differences(orc, case):
    name, shape, grid, K, lim, C_T = case
    U = state(case, 2)
    rng = np.random.default_rng(77)
    _fd_check(lambda V: orc.flux_divergence(V, grid, K, lim, C_T, GAMMA), _flags(orc, grid, K, lim, C_T),
              lambda Lb: RA.flux_divergence_vjp(U, Lb, grid, K, lim, C_T, GAMMA), U, rng)


@pytest.mark.parametrize("case", [CASES[0], CASES[1], CASES[2], CASES[6]], ids=[IDS[0], IDS[1], IDS[2], IDS[6]])
def test_reference_rk3_vjp_matches_oracle_differences(orc, case):
    """Through one step: the flags of all three stages are held fixed by
    checking those of the step's input (a small h keeps the stage states
    within rounding of each other's decisions)."""
    name, shape, grid, K, lim, C_T = case
    U = state(case, 3)
    dt = 0.4 / orc.max_wave_speed(U, grid, GAMMA)
    rng = np.random.default_rng(78)
    _fd_check(lambda V: orc.rk3_step(V, grid, K, lim, C_T, GAMMA, dt), _flags(orc, grid, K, lim, C_T),
              lambda Ub: RA.rk3_step_vjp(U, Ub, grid, K, lim, C_T, GAMMA, dt), U, rng, ndir=8)


def test_linear_scheme_adjoint_is_the_transpose():
    """C_T = 0: every candidate smooth, the reconstruction is the K-point
    linear scheme and the scalar divergence is a circulant matrix; its
    adjoint must be the exact transpose (built column by column)."""
    n = 16
    grid = dict(ndim=1, n=[n], dx=[0.1], bc=[0], system=0, adv=[1.3])
    U = W.random_scalar_lines((n,), seed=5, kind="mixed")
    J = np.zeros((n, n))
    for j in range(n):
        e = np.zeros((1, n))
        e[0, j] = 1.0
        J[:, j] = RA.flux_divergence_np(e, grid, 6, 1, 0.0, GAMMA)[0]
    rng = np.random.default_rng(3)
    Lbar = rng.standard_normal((1, n))
    g = RA.flux_divergence_vjp(U, Lbar, grid, 6, 1, 0.0, GAMMA)
    assert np.allclose(g[0], J.T @ Lbar[0], rtol=1e-13, atol=1e-12)
