"""Pins of the oracle's system layer: Roe-average characteristic projection,
Rusanov splitting, the conservative divergence and the SSP-RK3 step (Sec. 4),
against exact identities, symmetries and closed forms."""
import math

import numpy as np
import pytest

import workloads as W
from exact_poly import face_weights

GAMMA = 1.4


def prim_to_cons(rho, vel, p, gamma=GAMMA):
    vel = np.asarray(vel, dtype=np.float64)
    return np.concatenate([[rho], rho * vel, [p / (gamma - 1) + 0.5 * rho * vel @ vel]])


def phys_flux(U, ax, gamma=GAMMA):
    nd = len(U) - 2
    rho, m, E = U[0], U[1:1 + nd], U[-1]
    vel = m / rho
    p = (gamma - 1) * (E - 0.5 * rho * vel @ vel)
    F = np.empty_like(U)
    F[0] = m[ax]
    F[1:1 + nd] = m * vel[ax]
    F[1 + ax] += p
    F[-1] = (E + p) * vel[ax]
    return F


def fd_jacobian(U, ax, h=1e-6):
    n = len(U)
    J = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = h * max(1.0, abs(U[j]))
        J[:, j] = (phys_flux(U + e, ax) - phys_flux(U - e, ax)) / (2 * e[j])
    return J


def roe_state(UL, UR, gamma=GAMMA):
    """Conservative state with the Roe-averaged velocity and enthalpy (and
    density sqrt(rhoL rhoR)); the flux Jacobian depends only on (u, H)."""
    nd = len(UL) - 2

    def prim(U):
        rho = U[0]
        vel = U[1:1 + nd] / rho
        p = (gamma - 1) * (U[-1] - 0.5 * rho * vel @ vel)
        return rho, vel, (U[-1] + p) / rho

    rl, vl, Hl = prim(UL)
    rr, vr, Hr = prim(UR)
    sl, sr = math.sqrt(rl), math.sqrt(rr)
    u = (sl * vl + sr * vr) / (sl + sr)
    H = (sl * Hl + sr * Hr) / (sl + sr)
    rho = sl * sr
    E = rho * (H + (gamma - 1) * 0.5 * u @ u) / gamma
    return np.concatenate([[rho], rho * u, [E]]), u, H


def random_prim(rng, nd):
    return rng.uniform(0.2, 2.0), rng.uniform(-1.5, 1.5, nd), rng.uniform(0.2, 2.0)


@pytest.mark.parametrize("nd", [1, 2, 3])
def test_roe_eigensystem(orc, nd):
    rng = np.random.default_rng(nd)
    for _ in range(10):
        UL = prim_to_cons(*random_prim(rng, nd))
        UR = prim_to_cons(*random_prim(rng, nd))
        Ut, u, H = roe_state(UL, UR)
        c = math.sqrt((GAMMA - 1) * (H - 0.5 * u @ u))
        for ax in range(nd):
            R, L = orc.roe_eigenvectors(nd, GAMMA, ax, UL, UR)
            np.testing.assert_allclose(L @ R, np.eye(nd + 2), atol=1e-13)
            lam = np.array([u[ax] - c] + [u[ax]] * nd + [u[ax] + c])
            A = R @ np.diag(lam) @ L
            # R diag(lambda) L is the flux Jacobian at the Roe state ...
            np.testing.assert_allclose(A, fd_jacobian(Ut, ax), rtol=1e-6, atol=1e-6)
            # ... and satisfies Roe's property A (UR - UL) = F(UR) - F(UL)
            np.testing.assert_allclose(A @ (UR - UL), phys_flux(UR, ax) - phys_flux(UL, ax),
                                       rtol=1e-12, atol=1e-12)


def grid(ndim, n, dx=None, bc=None, system=1, adv=None):
    n = list(n)
    return dict(ndim=ndim, n=n, dx=dx or [1.0 / v for v in n], bc=bc or [0] * ndim, system=system,
                adv=adv or [0.0] * ndim)


@pytest.mark.parametrize("K,lim", [(6, 1), (8, 2), (8, 3), (6, 4)])
def test_constant_state_gives_physical_flux(orc, K, lim):
    """Consistency: on a uniform state every reconstruction returns the
    point value, and the LF split sums back to the physical flux."""
    U0 = prim_to_cons(0.7, np.array([0.3, -0.2, 0.5]), 1.3)
    g = grid(3, [9, 8, 7])
    U = np.broadcast_to(U0[:, None, None, None], (5, 7, 8, 9)).copy()
    for ax in range(3):
        F, fl, _ = orc.reconstruct_faces(U, g, K, lim, 1e-5, GAMMA, ax)
        np.testing.assert_allclose(F.reshape(5, -1), np.repeat(phys_flux(U0, ax)[:, None], F[0].size, 1),
                                   rtol=1e-13, atol=1e-13)
        assert np.all(fl == (1 << (K - 2)) - 1)


@pytest.mark.parametrize("nd,K,lim", [(1, 6, 1), (1, 8, 2), (2, 6, 3), (2, 8, 1), (3, 6, 1), (3, 8, 3)])
def test_periodic_conservation(orc, nd, K, lim):
    shape = {1: (64,), 2: (12, 14), 3: (8, 9, 10)}[nd]
    U = W.random_euler_state(shape, seed=nd * 10 + K, kind="mixed")
    g = grid(nd, list(reversed(shape)), dx=[0.1, 0.2, 0.3][:nd])
    dU = orc.flux_divergence(U, g, K, lim, 1e-5, GAMMA)
    scale = np.abs(dU).reshape(nd + 2, -1).max(axis=1)
    total = dU.reshape(nd + 2, -1).sum(axis=1)
    assert np.all(np.abs(total) <= 1e-12 * scale * dU[0].size)


def test_transmissive_boundary_flux_identity(orc):
    """Telescoping: sum_i dU_i dx = -(F_n - F_0) with clamped ghost cells."""
    U, dx = W.riemann_problem(80, W.SOD[0], W.SOD[1])
    g = grid(1, [80], dx=[dx], bc=[1])
    dU = orc.flux_divergence(U, g, 6, 1, 1e-5, GAMMA)
    F, _, _ = orc.reconstruct_faces(U, g, 6, 1, 1e-5, GAMMA, 0)
    np.testing.assert_allclose(dU.sum(axis=1) * dx, -(F[:, -1] - F[:, 0]), atol=1e-12)
    # far from the tube's waves the boundary faces carry the physical flux
    np.testing.assert_allclose(F[:, 0], phys_flux(U[:, 0], 0), rtol=1e-13)


@pytest.mark.parametrize("K,lim", [(6, 1), (8, 3), (8, 2)])
def test_reflection_symmetry(orc, K, lim):
    """x -> -x maps (rho, m, E) -> (rho, -m, E) and must commute with the
    scheme: the f- side is the mirror image of the f+ side."""
    U = W.random_euler_state((40,), seed=5, kind="jumps")
    g = grid(1, [40], bc=[0])
    dU = orc.flux_divergence(U, g, K, lim, 1e-5, GAMMA)
    Ur = U[:, ::-1].copy()
    Ur[1] *= -1
    dUr = orc.flux_divergence(Ur, g, K, lim, 1e-5, GAMMA)
    dUr = dUr[:, ::-1].copy()
    dUr[1] *= -1
    np.testing.assert_allclose(dUr, dU, rtol=1e-11, atol=1e-11 * np.abs(dU).max())


@pytest.mark.parametrize("K,lim", [(6, 1), (8, 3)])
def test_axis_permutation_symmetry(orc, K, lim):
    """Swapping x and y (and the two momenta) commutes with the scheme."""
    U = W.random_euler_state((6, 7, 8), seed=8, kind="mixed")
    g = grid(3, [8, 7, 6], dx=[0.1, 0.1, 0.2])
    dU = orc.flux_divergence(U, g, K, lim, 1e-5, GAMMA)
    Up = U.transpose(0, 1, 3, 2)[[0, 2, 1, 3, 4]].copy()
    gp = grid(3, [7, 8, 6], dx=[0.1, 0.1, 0.2])
    dUp = orc.flux_divergence(Up, gp, K, lim, 1e-5, GAMMA)
    back = dUp.transpose(0, 1, 3, 2)[[0, 2, 1, 3, 4]]
    np.testing.assert_allclose(back, dU, rtol=1e-11, atol=1e-11 * np.abs(dU).max())


@pytest.mark.parametrize("K", [6, 8])
def test_linear_advection_symbol_and_rk3_amplification(orc, K):
    """With C_T = 0 the scheme is linear: a Fourier mode is an eigenvector of
    dU/dt with the symbol of the K-point linear scheme (closed form), and one
    SSP-RK3 step multiplies it by 1 + z + z^2/2 + z^3/6."""
    n, a = 32, 1.0
    c = np.array([float(v) for v in face_weights(-(K // 2) + 1, K // 2)])
    offs = np.arange(-(K // 2) + 1, K // 2 + 1)
    dx = 1.0 / n
    g = grid(1, [n], dx=[dx], system=0, adv=[a])
    for k in (1, 3, 7):
        theta = 2 * math.pi * k / n
        # face i+1/2 flux of exp(i theta j): exp(i theta i) * sum_m c_m exp(i theta m)
        sym = -(a / dx) * (1 - np.exp(-1j * theta)) * np.sum(c * np.exp(1j * theta * offs))
        x = np.arange(n)
        u = np.cos(theta * x)[None, :]
        dU = orc.flux_divergence(u, g, K, 1, 0.0, GAMMA)
        expect = (sym * np.exp(1j * theta * x)).real
        np.testing.assert_allclose(dU[0], expect, atol=1e-11 * n)
        dt = 0.4 * dx
        z = sym * dt
        G = 1 + z + z * z / 2 + z ** 3 / 6
        un = orc.rk3_step(u, g, K, 1, 0.0, GAMMA, dt)
        np.testing.assert_allclose(un[0], (G * np.exp(1j * theta * x)).real, atol=1e-12)
    # the linear background is central: the symbol of a real mode is imaginary
    assert abs(sym.real) < 1e-9 * abs(sym)


def test_scalar_negative_speed_mirrors_positive(orc):
    """u_t - u_x = 0 on data u(x) equals u_t + u_x = 0 on u(-x), mirrored:
    exercises the f- (mirrored) reconstruction of the scalar split."""
    u = W.random_scalar_lines((50,), seed=3, kind="mixed")
    g_neg = grid(1, [50], dx=[0.02], system=0, adv=[-1.0])
    g_pos = grid(1, [50], dx=[0.02], system=0, adv=[1.0])
    d_neg = orc.flux_divergence(u, g_neg, 6, 1, 1e-5, GAMMA)
    d_pos = orc.flux_divergence(u[:, ::-1].copy(), g_pos, 6, 1, 1e-5, GAMMA)
    np.testing.assert_allclose(d_neg, d_pos[:, ::-1], rtol=1e-12, atol=1e-12)


def test_sampled_entry_points_match_whole_grid(orc):
    for nd, bc in ((1, [1]), (2, [0, 1]), (3, [0, 0, 0]), (3, [1, 0, 1])):
        shape = {1: (30,), 2: (10, 11), 3: (9, 8, 7)}[nd]
        U = W.random_euler_state(shape, seed=nd, kind="mixed")
        g = grid(nd, list(reversed(shape)), dx=[0.1, 0.12, 0.15][:nd], bc=bc)
        K, lim = (6, 1) if nd != 2 else (8, 3)
        ncell = int(np.prod(shape))
        rng = np.random.default_rng(nd)
        idx = rng.choice(ncell, size=min(12, ncell), replace=False)
        for ax in range(nd):
            F, fl, bd = orc.reconstruct_faces(U, g, K, lim, 1e-5, GAMMA, ax)
            fidx = rng.choice(F[0].size, size=10, replace=False)
            Fp, flp, _ = orc.faces_points(U, g, K, lim, 1e-5, GAMMA, ax, fidx)
            np.testing.assert_array_equal(Fp, F.reshape(nd + 2, -1)[:, fidx].T)
            np.testing.assert_array_equal(flp, fl.reshape(2 * (nd + 2), -1)[:, fidx].T)
        dU = orc.flux_divergence(U, g, K, lim, 1e-5, GAMMA)
        dp, _ = orc.dudt_points(U, g, K, lim, 1e-5, GAMMA, idx)
        np.testing.assert_allclose(dp, dU.reshape(nd + 2, -1)[:, idx].T, rtol=1e-13, atol=1e-13 * np.abs(dU).max())
        dt = 0.2 / orc.max_wave_speed(U, g, GAMMA)
        Un = orc.rk3_step(U, g, K, lim, 1e-5, GAMMA, dt)
        up, _ = orc.rk3_points(U, g, K, lim, 1e-5, GAMMA, dt, idx)
        np.testing.assert_allclose(up, Un.reshape(nd + 2, -1)[:, idx].T, rtol=1e-13, atol=1e-13)


def test_max_wave_speed(orc):
    U = W.random_euler_state((5, 6, 7), seed=2)
    g = grid(3, [7, 6, 5], dx=[0.1, 0.2, 0.3])
    rho = U[0]
    vel = U[1:4] / rho
    p = (GAMMA - 1) * (U[4] - 0.5 * rho * (vel ** 2).sum(0))
    c = np.sqrt(GAMMA * p / rho)
    s = sum((np.abs(vel[d]) + c) / g["dx"][d] for d in range(3))
    assert orc.max_wave_speed(U, g, GAMMA) == pytest.approx(s.max(), rel=1e-14)
