"""Integration pins of the oracle (Sec. 4): design order on smooth
advection, no new extrema on a square wave, shock tubes against the exact
Riemann solution, and the exact Riemann solver's own consistency."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import exact_riemann as ER
from fixtures import shock_tubes

GAMMA = 1.4


def g1(n, dx, bc=0, system=1, a=1.0):
    return dict(ndim=1, n=[n], dx=[dx], bc=[bc], system=system, adv=[a])


# -------------------------------------------------------------------------
# accuracy (Sec. 4.1.1)
# -------------------------------------------------------------------------

@pytest.mark.parametrize("K,lim", [(6, 1), (8, 1), (6, 3), (8, 2)])
def test_semi_discrete_design_order(orc, K, lim):
    """Gaussian pulse exp(-300 (x - 1/2)^2): once resolved (N = 320) every
    stencil is smooth, and the semi-discrete error of -u_x converges at
    order K.  On coarser grids only the exponentially small tails (where the
    profile decays by a large factor per cell) are flagged."""
    errs, ns = [], [80, 160, 320]
    for n in ns:
        u, dx = W.gaussian_pulse(n)
        x = W.cell_centres(n, 0.0, 1.0)
        g = g1(n, dx, system=0)
        F, fl, _ = orc.reconstruct_faces(u, g, K, lim, 1e-5 if K == 6 else 1e-7, GAMMA, 0)
        smooth = fl[0, 0] == (1 << (K - 2)) - 1
        uf = np.concatenate([u[0][-1:], u[0]])  # value left of each face
        assert np.all(smooth[uf > 1e-3])
        if n == ns[-1]:
            assert np.all(smooth)
        dU = orc.flux_divergence(u, g, K, lim, 1e-5 if K == 6 else 1e-7, GAMMA)
        exact = 600.0 * (x - 0.5) * np.exp(-300.0 * (x - 0.5) ** 2)
        errs.append(np.max(np.abs(dU[0] - exact)))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert orders[-1] > K - 0.4, (errs, orders)


def test_full_discrete_order_with_small_steps(orc):
    """sin(pi x) advected once around [-1, 1] with dt ~ dx^2: the L_inf error
    shows the sixth-order spatial convergence of the K = 6 scheme."""
    errs = []
    for n in (20, 40):
        u, dx = W.advection_sine_pulse(n, pulse=False)
        g = g1(n, dx, system=0)
        T, dt0 = 0.5, 0.4 * dx * (dx / 0.1)
        steps = int(math.ceil(T / dt0))
        dt = T / steps
        for _ in range(steps):
            u = orc.rk3_step(u, g, 6, 1, 1e-5, GAMMA, dt)
        x = W.cell_centres(n, -1.0, 1.0)
        errs.append(np.max(np.abs(u[0] - np.sin(np.pi * (x - T)))))
    order = math.log2(errs[0] / errs[1])
    assert order > 5.5, (errs, order)


# -------------------------------------------------------------------------
# no new extrema (Sec. 4.1.2)
# -------------------------------------------------------------------------

@pytest.mark.parametrize("K,lim", [(6, 1), (8, 1), (6, 3), (8, 2), (6, 4)])
def test_square_wave_no_new_extrema(orc, K, lim):
    """Sec. 4.1.2: the square wave is advected without oscillations.  The
    limiters act only on candidates classified nonsmooth, so the scheme is
    not strictly monotonicity preserving: candidates classified smooth near
    the smeared plateau may overshoot by round-off-like amounts.  Pinned:
    no new extremum larger than 1e-5 of the jump, none at all below."""
    n = 100
    u, dx = W.square_wave(n)
    g = g1(n, dx, system=0)
    dt = 0.4 * dx
    for _ in range(60):
        u = orc.rk3_step(u, g, K, lim, 1e-5 if K == 6 else 1e-7, GAMMA, dt)
    assert u.min() >= -1e-15 and u.max() <= 1.0 + 1e-5, (u.min(), u.max())
    assert abs(u.sum() * dx - 0.25) < 1e-12  # conservation


def test_advection_config_sine_plus_pulse(orc):
    """sin(pi x) + unit pulse on [-0.4, -0.2], N = 200, TENO6-M-MP, CFL 0.4, to
    t = 2 (one period): conservation to round-off, and the smooth part away
    from the two jumps returns close to its initial values (the jumps sweep
    the whole period once, so their limiting leaves a small trail)."""
    n = 200
    u, dx = W.advection_sine_pulse(n)
    u0 = u.copy()
    g = g1(n, dx, system=0)
    steps = int(round(2.0 / (0.4 * dx)))
    dt = 2.0 / steps
    for _ in range(steps):
        u = orc.rk3_step(u, g, 6, 1, 1e-5, GAMMA, dt)
    assert abs(u.sum() - u0.sum()) < 1e-10
    x = W.cell_centres(n, -1.0, 1.0)
    far = (np.abs(x + 0.4) > 0.15) & (np.abs(x + 0.2) > 0.15)
    assert np.max(np.abs(u[0][far] - u0[0][far])) < 2e-3
    assert np.median(np.abs(u[0][far] - u0[0][far])) < 1e-4
    # the plateau of the pulse keeps its height
    assert u.max() <= u0.max() + 1e-3


# -------------------------------------------------------------------------
# exact Riemann solver pins
# -------------------------------------------------------------------------

def cons(rho, u, p):
    return np.array([rho, rho * u, p / (GAMMA - 1) + 0.5 * rho * u * u])


def flux(rho, u, p):
    E = p / (GAMMA - 1) + 0.5 * rho * u * u
    return np.array([rho * u, rho * u * u + p, (E + p) * u])


@pytest.mark.parametrize("seed", range(8))
def test_exact_riemann_integral_conservation(seed):
    """d/dt int U dx = F(U_L) - F(U_R) exactly while waves stay inside: the
    sampled exact solution must satisfy it (pins p*, u* and every wave)."""
    left, right = W.riemann_states(seed)
    sl, sr = ER.wave_speeds(left, right)
    t = 1.0
    a, b = sl * t - 1.0, sr * t + 1.0
    x = np.linspace(a, b, 400001)
    rho, u, p = ER.sample(left, right, x / t)
    U = np.stack([rho, rho * u, p / (GAMMA - 1) + 0.5 * rho * u * u])
    integ = np.trapezoid(U, x, axis=1)
    init = cons(*left) * (0 - a) + cons(*right) * (b - 0)
    expect = init + t * (flux(*left) - flux(*right))
    np.testing.assert_allclose(integ, expect, rtol=2e-5, atol=2e-5)


def test_exact_riemann_invariants():
    left, right = W.SOD
    ps, us = ER.star_state(left, right)
    # Sod: left rarefaction, right shock
    rho, u, p = ER.sample(left, right, np.linspace(-1.2, 1.8, 3001))
    fan = (p < left[2] - 1e-9) & (p > ps + 1e-9)
    c = np.sqrt(GAMMA * p / rho)
    # across the left fan: u + 2c/(gamma-1) and p / rho^gamma are constant
    cl = math.sqrt(GAMMA * left[2] / left[0])
    np.testing.assert_allclose(u[fan] + 2 * c[fan] / (GAMMA - 1), left[1] + 2 * cl / (GAMMA - 1), rtol=1e-12)
    np.testing.assert_allclose(p[fan] / rho[fan] ** GAMMA, left[2] / left[0] ** GAMMA, rtol=1e-12)
    # Rankine-Hugoniot at the right shock moving with speed S:
    # F(post) - S U(post) = F(pre) - S U(pre), for all three components
    _, S = ER.wave_speeds(left, right)
    r1, u1, p1 = (v[0] for v in ER.sample(left, right, [S - 1e-9]))
    assert p1 == pytest.approx(ps, rel=1e-14) and u1 == pytest.approx(us, rel=1e-14)
    np.testing.assert_allclose(flux(r1, u1, p1) - S * cons(r1, u1, p1),
                               flux(*right) - S * cons(*right), rtol=1e-12, atol=1e-12)
    # symmetric collision: u* = 0
    assert abs(ER.star_state((1, 0.5, 1), (1, -0.5, 1))[1]) < 1e-14
    # identical states: no waves
    pst, ust = ER.star_state((0.3, 0.2, 0.7), (0.3, 0.2, 0.7))
    assert pst == pytest.approx(0.7, rel=1e-14) and ust == pytest.approx(0.2, rel=1e-14)


# -------------------------------------------------------------------------
# shock tubes (Sec. 4.2.1) and seeded Riemann problems
# -------------------------------------------------------------------------

def run_tube(orc, n, left, right, t_end, K, lim, C_T):
    U, dx = W.riemann_problem(n, left, right)
    g = g1(n, dx, bc=1)
    t = 0.0
    while t < t_end - 1e-14:
        dt = min(0.4 / orc.max_wave_speed(U, g, GAMMA), t_end - t)
        U = orc.rk3_step(U, g, K, lim, C_T, GAMMA, dt)
        t += dt
    x = W.cell_centres(n, 0.0, 1.0)
    rho, _, _ = ER.sample(left, right, (x - 0.5) / t_end)
    return np.mean(np.abs(U[0] - rho)), U


@pytest.mark.parametrize("name", ["sod", "lax"])
@pytest.mark.parametrize("K,lim,C_T", [(6, 1, 1e-5), (8, 2, 1e-7)])
def test_shock_tubes_converge_to_exact_solution(orc, name, K, lim, C_T):
    """Sec. 4.2.1 (Eqs. sod, lax): states, end time and the coarse N come
    from the fixture; the error must fall when N doubles."""
    tube = shock_tubes()[name]
    left, right, t_end, n = tube["left"], tube["right"], tube["t_end"], tube["n"]
    e100, U = run_tube(orc, n, left, right, t_end, K, lim, C_T)
    e200, _ = run_tube(orc, 2 * n, left, right, t_end, K, lim, C_T)
    assert e100 < (0.02 if name == "sod" else 0.05), e100
    assert e200 < 0.75 * e100, (e100, e200)
    assert np.all(U[0] > 0)


@pytest.mark.slow
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_seeded_riemann_problems(orc, seed):
    """Seeded states (rho, p in [0.1, 1], u in [-1, 1]), TENO8-M-TVD(minmod),
    C_T = 1e-7, to t = min(0.2, 0.45/S_max) so no wave reaches the boundary."""
    left, right = W.riemann_states(seed)
    sl, sr = ER.wave_speeds(left, right)
    t_end = min(0.2, 0.45 / max(abs(sl), abs(sr)))
    e1, U = run_tube(orc, 256, left, right, t_end, 8, 2, 1e-7)
    e2, _ = run_tube(orc, 512, left, right, t_end, 8, 2, 1e-7)
    assert e2 < e1
    assert e1 < 0.02
