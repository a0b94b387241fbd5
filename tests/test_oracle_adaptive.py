"""Pins of the adaptive cutoff (Sec. 2.4, Eqs. shock_indicator and
cut-off_adjust) used by the eight-point TENO8A scheme, and of the limiter
variants of Secs. 3.2.1 and 4 (Van Albada, MP with d^MM and beta 2 or 1,
classic renormalised TENO) at scheme level."""
import numpy as np
import pytest

import workloads as W
from oracle import exact_riemann as ER

A = 8 | 0x100  # eight points, adaptive cutoff


def geometric(r, n=8, d0=1.0):
    """Values whose consecutive differences grow by the factor r."""
    d = d0 * r ** np.arange(n - 1)
    return np.concatenate([[0.0], np.cumsum(d)])


def test_smooth_data_gets_the_smallest_cutoff(orc):
    """eta ~ 1 on smooth data (equal neighbouring differences): m = 0, g = 1,
    beta = alpha_1 = 10.5, C_T = 1e-10."""
    for h in (0.3, 0.1, 0.01):
        v = np.sin(0.4 + h * np.arange(8))
        _, tr = orc.teno_m(A, orc.LIM_MP, 123.0, v)  # the C_T argument is ignored
        assert tr.m == 0.0
        assert tr.ct == 1e-10


def test_discontinuity_gets_the_largest_cutoff(orc):
    """A jump makes one difference dominate its neighbour: eta -> 0, m -> 1,
    g -> 0, beta -> alpha_1 - alpha_2 = 7, C_T = 1e-7."""
    v = np.array([0, 0, 0, 0, 5, 5, 5, 5.0]) + 1e-3 * np.arange(8)
    _, tr = orc.teno_m(A, orc.LIM_MP, 0.0, v)
    assert tr.m > 0.99
    assert tr.ct == 1e-7
    # beta >= 7 holds exactly (g >= 0), so beta -> 7 is no rounding band
    _, tr = orc.teno_m(A, orc.LIM_MP, 0.0, np.array([0, 0, 0, 0, 1, 1, 1, 1.0]))
    assert tr.m == 1.0 - tr.eta / 0.23 and tr.ct == 1e-7 and tr.ct_band == 0


def test_band_marks_the_interior_cutoff_switches(orc):
    """Bisection on the ratio of geometric data to the switch 1e-9 -> 1e-8
    (beta crossing 9): the last point below and the first above differ in
    C_T and lie in the band; points well away from it do not."""
    lo, hi = 1.0, 0.002  # ct(lo) = 1e-10, ct(hi) = 1e-7
    ct = lambda r: orc.teno_m(A, orc.LIM_MP, 0.0, geometric(r, d0=10.0))[1]
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if ct(mid).ct <= 1e-9:
            lo = mid
        else:
            hi = mid
    a, b = ct(lo), ct(hi)
    assert a.ct == 1e-9 and b.ct == 1e-8
    assert a.ct_band == 1 and b.ct_band == 1
    assert ct(0.5 * (lo + 1.0)).ct_band == 0


def test_jumps_below_xi_count_as_smooth(orc):
    """With differences far below xi = 1e-3 the indicator's epsilon dominates
    and eta -> 1: a tiny step keeps the smallest cutoff, the same step at
    unit size gets the largest."""
    step = np.array([0, 0, 0, 0, 1, 1, 1, 1.0])
    _, tr = orc.teno_m(A, orc.LIM_MP, 0.0, 1e-7 * step)
    assert tr.eta == pytest.approx(1.0, abs=1e-6)
    assert tr.ct == 1e-10
    _, tr = orc.teno_m(A, orc.LIM_MP, 0.0, step)
    assert tr.ct == 1e-7


def test_cutoff_is_monotone_and_takes_the_four_values(orc):
    """eta = 2r/(1+r^2) for geometric data: the cutoff rises from 1e-10 to
    1e-7 as the ratio departs from 1, through each power of ten."""
    seen = []
    for r in np.linspace(1.0, 0.002, 400):
        _, tr = orc.teno_m(A, orc.LIM_MP, 0.0, geometric(r, d0=10.0))
        seen.append(tr.ct)
    assert seen == sorted(seen)
    assert sorted(set(seen)) == [1e-10, 1e-9, 1e-8, 1e-7]


def test_adaptive_is_eight_point_only(orc):
    import math
    out, _ = orc.teno_m(6 | 0x100, orc.LIM_MP, 0.0, np.arange(6.0))
    assert math.isnan(out)


@pytest.mark.parametrize("lim", [1, 3, 4, 0])
def test_teno8a_sod_converges(orc, lim):
    """TENO8A-M with MP, TVD5, VA and classic TENO8A on Sod (Sec. 4.2.1)."""
    errs = []
    for n in (100, 200):
        U, dx = W.riemann_problem(n, W.SOD[0], W.SOD[1])
        g = dict(ndim=1, n=[n], dx=[dx], bc=[1], system=1)
        t = 0.0
        while t < 0.2 - 1e-14:
            dt = min(0.4 / orc.max_wave_speed(U, g, 1.4), 0.2 - t)
            U = orc.rk3_step(U, g, A, lim, 0.0, 1.4, dt)
            t += dt
        x = W.cell_centres(n, 0.0, 1.0)
        rho, _, _ = ER.sample(W.SOD[0], W.SOD[1], (x - 0.5) / 0.2)
        errs.append(np.mean(np.abs(U[0] - rho)))
    assert errs[0] < 0.02 and errs[1] < 0.75 * errs[0], errs


@pytest.mark.parametrize("lim", [4, 5, 6, 7, 8])
def test_limiter_variants_square_wave(orc, lim):
    """Van Albada and the MP variants keep the square wave within 1e-5 of
    its range (Sec. 4.1.2) and conserve it."""
    n = 100
    u, dx = W.square_wave(n)
    g = dict(ndim=1, n=[n], dx=[dx], bc=[0], system=0, adv=[1.0])
    for _ in range(60):
        u = orc.rk3_step(u, g, 6, lim, 1e-5, 1.4, 0.4 * dx)
    assert u.min() >= -1e-15 and u.max() <= 1.0 + 1e-5
    assert abs(u.sum() * dx - 0.25) < 1e-12


def test_mp_curvature_measures(orc):
    """d^M4 (Eq. maximal_curvature) is the more restrictive measure: it never
    exceeds d^MM = minmod(d_i, d_i+1) (Eq. maximal_curvature1) in size, it
    shares its sign, and it vanishes when d_i+1/d_i leaves (1/4, 4)."""
    rng = np.random.default_rng(17)
    for _ in range(500):
        a, b = rng.standard_normal(2)
        m4 = orc.minmod4(4 * a - b, 4 * b - a, a, b)
        mm = orc.minmod2(a, b)
        assert abs(m4) <= abs(mm) + 1e-15
        assert m4 == 0.0 or np.sign(m4) == np.sign(mm)
        if a * b > 0 and not (0.25 < b / a < 4.0):
            assert m4 == 0.0
    # the variants give different bounds somewhere, each still brackets f_i
    differ = 0
    for _ in range(300):
        f = rng.standard_normal(5)
        b = [orc.mp_bounds(f, c, beta) for c, beta in ((0, 4.0), (0, 2.0), (1, 4.0), (1, 2.0), (1, 1.0))]
        differ += len(set(b)) > 1
        assert all(lo <= f[2] <= hi for lo, hi in b)
    assert differ > 50
