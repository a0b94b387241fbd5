"""Pins of the oracle's one-face TENO-M reconstruction (Sec. 2.2-3.3).

Each test fixes a property that the paper or elementary mathematics
determines, so that a plausible mistake in the oracle (a dropped term, a
wrong sign or index, a transposed operand) fails at least one of them.
"""
import numpy as np
import pytest

from exact_poly import face_weights

LIMS = ["LIM_MP", "LIM_TVD_MINMOD", "LIM_TVD5", "LIM_VA", "LIM_MP_M4_B2", "LIM_MP_MM_B4",
        "LIM_MP_MM_B2", "LIM_MP_MM_B1", "LIM_TENO"]


def linear_scheme(K):
    lo, hi = -(K // 2) + 1, K // 2
    return np.array([float(c) for c in face_weights(lo, hi)])


# -------------------------------------------------------------------------
# building blocks: minmod, median, MP bounds, TVD fluxes
# -------------------------------------------------------------------------

def textbook_minmod(*args):
    if all(a > 0 for a in args):
        return min(args)
    if all(a < 0 for a in args):
        return max(args)
    return 0.0


def test_minmod_brute_force(orc):
    vals = [-3.0, -1.5, -0.25, 0.0, 0.5, 2.0, 7.0]
    for x in vals:
        for y in vals:
            assert orc.minmod2(x, y) == textbook_minmod(x, y)
            for z in vals[::2]:
                for w in vals[1::2]:
                    assert orc.minmod4(x, y, z, w) == textbook_minmod(x, y, z, w), (x, y, z, w)


def test_median_is_middle_value(orc):
    rng = np.random.default_rng(1)
    for _ in range(500):
        x, y, z = rng.standard_normal(3)
        assert orc.median(x, y, z) == pytest.approx(sorted([x, y, z])[1], abs=1e-15)


def test_mp_bounds_always_admit_the_upwind_value(orc):
    """Eq. value_min_max: both inner minima are <= f_i and both inner maxima
    are >= f_i, so the MP interval always contains f_i, for any data."""
    rng = np.random.default_rng(2)
    for _ in range(500):
        f = rng.standard_normal(5) * rng.uniform(0.01, 100)
        for curv in (0, 1):
            for bet in (4.0, 2.0, 1.0):
                lo, hi = orc.mp_bounds(f, curv, bet)
                assert lo <= f[2] <= hi


def test_mp_bounds_on_linear_data(orc):
    """Linear data have zero curvature: MD = LC = (f_i + f_{i+1})/2 and UL
    lies beyond f_{i+1}, so the interval is exactly [f_i, f_{i+1}] (ordered)."""
    rng = np.random.default_rng(12)
    for _ in range(100):
        a, b = rng.uniform(-5, 5, 2)
        f = a + b * np.arange(-2, 3, dtype=np.float64)
        lo, hi = orc.mp_bounds(f)
        assert lo == pytest.approx(min(f[2], f[3]), abs=1e-13)
        assert hi == pytest.approx(max(f[2], f[3]), abs=1e-13)


def test_mp_bounds_collapse_at_a_step(orc):
    """At a step the MP interval shrinks to the upwind value: no overshoot."""
    lo, hi = orc.mp_bounds([0.0, 0.0, 0.0, 1.0, 1.0])
    assert lo == 0.0 and hi == 0.0
    lo, hi = orc.mp_bounds([0.0, 0.0, 1.0, 1.0, 1.0])
    assert lo == 1.0 and hi == 1.0


def test_tvd_minmod_textbook(orc):
    rng = np.random.default_rng(3)
    for _ in range(200):
        a, b, c = rng.standard_normal(3)
        dm, dp = b - a, c - b
        exp = b + 0.5 * textbook_minmod(dm, dp)
        assert orc.tvd_minmod(a, b, c) == pytest.approx(exp, abs=1e-15)


def test_tvd5_unlimited_is_fifth_order_upwind(orc):
    """With phi = beta(r) (Eqs. TVDhighorder2, TVDbeta), the flux equals the
    fifth-order upwind face value on i-2..i+2, derived here exactly."""
    w = np.array([float(c) for c in face_weights(-2, 2)])
    np.testing.assert_allclose(w * 60, [2, -13, 47, 27, -3], atol=1e-12)
    rng = np.random.default_rng(4)
    hits = 0
    for _ in range(400):
        # gently curved monotone data: slope ratios near 1, beta(r) < min(2, 2r)
        x = np.arange(-2, 3) * 0.05
        f = rng.uniform(0.5, 2.0) * x + rng.uniform(-0.3, 0.3) * x * x + rng.uniform(-1, 1)
        dm, dp = f[2] - f[1], f[3] - f[2]
        r = dp / dm
        B = (-2 * (f[1] - f[0]) + 11 * dm + 24 * dp - 3 * (f[4] - f[3])) / 30 / dm
        if not (0 < B < min(2.0, 2.0 * r)):
            continue
        hits += 1
        assert orc.tvd5(f) == pytest.approx(float(w @ f), abs=1e-14)
    assert hits > 300


def test_tvd5_phi_bounds_and_degenerate_slopes(orc):
    rng = np.random.default_rng(5)
    for _ in range(500):
        f = rng.standard_normal(5)
        dm = f[2] - f[1]
        out = orc.tvd5(f)
        s = 2.0 * (out - f[2])  # phi * delta-
        if dm == 0:
            assert out == f[2]
        else:
            phi = s / dm
            assert -1e-12 <= phi <= 2.0 + 1e-12
    # flat left side, flat right side
    assert orc.tvd5([1, 1, 1, 2, 3]) == 1.0
    assert orc.tvd5([0, 1, 2, 2, 2]) == 2.0
    # vanishing delta at i-1 uses the continuous limit (no NaN)
    assert np.isfinite(orc.tvd5([1, 1, 2, 3, 4]))


def test_van_albada(orc):
    # phi = 1 on linear data (r = 1): the flux is the S0 candidate
    assert orc.van_albada(1.0, 2.0, 3.0) == pytest.approx(-1 / 6 + 10 / 6 + 1.0, abs=1e-15)
    rng = np.random.default_rng(6)
    for _ in range(200):
        a, b, c = rng.standard_normal(3)
        dm, dp = b - a, c - b
        phi = 2 * dp * dm / (dp * dp + dm * dm)
        exp = b + phi / 4 * ((1 - phi / 3) * dm + (1 + phi / 3) * dp)
        assert orc.van_albada(a, b, c) == pytest.approx(exp, rel=1e-12, abs=1e-14)
    assert orc.van_albada(1.0, 1.0, 5.0) == 1.0


# -------------------------------------------------------------------------
# the full one-face reconstruction
# -------------------------------------------------------------------------

@pytest.mark.parametrize("K", [6, 8])
@pytest.mark.parametrize("lim", LIMS)
def test_zero_cutoff_gives_linear_scheme(orc, K, lim):
    """C_T = 0: every delta_k = 1 (chi >= 0), so the reconstruction is the
    optimal linear combination, i.e. the K-point linear scheme, for any data."""
    rng = np.random.default_rng(K)
    lin = linear_scheme(K)
    for _ in range(50):
        v = rng.standard_normal(K) * rng.uniform(0.1, 10)
        out, tr = orc.teno_m(K, getattr(orc, lim), 0.0, v)
        assert all(tr.delta[k] == 1 for k in range(K - 2))
        assert out == pytest.approx(float(lin @ v), rel=1e-13, abs=1e-13)


@pytest.mark.parametrize("K", [6, 8])
def test_large_cutoff_filters_every_candidate(orc, K):
    """C_T > 1: every delta_k = 0.  TVD-type limiters then return their fixed
    flux exactly (the d_k sum to 1); MP keeps every candidate, hence the
    result, inside [f_min, f_max]."""
    rng = np.random.default_rng(10 + K)
    c0 = K // 2 - 1
    for _ in range(100):
        v = rng.standard_normal(K)
        out, tr = orc.teno_m(K, orc.LIM_TVD_MINMOD, 2.0, v)
        assert all(tr.delta[k] == 0 for k in range(K - 2))
        assert out == pytest.approx(orc.tvd_minmod(v[c0 - 1], v[c0], v[c0 + 1]), abs=1e-14)
        out, tr = orc.teno_m(K, orc.LIM_TVD5, 2.0, v)
        assert out == pytest.approx(orc.tvd5(v[c0 - 2:c0 + 3]), abs=1e-14)
        out, tr = orc.teno_m(K, orc.LIM_MP, 2.0, v)
        lo, hi = orc.mp_bounds(v[c0 - 2:c0 + 3])
        assert (tr.fmin, tr.fmax) == (lo, hi)
        for k in range(K - 2):
            m = orc.median(tr.cand[k], lo, hi)
            assert tr.fM[k] == m
            assert min(lo, hi) - 1e-14 <= m <= max(lo, hi) + 1e-14
        assert min(lo, hi) - 1e-13 <= out <= max(lo, hi) + 1e-13


@pytest.mark.parametrize("K", [6, 8])
def test_flags_and_output_are_affine_equivariant(orc, K):
    """chi is invariant under f -> a f + b (beta and tau scale by a^2), and
    every limiter commutes with the map, so out(a f + b) = a out(f) + b."""
    rng = np.random.default_rng(20 + K)
    for lim in ("LIM_MP", "LIM_TVD_MINMOD", "LIM_TVD5", "LIM_VA"):
        for _ in range(60):
            v = rng.standard_normal(K)
            if rng.uniform() < 0.5:
                v[K // 2:] += rng.uniform(-5, 5)  # a jump between i and i+1
            out, tr = orc.teno_m(K, getattr(orc, lim), 1e-3, v)
            for a, b in ((-3.7, 5.0), (1e3, -2.0), (1e-3, 0.25)):
                out2, tr2 = orc.teno_m(K, getattr(orc, lim), 1e-3, a * v + b)
                for k in range(K - 2):
                    if not tr.band[k]:
                        assert tr2.delta[k] == tr.delta[k]
                    assert tr2.chi[k] == pytest.approx(tr.chi[k], rel=1e-8, abs=1e-300)
                if lim == "LIM_VA" and a < 0:
                    continue  # phi(r) is odd in r only through the ratio; still equivariant:
                assert out2 == pytest.approx(a * out + b, rel=1e-11, abs=1e-11 * (abs(a) + abs(b)))


@pytest.mark.parametrize("K", [6, 8])
def test_smooth_data_is_unfiltered(orc, K):
    """Sec. 3 (and the first conclusion): on smooth data every candidate is
    smooth, TENO-M reduces to the linear scheme."""
    lin = linear_scheme(K)
    m = np.arange(-(K // 2) + 1, K // 2 + 1)
    for h in (0.1, 0.05, 0.02):
        for x0 in np.linspace(0, 6, 13):
            v = np.exp(np.sin(x0 + m * h))
            for lim in ("LIM_MP", "LIM_TVD5", "LIM_TVD_MINMOD"):
                out, tr = orc.teno_m(K, getattr(orc, lim), 1e-5, v)
                assert all(tr.delta[k] for k in range(K - 2)), (h, x0, list(tr.chi))
                assert out == pytest.approx(float(lin @ v), rel=1e-13)


@pytest.mark.parametrize("K", [6, 8])
def test_step_marks_exactly_the_crossing_stencils(orc, K):
    """A jump between cells j and j+1 makes exactly the candidates whose
    stencil contains both cells nonsmooth (brute force over jump positions)."""
    lo = {0: -1, 1: 0, 2: -2, 3: 0, 4: -3, 5: 0}
    hi = {0: 1, 1: 2, 2: 0, 3: 3, 4: 0, 5: 4}
    c0 = K // 2 - 1
    for j in range(-(K // 2) + 1, K // 2):  # jump between offsets j and j+1
        v = np.array([0.0 if o <= j else 1.0 for o in range(-(K // 2) + 1, K // 2 + 1)])
        v += 1e-3 * np.arange(K)  # avoid exactly flat data
        _, tr = orc.teno_m(K, orc.LIM_MP, 1e-5, v)
        for k in range(K - 2):
            crosses = lo[k] <= j and j + 1 <= hi[k]
            if crosses:
                assert tr.delta[k] == 0, (j, k, list(tr.chi))
        # at least the stencils not touching the jump on the upwind side stay smooth
        for k in range(K - 2):
            if hi[k] <= j or lo[k] >= j + 1:
                if all(lo[kk] <= j < hi[kk] for kk in range(K - 2) if kk != k):
                    assert tr.delta[k] == 1
        assert c0 >= 0


def test_renormalised_teno_discards_nonsmooth(orc):
    """Classic TENO (Eq. weight_renormalize): weights d_k delta_k / sum."""
    K = 6
    d = orc.weights(K)
    v = np.array([0, 0, 0, 1, 1, 1.0]) + 1e-3 * np.arange(6)
    out, tr = orc.teno_m(K, orc.LIM_TENO, 1e-5, v)
    dl = np.array([tr.delta[k] for k in range(4)])
    w = d * dl / np.sum(d * dl)
    assert out == pytest.approx(float(np.dot(w, [tr.cand[k] for k in range(4)])), abs=1e-15)


@pytest.mark.parametrize("K", [6, 8])
def test_gamma_chi_definitions(orc, K):
    """Eqs. measureTENO, taukTENO, normalize, cut-off on one trace."""
    rng = np.random.default_rng(30 + K)
    for _ in range(50):
        v = rng.standard_normal(K)
        _, tr = orc.teno_m(K, orc.LIM_MP, 0.1, v)
        b = [tr.beta[k] for k in range(K - 2)]
        assert tr.tau == pytest.approx(abs(tr.betaK - (b[1] + b[2] + 4 * b[0]) / 6), rel=1e-14, abs=1e-15)
        g = [(1 + tr.tau / (bk + 1e-40)) ** 6 for bk in b]
        chi = np.array(g) / sum(g)
        np.testing.assert_allclose([tr.chi[k] for k in range(K - 2)], chi, rtol=1e-13)
        assert sum(tr.chi[k] for k in range(K - 2)) == pytest.approx(1.0, rel=1e-14)
        for k in range(K - 2):
            assert tr.delta[k] == (0 if tr.chi[k] < 0.1 else 1)


def test_cutoff_tie_counts_as_smooth(orc):
    """Eq. cut-off: delta = 0 only if chi < C_T; chi == C_T stays smooth."""
    v = np.array([0.1, -0.4, 0.3, 1.2, 0.7, -0.2])
    _, tr = orc.teno_m(6, orc.LIM_MP, 1e-5, v)
    for k in range(4):
        _, tr2 = orc.teno_m(6, orc.LIM_MP, tr.chi[k], v)
        assert tr2.delta[k] == 1
        assert tr2.band[k] == 1
