"""Pins of the oracle's constants against the paper and exact arithmetic.

* Table 1 (Sec. 3.1) is read from a golden fixture; every row must reproduce
  the face value of every polynomial of degree r_k - 1 exactly (Eqs.
  definitionEq and approximatepolynomial), and the oracle's candidate fluxes
  must equal the printed rows.
* The optimal weights d_k (Sec. 3.3, read as the maximum-order weights) and
  the full-stencil linear schemes are re-derived exactly from polynomial
  exactness conditions and compared with the oracle's floating-point values.
* The smoothness indicator (Sec. 2.2, second Eq. measureTENO) is checked
  against the exact measure of known polynomials, the textbook Jiang-Shu
  form on 3-point stencils, and its invariances.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

from exact_poly import (cell_avg_poly, face_weights, js_beta_of_poly, poly_eval, solve)
from fixtures import table1

STENCILS = {0: (-1, 1), 1: (0, 2), 2: (-2, 0), 3: (0, 3), 4: (-3, 0), 5: (0, 4)}


def test_table1_rows_are_exact_for_their_polynomial_degree():
    rows = table1()
    assert sorted(rows) == list(range(6))
    for k, (lo, hi) in STENCILS.items():
        r = hi - lo + 1
        coef = rows[k]
        # no entries outside the stencil
        for off in range(-3, 5):
            if not lo <= off <= hi:
                assert coef[off + 3] == 0, (k, off)
        for deg in range(r):
            mono = [0] * deg + [1]
            approx = sum(coef[m + 3] * cell_avg_poly(mono, m) for m in range(lo, hi + 1))
            assert approx == poly_eval(mono, Fr(1, 2)), (k, deg)
        # degree r is not reproduced (the order is exactly r)
        mono = [0] * r + [1]
        approx = sum(coef[m + 3] * cell_avg_poly(mono, m) for m in range(lo, hi + 1))
        assert approx != poly_eval(mono, Fr(1, 2))


@pytest.mark.parametrize("K", [6, 8])
def test_oracle_candidates_equal_table1(orc, K):
    rows = table1()
    h = K // 2
    for j in range(K):
        v = np.zeros(K)
        v[j] = 1.0
        _, tr = orc.teno_m(K, orc.LIM_MP, 0.0, v)
        off = j - h + 1
        for k in range(K - 2):
            assert tr.cand[k] == pytest.approx(float(rows[k][off + 3]), abs=1e-15)


def exact_weights(K):
    """d_k such that sum_k d_k f_k reproduces degree K-1 polynomials (exact)."""
    rows = table1()
    nk = K - 2
    lo, hi = -(K // 2) + 1, K // 2
    # exactness for monomials of degree 0..nk-1 gives a square system; the
    # remaining degrees up to K-1 are then checked.
    def row_apply(k, mono):
        return sum(rows[k][m + 3] * cell_avg_poly(mono, m) for m in range(lo, hi + 1))
    A, b = [], []
    for deg in range(K):
        mono = [0] * deg + [1]
        A.append([row_apply(k, mono) for k in range(nk)])
        b.append(poly_eval(mono, Fr(1, 2)))
    # pick nk independent equations by trying degrees in order
    import itertools
    for sel in itertools.combinations(range(K), nk):
        try:
            d = solve([A[i] for i in sel], [b[i] for i in sel])
        except StopIteration:
            continue
        if all(sum(a * x for a, x in zip(A[i], d)) == b[i] for i in range(K)):
            return d
    raise AssertionError("no consistent weights")


@pytest.mark.parametrize("K", [6, 8])
def test_optimal_weights_are_maximum_order(orc, K):
    d = exact_weights(K)
    assert sum(d) == 1
    assert all(x > 0 for x in d)
    np.testing.assert_allclose(orc.weights(K), [float(x) for x in d], rtol=0, atol=1e-15)


def test_optimal_weights_known_values(orc):
    # the exact solutions of the exactness conditions, for the record
    assert exact_weights(6) == [Fr(9, 20), Fr(3, 10), Fr(1, 20), Fr(1, 5)]
    assert exact_weights(8) == [Fr(3, 7), Fr(9, 35), Fr(2, 35), Fr(6, 35), Fr(1, 70), Fr(1, 14)]


@pytest.mark.parametrize("lo,hi", [(-1, 1), (0, 2), (-2, 0), (0, 3), (-3, 0), (0, 4), (-2, 3), (-3, 4), (-2, 2)])
def test_oracle_face_polynomial_matches_exactness_conditions(orc, lo, hi):
    exact = [float(c) for c in face_weights(lo, hi)]
    np.testing.assert_allclose(orc.poly_face(lo, hi), exact, rtol=0, atol=2e-14)


def test_full_stencil_linear_schemes(orc):
    assert [c * 60 for c in face_weights(-2, 3)] == [1, -8, 37, 37, -8, 1]
    assert [c * 840 for c in face_weights(-3, 4)] == [-3, 29, -139, 533, 533, -139, 29, -3]
    # K-th order: truncation error of the face value on a smooth function
    for K, (lo, hi) in ((6, (-2, 3)), (8, (-3, 4))):
        c = orc.poly_face(lo, hi)
        errs = []
        for h in (0.1, 0.05):
            # point values of f = exp(sin) are read as cell averages of h(x)
            # only to leading order; use an exact primitive instead:
            # h(x) = cos(x) has cell averages (sin(x+h/2)-sin(x-h/2))/h
            m = np.arange(lo, hi + 1)
            avg = (np.sin((m + 0.5) * h + 0.3) - np.sin((m - 0.5) * h + 0.3)) / h
            errs.append(abs(c @ avg - np.cos(0.5 * h + 0.3)))
        order = np.log(errs[0] / errs[1]) / np.log(2.0)
        assert order > K - 0.3, (K, order)


# -------------------------------------------------------------------------
# smoothness indicator
# -------------------------------------------------------------------------

ALL_BETA_STENCILS = list(STENCILS.values()) + [(-2, 3), (-3, 4)]


@pytest.mark.parametrize("lo,hi", ALL_BETA_STENCILS)
def test_beta_of_known_polynomials(orc, lo, hi):
    """Averages of a random polynomial of degree r-1 determine it exactly, so
    beta must equal the exact Jiang-Shu measure of that polynomial."""
    rng = np.random.default_rng(lo * 10 + hi + 100)
    r = hi - lo + 1
    for _ in range(5):
        coefs = [Fr(int(c), int(d)) for c, d in zip(rng.integers(-9, 10, r), rng.integers(1, 5, r))]
        v = np.array([float(cell_avg_poly(coefs, m)) for m in range(lo, hi + 1)])
        exact = float(js_beta_of_poly(coefs, r))
        assert orc.beta(lo, hi, v) == pytest.approx(exact, rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("lo,hi", ALL_BETA_STENCILS)
def test_beta_special_values(orc, lo, hi):
    m = np.arange(lo, hi + 1, dtype=np.float64)
    # constants: exactly zero (differences only)
    assert orc.beta(lo, hi, np.full(m.shape, 3.7)) == 0.0
    # point values m (averages of xi): beta = 1
    assert orc.beta(lo, hi, m) == pytest.approx(1.0, rel=1e-13)
    # averages of xi^2: beta = 13/3 on every stencil
    x2 = np.array([float(cell_avg_poly([0, 0, 1], int(k))) for k in m])
    assert orc.beta(lo, hi, x2) == pytest.approx(13.0 / 3.0, rel=1e-13)
    # quadratic scaling and shift invariance
    rng = np.random.default_rng(7)
    v = rng.standard_normal(m.shape)
    b = orc.beta(lo, hi, v)
    assert orc.beta(lo, hi, -2.5 * v + 11.0) == pytest.approx(6.25 * b, rel=1e-12)


def test_beta_three_point_textbook_form(orc):
    """Jiang-Shu: 13/12 (a - 2b + c)^2 + 1/4 (a - c)^2 for the central
    stencil, and the one-sided variants for S1 and S2."""
    rng = np.random.default_rng(3)
    for _ in range(20):
        a, b, c = rng.standard_normal(3)
        assert orc.beta(-1, 1, [a, b, c]) == pytest.approx(13 / 12 * (a - 2 * b + c) ** 2 + 0.25 * (a - c) ** 2, rel=1e-12)
        # S1 = {i, i+1, i+2}: values (a, b, c)
        assert orc.beta(0, 2, [a, b, c]) == pytest.approx(13 / 12 * (a - 2 * b + c) ** 2 + 0.25 * (3 * a - 4 * b + c) ** 2, rel=1e-12)
        # S2 = {i-2, i-1, i}
        assert orc.beta(-2, 0, [a, b, c]) == pytest.approx(13 / 12 * (a - 2 * b + c) ** 2 + 0.25 * (a - 4 * b + 3 * c) ** 2, rel=1e-12)


@pytest.mark.parametrize("K", [6, 8])
def test_tau_is_sixth_order(orc, K):
    """Eq. taukTENO: tau_K = O(dx^6) on smooth data."""
    taus = []
    hs = [0.2, 0.1, 0.05]
    for h in hs:
        m = np.arange(-(K // 2) + 1, K // 2 + 1)
        v = np.sin(0.7 + m * h) + 0.3 * np.cos(1.1 + 2 * m * h)
        _, tr = orc.teno_m(K, orc.LIM_MP, 1e-5, v)
        taus.append(tr.tau)
    orders = np.log(np.array(taus[:-1]) / np.array(taus[1:])) / np.log(2.0)
    assert np.all(orders > 5.5), orders
    # beta_k themselves are O(dx^2): tau/beta vanishes like dx^4
    assert taus[-1] < 1e-6
