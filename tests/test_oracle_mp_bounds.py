"""Exact pins of the oracle's MP bounds (Sec. 3.2.2).

The bounds of Eqs. curvature, maximal_curvature (d^M4) or maximal_curvature1
(d^MM), upper_limiter (alpha = 1.25), median_value, large_curvature (beta/3)
and value_min_max are evaluated by hand on four 5-point data sets
f_{i-2..i+2}.  The data are chosen so that each of UL, MD and LC is in turn
the active bound, and so that d_{i+1/2} and d_{i-1/2} differ and are nonzero
where MD or LC is active.  The worked values below were done in exact
fractions; the oracle must reproduce them to rounding, and a plausible
misreading (alpha = 1.5, beta/2 instead of beta/3, the two interface
curvatures swapped between MD and LC, d^M4 and d^MM exchanged, or a limiter
ID mapped to the wrong beta) moves at least one of them by far more than
rounding.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

from fixtures import table1

# f_{i-2..i+2}; (curvature measure, beta) -> exact (f_min, f_max).
# curvature measure 0 = d^M4 (Eq. maximal_curvature), 1 = d^MM (Eq.
# maximal_curvature1).
#
# A = (-8, -8, -7, -2, -4): d_{i-1} = -7+16-8 = 1, d_i = -2+14-8 = 4,
#   d_{i+1} = -4+4-7 = -7.  d^M4_{i+1/2} = minmod(23, -32, 4, -7) = 0,
#   d^M4_{i-1/2} = minmod(0, 15, 1, 4) = 0.  UL = -7 + 1.25 = -23/4,
#   MD = (-7-2)/2 = -9/2, LC = -7 + 1/2 = -13/2.
#   f_min = max(min(-7, -2, -9/2), min(-7, -23/4, -13/2)) = -7,
#   f_max = min(max(-7, -2, -9/2), max(-7, -23/4, -13/2)) = -23/4 (UL).
#   With d^MM: d_{i-1/2} = minmod(1, 4) = 1, LC = -13/2 + beta/3, so for
#   beta = 4 LC = -31/6 > UL is the larger inner maximum: f_max = -31/6.
# B = (-2, -4, -5, -4, -1): d = (1, 2, 2).  d^M4_{i+1/2} = minmod(6, 6, 2, 2)
#   = 2, d^M4_{i-1/2} = minmod(2, 7, 1, 2) = 1.  UL = -5 - 5/4 = -25/4,
#   MD = -9/2 - 1 = -11/2, LC = -5 - 1/2 + 4/3 = -25/6.
#   f_min = max(min(-5, -4, -11/2), min(-5, -25/4, -25/6)) = -11/2 (MD),
#   f_max = min(max(-5, -4, -11/2), max(-5, -25/4, -25/6)) = -25/6 (LC).
# C = (-5, -2, 0, -1, -5): d = (-1, -3, -3).  d^M4_{i+1/2} =
#   minmod(-9, -9, -3, -3) = -3, d^M4_{i-1/2} = minmod(-1, -11, -1, -3) = -1.
#   UL = 5/2, MD = -1/2 + 3/2 = 1, LC = 0 + 1 - 4/3 = -1/3.
#   f_min = max(min(0, -1, 1), min(0, 5/2, -1/3)) = -1/3 (LC),
#   f_max = min(max(0, -1, 1), max(0, 5/2, -1/3)) = 1 (MD).
# D = (0, 0, 1, 7, 18): d = (1, 5, 5); the ratio 5 > 4 makes d^M4 and d^MM
#   differ at i-1/2: d^M4_{i-1/2} = minmod(-1, 19, 1, 5) = 0 but
#   d^MM_{i-1/2} = minmod(1, 5) = 1; d_{i+1/2} = 5 for both.  UL = 9/4,
#   MD = 4 - 5/2 = 3/2, LC = 3/2 (d^M4) or 3/2 + beta/3 (d^MM).
#   d^M4: f_min = 1, f_max = min(7, max(1, 9/4, 3/2)) = 9/4 (UL);
#   d^MM, beta = 4: f_max = min(7, max(1, 9/4, 17/6)) = 17/6 (LC).
WORKED = {
    "A": ((-8, -8, -7, -2, -4), {
        (0, 4): ("-7", "-23/4"), (0, 2): ("-7", "-23/4"), (0, 1): ("-7", "-23/4"),
        (1, 4): ("-7", "-31/6"), (1, 2): ("-7", "-23/4"), (1, 1): ("-7", "-23/4")}),
    "B": ((-2, -4, -5, -4, -1), {
        (0, 4): ("-11/2", "-25/6"), (0, 2): ("-11/2", "-29/6"), (0, 1): ("-11/2", "-5"),
        (1, 4): ("-11/2", "-25/6"), (1, 2): ("-11/2", "-29/6"), (1, 1): ("-11/2", "-5")}),
    "C": ((-5, -2, 0, -1, -5), {
        (0, 4): ("-1/3", "1"), (0, 2): ("0", "1"), (0, 1): ("0", "1"),
        (1, 4): ("-1/3", "1"), (1, 2): ("0", "1"), (1, 1): ("0", "1")}),
    "D": ((0, 0, 1, 7, 18), {
        (0, 4): ("1", "9/4"), (0, 2): ("1", "9/4"), (0, 1): ("1", "9/4"),
        (1, 4): ("1", "17/6"), (1, 2): ("1", "9/4"), (1, 1): ("1", "9/4")}),
}
COMBOS = [(c, b) for c in (0, 1) for b in (4, 2, 1)]

# C-ABI / oracle limiter IDs of the MP family -> (curvature measure, beta)
MP_IDS = {1: (0, 4), 5: (0, 2), 6: (1, 4), 7: (1, 2), 8: (1, 1)}


def _minmod(*a):
    """Smallest-magnitude argument if all share a strict sign, else 0."""
    if all(x > 0 for x in a):
        return min(a)
    if all(x < 0 for x in a):
        return max(a)
    return Fr(0)


def exact_parts(f, curv, beta, alpha=Fr(5, 4), lc_div=3, swap=False, curv_of_lc=None):
    """Eqs. curvature .. value_min_max in exact fractions: UL, MD, LC and
    the bounds.  The keyword arguments plant one misreading each (alpha, the
    beta divisor, the two interface curvatures exchanged, or another
    curvature measure for LC)."""
    fm2, fm1, f0, fp1, fp2 = (Fr(x) for x in f)
    d_m, d_0, d_p = f0 - 2 * fm1 + fm2, fp1 - 2 * f0 + fm1, fp2 - 2 * fp1 + f0

    def at_faces(c):
        if c == 0:
            return (_minmod(4 * d_0 - d_p, 4 * d_p - d_0, d_0, d_p),
                    _minmod(4 * d_m - d_0, 4 * d_0 - d_m, d_m, d_0))
        return _minmod(d_0, d_p), _minmod(d_m, d_0)

    d_r, d_l = at_faces(curv)
    if curv_of_lc is not None:
        d_l = at_faces(curv_of_lc)[1]
    if swap:
        d_r, d_l = d_l, d_r
    ul = f0 + alpha * (f0 - fm1)
    md = (f0 + fp1) / 2 - d_r / 2
    lc = f0 + (f0 - fm1) / 2 + Fr(beta, lc_div) * d_l
    lo = max(min(f0, fp1, md), min(f0, ul, lc))
    hi = min(max(f0, fp1, md), max(f0, ul, lc))
    return dict(ul=ul, md=md, lc=lc, lo=lo, hi=hi, d_r=d_r, d_l=d_l, f0=f0, fp1=fp1)


def exact_bounds(f, curv, beta, **misreading):
    p = exact_parts(f, curv, beta, **misreading)
    return p["lo"], p["hi"]


def _close(x, exact, scale):
    return abs(x - float(exact)) <= 4e-16 * scale


def test_exact_evaluation_reproduces_the_worked_values():
    for name, (f, table) in WORKED.items():
        for (curv, beta), (lo, hi) in table.items():
            assert exact_bounds(f, curv, beta) == (Fr(lo), Fr(hi)), (name, curv, beta)


@pytest.mark.parametrize("name", sorted(WORKED))
def test_oracle_mp_bounds_equal_the_worked_values(orc, name):
    f, table = WORKED[name]
    scale = max(abs(x) for x in f)
    for (curv, beta), (lo, hi) in table.items():
        glo, ghi = orc.mp_bounds(f, curv, float(beta))
        assert _close(glo, Fr(lo), scale) and _close(ghi, Fr(hi), scale), (name, curv, beta, glo, ghi)


def test_each_bound_is_active_somewhere():
    """UL, MD and LC each set f_min or f_max alone in some worked case; MD
    and LC each set both bounds in cases where d_{i+1/2} and d_{i-1/2} are
    nonzero and differ."""
    active = set()
    for f, table in WORKED.values():
        for curv, beta in table:
            p = exact_parts(f, curv, beta)
            for bound in ("lo", "hi"):
                hits = [k for k in ("ul", "md", "lc", "f0", "fp1") if p[k] == p[bound]]
                distinct = p["d_r"] != p["d_l"] and p["d_r"] != 0 and p["d_l"] != 0
                if len(hits) == 1 and (hits[0] == "ul" or (hits[0] in ("md", "lc") and distinct)):
                    active.add((hits[0], bound))
    assert {k for k, _ in active} == {"ul", "md", "lc"}
    assert ("md", "lo") in active and ("md", "hi") in active
    assert ("lc", "lo") in active and ("lc", "hi") in active


MISREADINGS = {
    "alpha = 1.5": dict(alpha=Fr(3, 2)),
    "beta / 2": dict(lc_div=2),
    "curvatures swapped": dict(swap=True),
}


@pytest.mark.parametrize("what", sorted(MISREADINGS))
@pytest.mark.parametrize("curv", [0, 1])
def test_misreadings_move_a_worked_value(orc, what, curv):
    """For either curvature measure, each misreading changes at least one
    worked value by far more than rounding, so an oracle that matches the
    worked values cannot carry it."""
    moved = 0.0
    for f, table in WORKED.values():
        for (c, beta), (lo, hi) in table.items():
            if c != curv:
                continue
            mlo, mhi = exact_bounds(f, c, beta, **MISREADINGS[what])
            moved = max(moved, abs(float(mlo - Fr(lo))), abs(float(mhi - Fr(hi))))
            glo, ghi = orc.mp_bounds(f, c, float(beta))
            assert _close(glo, Fr(lo), 20) and _close(ghi, Fr(hi), 20)
    assert moved > 0.1, what


def test_curvature_measures_and_betas_are_distinguished():
    """d^M4 and d^MM, and beta 4 / 2 / 1, give different worked values."""
    f, table = WORKED["D"]
    assert table[(0, 4)] != table[(1, 4)]
    assert exact_bounds(f, 1, 4, curv_of_lc=0) != exact_bounds(f, 1, 4)
    f, table = WORKED["B"]
    assert len({table[(0, b)] for b in (4, 2, 1)}) == 3


def test_mp_bounds_match_exact_evaluation_on_random_rational_data(orc):
    rng = np.random.default_rng(3202)
    for _ in range(3000):
        den = int(rng.choice([1, 2, 4, 8]))
        f = [Fr(int(v), den) for v in rng.integers(-40, 41, 5)]
        scale = max(1.0, max(abs(float(x)) for x in f))
        for curv, beta in COMBOS:
            lo, hi = exact_bounds(f, curv, beta)
            glo, ghi = orc.mp_bounds([float(x) for x in f], curv, float(beta))
            assert _close(glo, lo, 4 * scale) and _close(ghi, hi, 4 * scale), (f, curv, beta)


EXACT_D = {6: [Fr(9, 20), Fr(3, 10), Fr(1, 20), Fr(1, 5)],
           8: [Fr(3, 7), Fr(9, 35), Fr(2, 35), Fr(6, 35), Fr(1, 70), Fr(1, 14)]}


@pytest.mark.parametrize("K", [6, 8])
@pytest.mark.parametrize("lim", sorted(MP_IDS))
def test_mp_limiter_ids_inside_the_reconstruction(orc, K, lim):
    """With C_T > 1 every candidate is nonsmooth, so the TENO-M output is
    sum_k d_k median(f_k, f_min, f_max) (Eqs. mp_flux, value_monotonicity_
    preserving, reconstuction) with the bounds of the limiter ID's
    curvature measure and beta.  Table 1 candidates and the weights are
    exact fractions here."""
    curv, beta = MP_IDS[lim]
    rows = table1()
    for name, (f5, table) in WORKED.items():
        # K-point window f_{i-K/2+1..i+K/2} around the worked 5 points
        pad_l = [f5[0] - 3, f5[0] + 1][: K // 2 - 3]
        pad_r = [f5[-1] + 2, f5[-1] - 5][: K // 2 - 2]
        v = [Fr(x) for x in list(reversed(pad_l)) + list(f5) + pad_r]
        assert len(v) == K
        c0 = K // 2 - 1
        lo, hi = (Fr(x) for x in table[(curv, beta)])
        expect = Fr(0)
        for k in range(K - 2):
            cand = sum(rows[k][off + 3] * v[c0 + off] for off in range(-3, 5) if 0 <= c0 + off < K)
            expect += EXACT_D[K][k] * min(max(cand, lo), hi)
        out, tr = orc.teno_m(K, lim, 2.0, np.array([float(x) for x in v]))
        assert all(tr.delta[k] == 0 for k in range(K - 2))
        scale = max(abs(float(x)) for x in v)
        assert _close(tr.fmin, lo, scale) and _close(tr.fmax, hi, scale), (name, tr.fmin, tr.fmax)
        assert abs(out - float(expect)) <= 1e-14 * scale, (name, out, float(expect))
