"""Pins of the itemised algorithmic operation counts (opcount.py) that the
benchmark's roofline fractions divide by.

* The candidate stencil widths are the nonzero columns of Table 1.
* Each smoothness indicator (Eq. measureTENO) is a positive definite
  quadratic form in the r - 1 adjacent differences of its r points whose
  LDL^T factor is dense, derived here exactly from the definition (the
  polynomial with the given cell averages, sum_j int (p^(j))^2): so the
  weighted sum of n = r - 1 squares with n(n-1)/2 multiply-adds inside the
  squares is what the method needs, no term can be dropped, and
  opcount.beta_ops counts exactly that evaluation.
* The totals of the configurations the benchmark reports are fixed so that
  a change to an item shows up in review.
"""
from fractions import Fraction as Fr

import pytest

from exact_poly import cell_avg_poly, js_beta_of_poly, solve
from fixtures import table1
from paper_2010_13289_amd import opcount as O


def test_stencil_widths_are_table1s():
    rows = table1()
    for K, pts in O.STENCIL_POINTS.items():
        assert len(pts) == K - 2
        for k, r in enumerate(pts):
            assert sum(1 for c in rows[k] if c != 0) == r, (K, k)


def beta_gram_in_differences(r):
    """Exact matrix Q with beta(v) = x^T Q x, x the r - 1 adjacent
    differences of the r cell averages v (v_0 = 0)."""
    n = r - 1

    def beta_of_differences(x):
        v = [Fr(0)]
        for d in x:
            v.append(v[-1] + d)
        # polynomial of degree r - 1 with these cell averages on cells 0..r-1
        A = [[cell_avg_poly([0] * l + [1], m) for l in range(r)] for m in range(r)]
        coefs = solve(A, v)
        return js_beta_of_poly(coefs, r)

    e = [[Fr(int(i == j)) for j in range(n)] for i in range(n)]
    diag = [beta_of_differences(e[i]) for i in range(n)]
    Q = [[Fr(0)] * n for _ in range(n)]
    for i in range(n):
        Q[i][i] = diag[i]
        for j in range(i + 1, n):
            both = beta_of_differences([e[i][k] + e[j][k] for k in range(n)])
            Q[i][j] = Q[j][i] = (both - diag[i] - diag[j]) / 2
    return Q


def ldlt(Q):
    n = len(Q)
    L = [[Fr(int(i == j)) for j in range(n)] for i in range(n)]
    D = [Fr(0)] * n
    for j in range(n):
        D[j] = Q[j][j] - sum(L[j][k] ** 2 * D[k] for k in range(j))
        for i in range(j + 1, n):
            L[i][j] = (Q[i][j] - sum(L[i][k] * L[j][k] * D[k] for k in range(j))) / D[j]
    return L, D


@pytest.mark.parametrize("r", [3, 4, 5, 6, 8])
def test_indicator_forms_are_dense_and_definite(r):
    Q = beta_gram_in_differences(r)
    # a known value: linear data (every difference 1) has beta = 1
    n = r - 1
    assert sum(Q[i][j] for i in range(n) for j in range(n)) == 1
    L, D = ldlt(Q)
    assert all(d > 0 for d in D), D                       # rank n: n squares are needed
    assert all(L[i][j] != 0 for i in range(n) for j in range(i)), L  # no multiply-add can be dropped
    # the evaluation opcount.beta_ops counts: the n - 1 - l multiply-adds
    # of each y_l, a square and a weight per y_l, the additions fused
    fmas_inside = n * (n - 1) // 2
    assert O.beta_ops(r) == 2 * fmas_inside + 2 * n + (n - 1)


def test_reconstruction_totals():
    assert O.reconstruction_ops(6, O.LIM_MP) == 188
    assert O.reconstruction_ops(8, O.LIM_MP) == 291
    assert O.reconstruction_ops(8, O.LIM_MP, adaptive=True) == 346
    assert O.reconstruction_ops(6, O.LIM_TENO) == 140
    # d^MM needs fewer operations than d^M4, beta does not change the count
    assert O.reconstruction_ops(6, O.LIM_MP_MM_B4) < O.reconstruction_ops(6, O.LIM_MP)
    assert O.reconstruction_ops(6, O.LIM_MP_MM_B1) == O.reconstruction_ops(6, O.LIM_MP_MM_B4)


def test_face_vector_totals_of_the_benchmarked_configurations():
    # 3D Euler, six points, MP: the timed step
    items = O.face_vector_items("euler", 3, 6, O.LIM_MP)
    assert items["reconstructions"] == 10 * 188
    assert items["projections"] == 12 * 22
    assert O.face_vector_ops("euler", 3, 6, O.LIM_MP) == pytest.approx(2362.5556, abs=1e-3)
    # 1D Euler, eight points, MP: the batched sweep
    assert O.face_vector_ops("euler", 1, 8, O.LIM_MP) == 2135
    # 2D Euler, six points, MP: the adjoint workload's forward and its VJP
    assert O.face_vector_ops("euler", 2, 6, O.LIM_MP) == pytest.approx(1900.6667, abs=1e-3)
    assert O.adjoint_face_vector_ops(2, 6, O.LIM_MP) == pytest.approx(3305.3333, abs=1e-3)
    assert O.rk3_bytes_per_cell(5) == 320


def test_every_variant_has_a_count():
    for K in (6, 8):
        for lim in range(9):
            for adaptive in ((False, True) if K == 8 else (False,)):
                assert O.face_vector_ops("euler", 3, K, lim, adaptive) > 0
    with pytest.raises(ValueError):
        O.reconstruction_ops(6, 9)


def test_measured_limiter_share():
    """The limiter counted where the data need it: every candidate nonsmooth
    gives the full count, none gives the count without the limiter's items,
    and the count is linear in the shares in between."""
    for K, lim, nk in ((6, O.LIM_MP, 4), (8, O.LIM_MP, 6), (8, O.LIM_TVD5, 6), (6, O.LIM_VA, 4)):
        full = O.face_vector_ops("euler", 3, K, lim)
        assert O.face_vector_ops("euler", 3, K, lim, rough=1.0, nonsmooth=nk) == pytest.approx(full)
        rec = O.reconstruction_items(K, lim)
        lim_items = sum(v for k, v in rec.items() if k in ("mp_bounds", "medians", "tvd_flux"))
        none = O.face_vector_ops("euler", 3, K, lim, rough=0.0, nonsmooth=0.0)
        assert none == pytest.approx(full - 2 * 5 * lim_items)
        half = O.face_vector_ops("euler", 3, K, lim, rough=0.5, nonsmooth=nk / 2)
        assert half == pytest.approx((full + none) / 2)
    # MP six points: 46 for the bounds and 2 per clamped candidate
    assert O.reconstruction_ops(6, O.LIM_MP, rough=0.25, nonsmooth=0.5) == pytest.approx(188 - 54 + 0.25 * 46 + 1)
    assert O.adjoint_face_vector_ops(2, 6, O.LIM_MP, rough=1.0, nonsmooth=4) == pytest.approx(
        O.adjoint_face_vector_ops(2, 6, O.LIM_MP))
    with pytest.raises(ValueError):
        O.reconstruction_ops(6, O.LIM_MP, rough=0.1)
    with pytest.raises(ValueError):
        O.reconstruction_ops(6, O.LIM_MP, rough=0.1, nonsmooth=0.5)  # more nonsmooth candidates than 4 x rough


def test_limiter_share_from_flags():
    import numpy as np
    # four reconstructions of six points: all smooth, one nonsmooth, all nonsmooth, two nonsmooth
    flags = np.array([0b1111, 0b1110, 0b0000, 0b0101], dtype=np.uint8)
    rough, nonsmooth = O.limiter_share(flags, 4)
    assert rough == 0.75
    assert nonsmooth == (0 + 1 + 4 + 2) / 4
    # bits above the candidates are ignored
    assert O.limiter_share(np.array([0xFF, 0xF0], dtype=np.uint8), 4) == (0.5, 2.0)
