"""Generate teno_tables.h: the exact-rational constants of the TENO-M
reconstruction, as straight-line device code in difference form.

Everything is written in terms of the K-1 adjacent differences
D_j = v_{j+1} - v_j of the K stencil values (v_0 is the leftmost cell,
i - K/2 + 1), so that constant data give exactly zero indicators and the
reconstruction is exactly translation-equivariant.

* candidate fluxes f_k - v_i (the candidate stencils of Table 1, Sec. 3.1),
* the smoothness measures beta_{k,r} of the candidates and beta_K of the
  full stencil (Sec. 2.2): sum_{j=1}^{r-1} int_{-1/2}^{1/2} (p^(j))^2 dxi of
  the degree r-1 polynomial whose cell averages are the stencil values,
  emitted as a positive sum of squares sum_q w_q y_q^2: six points from an
  exact LDL^T factorisation in the differences (y = L^T D); eight points
  from the exact LDL^T over the polynomial's Taylor coefficients, each row
  written in the differences with coprime integer coefficients and the
  weights times one common scale (beta_scale), so that almost every
  constant is an instruction literal (see emit),
* the optimal (maximum-order) linear weights d_k (Sec. 3.3).

Run: python gen_tables.py > teno_tables.h  (the build does this).
"""
from __future__ import annotations

import struct
import sys
from fractions import Fraction as Fr
from math import factorial, gcd

# candidate stencils S_k as offsets [lo, hi] relative to cell i (Table 1)
CANDIDATES = [(-1, 1), (0, 2), (-2, 0), (0, 3), (-3, 0), (0, 4)]


def cell_avg(l, m):
    a, b = Fr(2 * m - 1, 2), Fr(2 * m + 1, 2)
    return (b ** (l + 1) - a ** (l + 1)) / (l + 1)


def inverse(A):
    n = len(A)
    M = [list(row) + [Fr(int(i == j)) for j in range(n)] for i, row in enumerate(A)]
    for c in range(n):
        p = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[p] = M[p], M[c]
        piv = M[c][c]
        M[c] = [x / piv for x in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [x - f * y for x, y in zip(M[r], M[c])]
    return [row[n:] for row in M]


def poly_map(lo, hi):
    """Matrix P with a = P v: coefficients of the polynomial in xi = (x-x_i)/dx
    whose averages over cells lo..hi are v."""
    r = hi - lo + 1
    A = [[cell_avg(l, m) for l in range(r)] for m in range(lo, hi + 1)]
    return inverse(A)


def face_coeffs(lo, hi):
    P = poly_map(lo, hi)
    r = hi - lo + 1
    return [sum(P[l][j] * Fr(1, 2) ** l for l in range(r)) for j in range(r)]


def beta_gram(lo, hi):
    """Gram matrix G (over the r values) with beta = v^T G v."""
    P = poly_map(lo, hi)
    r = hi - lo + 1

    def mom(e):
        return Fr(0) if e % 2 else 2 * Fr(1, 2) ** (e + 1) / (e + 1)

    G = [[Fr(0)] * r for _ in range(r)]
    for j in range(1, r):
        for l1 in range(j, r):
            for l2 in range(j, r):
                c = Fr(factorial(l1), factorial(l1 - j)) * Fr(factorial(l2), factorial(l2 - j)) * mom(l1 + l2 - 2 * j)
                for a in range(r):
                    for b in range(r):
                        G[a][b] += c * P[l1][a] * P[l2][b]
    return G


def values_from_diffs(r):
    """T with v - v_0 = T D (D_j = v_{j+1} - v_j): v_m - v_0 = sum_{j<m} D_j."""
    return [[Fr(1) if j < m else Fr(0) for j in range(r - 1)] for m in range(r)]


def diff_quadratic(lo, hi):
    """Q over the r-1 differences with beta = D^T Q D (constants drop out)."""
    G = beta_gram(lo, hi)
    r = hi - lo + 1
    T = values_from_diffs(r)
    n = r - 1
    return [[sum(T[a][i] * G[a][b] * T[b][j] for a in range(r) for b in range(r)) for j in range(n)] for i in range(n)]


def ldl(Q):
    """Q = L diag(w) L^T with L unit lower triangular (exact)."""
    n = len(Q)
    L = [[Fr(int(i == j)) for j in range(n)] for i in range(n)]
    w = [Fr(0)] * n
    for j in range(n):
        w[j] = Q[j][j] - sum(L[j][k] ** 2 * w[k] for k in range(j))
        assert w[j] > 0
        for i in range(j + 1, n):
            L[i][j] = (Q[i][j] - sum(L[i][k] * L[j][k] * w[k] for k in range(j))) / w[j]
    return L, w


def optimal_weights(K):
    """d_k with sum_k d_k f_k equal to the K-point linear scheme."""
    nk = K - 2
    lo, hi = -(K // 2) + 1, K // 2
    full = face_coeffs(lo, hi)
    cols = []
    for k in range(nk):
        a, b = CANDIDATES[k]
        c = face_coeffs(a, b)
        col = [Fr(0)] * K
        for j, m in enumerate(range(a, b + 1)):
            col[m - lo] = c[j]
        cols.append(col)
    # normal equations (exact arithmetic, consistent system)
    A = [[sum(cols[i][m] * cols[j][m] for m in range(K)) for j in range(nk)] for i in range(nk)]
    b = [sum(cols[i][m] * full[m] for m in range(K)) for i in range(nk)]
    Ai = inverse(A)
    d = [sum(Ai[i][j] * b[j] for j in range(nk)) for i in range(nk)]
    for m in range(K):
        assert sum(d[k] * cols[k][m] for k in range(nk)) == full[m]
    return d


def taylor_rows(lo, hi):
    """beta on the stencil [lo, hi] as sum_q w_q (row_q . D)^2 with integer
    rows: the exact LDL^T of the measure's Gram matrix over the Taylor
    coefficients a_1 .. a_{r-1} of the polynomial about x_i (ascending),
    each row of L^T a written in the differences D and scaled to coprime
    integers (the scale moves into w_q).  Returns [(ints, w)]."""
    r = hi - lo + 1
    n = r - 1
    P = poly_map(lo, hi)
    T = values_from_diffs(r)
    # Taylor coefficients a_l (l = 1..r-1) in the differences
    M = [[sum(P[l][a] * T[a][j] for a in range(r)) for j in range(n)] for l in range(1, r)]

    def mom(e):
        return Fr(0) if e % 2 else 2 * Fr(1, 2) ** (e + 1) / (e + 1)

    H = [[Fr(0)] * n for _ in range(n)]
    for j in range(1, r):
        for k1 in range(j, r):
            for k2 in range(j, r):
                H[k1 - 1][k2 - 1] += (Fr(factorial(k1), factorial(k1 - j)) * Fr(factorial(k2), factorial(k2 - j))
                                      * mom(k1 + k2 - 2 * j))
    L, w = ldl(H)
    rows = []
    for q in range(n):
        row = [sum(L[i][q] * M[i][j] for i in range(n)) for j in range(n)]
        den = 1
        for c in row:
            den = den * c.denominator // gcd(den, c.denominator)
        ints = [c * den for c in row]
        g = 0
        for c in ints:
            g = gcd(g, abs(int(c)))
        ints = [c / g for c in ints]
        scale = Fr(den, g)
        rows.append((ints, w[q] / (scale * scale)))
    # the form is the measure: sum_q w_q (row_q . D)^2 == D^T Q D
    Q = diff_quadratic(lo, hi)
    for i in range(n):
        for j in range(n):
            assert sum(wq * ints[i] * ints[j] for ints, wq in rows) == Q[i][j]
    return rows


def literal_ok(x: Fr) -> bool:
    """True when x is a double whose low 32 bits are zero: such a constant
    is a 32-bit literal of the instruction, with no register to load."""
    if x != Fr(float(x)):
        return False
    bits = struct.unpack("<Q", struct.pack("<d", float(x)))[0]
    return (bits & 0xFFFFFFFF) == 0


def lit(x: Fr) -> str:
    """A double literal for the exact rational x: p/q evaluated at compile
    time when p and q are exact doubles (IEEE division rounds correctly),
    else the correctly rounded decimal of x."""
    if x.denominator == 1 and abs(x.numerator) < 2 ** 53:
        return f"{x.numerator}.0"
    if abs(x.numerator) < 2 ** 53 and x.denominator < 2 ** 53:
        return f"({x.numerator}.0 / {x.denominator}.0)"
    return repr(float(x))


def linear_form(coefs, names):
    """sum_j coefs[j] * names[j] as an explicit chain of fused multiply-adds
    (the library is compiled without contraction, so the rounding of every
    step is the one written here)."""
    terms = [(c, n) for c, n in zip(coefs, names) if c != 0]
    if not terms:
        return "0.0"
    c, n = terms[0]
    expr = n if c == 1 else (f"-{n}" if c == -1 else f"{lit(c)} * {n}")
    for c, n in terms[1:]:
        if c == 1:
            expr = f"{expr} + {n}"
        elif c == -1:
            expr = f"{expr} - {n}"
        else:
            expr = f"fma({lit(c)}, {n}, {expr})"
    return expr


def candidate_coeffs(K: int, k: int) -> list:
    """f_k - v_i = sum_j coefs[j] D[j] (Table 1 candidate k, differences)."""
    c0 = K // 2 - 1  # index of v_i in the K stencil values
    a, b = CANDIDATES[k]
    fc = face_coeffs(a, b)
    coefs = [Fr(0)] * (K - 1)
    for jj, m in enumerate(range(a, b + 1)):
        idx = m + c0  # stencil index of offset m
        if idx > c0:
            for j in range(c0, idx):
                coefs[j] += fc[jj]
        elif idx < c0:
            for j in range(idx, c0):
                coefs[j] -= fc[jj]
    return coefs


def emit(K: int, literal: bool) -> str:
    """Device code of one scheme.  literal: every constant that multiplies
    data is, where the exact rationals allow, a double whose low 32 bits are
    zero (an instruction literal): candidates as 1/den times an integer
    form, the indicators in integer Taylor-coefficient rows with weights
    scaled by one common factor (beta_scale, a power of two times the lcm
    of the candidate stencils' weight denominators).  Otherwise the rational
    coefficients are used directly (a triangular LDL^T in the differences)
    and beta_scale = 1."""
    nk = K - 2
    lo_full = -(K // 2) + 1
    lines = []
    w = lines.append
    w(f"// ---- K = {K}: stencil values v[0..{K - 1}] = f_(i{lo_full:+d}) .. f_(i+{K // 2}),")
    w(f"//      differences D[j] = v[j+1] - v[j], j = 0..{K - 2}")
    w(f"template <> struct TenoTables<{K}> {{")
    w(f"  static constexpr int NK = {nk};")
    d = optimal_weights(K)
    w("  // optimal linear weights d_k (maximum order)")
    w("  static __device__ __forceinline__ constexpr double d(int k) {")
    expr = lit(d[nk - 1])
    for k in range(nk - 2, -1, -1):
        expr = f"k == {k} ? {lit(d[k])} : {expr}"
    w(f"    return {expr};")
    w("  }")
    names = [f"D[{j}]" for j in range(K - 1)]
    cand = [candidate_coeffs(K, k) for k in range(nk)]
    stencils = [(k, CANDIDATES[k]) for k in range(nk)] + [("K", (lo_full, K // 2))]
    scale = Fr(1)
    if literal:
        trows = {tag: taylor_rows(a, b) for tag, (a, b) in stencils}
        den = 1
        for tag, _ in stencils:
            if tag == "K":
                continue
            for _, wq in trows[tag]:
                den = den * wq.denominator // gcd(den, wq.denominator)
        scale = Fr(den)
        while scale > 2:
            scale /= 2
        for tag, _ in stencils:
            if tag != "K":
                assert all(literal_ok(wq * scale) for _, wq in trows[tag]), tag
    w("  // every beta below is beta_scale times the measure of Eq. measureTENO;")
    w("  // the cutoff scales eps by the same factor")
    w(f"  static constexpr double beta_scale = {lit(scale)};")
    # candidates relative to v_i
    w("  // candidate fluxes minus v_i, from the candidate stencils of Table 1")
    w("  static __device__ __forceinline__ void candidates(const double* D, double* c) {")
    cand_den = []
    for k in range(nk):
        if literal:
            den = 1
            for c in cand[k]:
                den = den * c.denominator // gcd(den, c.denominator)
            ints = [c * den for c in cand[k]]
            cand_den.append(den)
            w(f"    c[{k}] = {lit(Fr(1, den))} * ({linear_form(ints, names)});")
        else:
            w(f"    c[{k}] = {linear_form(cand[k], names)};")
    w("  }")
    # transpose of the candidate map, for the adjoint: Dbar += C^T cbar
    w("  // adjoint of candidates: Dbar[j] += sum_k (d c_k / d D_j) cbar[k]")
    w("  static __device__ __forceinline__ void candidates_vjp(const double* cbar, double* Dbar) {")
    if literal:
        for k in range(nk):
            w(f"    const double s{k} = {lit(Fr(1, cand_den[k]))} * cbar[{k}];")
        src = [f"s{k}" for k in range(nk)]
        mats = [[c * cand_den[k] for c in cand[k]] for k in range(nk)]
    else:
        src = [f"cbar[{k}]" for k in range(nk)]
        mats = cand
    for j in range(K - 1):
        col = [mats[k][j] for k in range(nk)]
        if any(c != 0 for c in col):
            w(f"    Dbar[{j}] = {linear_form(col + [Fr(1)], src + [f'Dbar[{j}]'])};")
    w("  }")
    # betas
    w("  // smoothness measures beta_k (candidates) and beta_K (full stencil)")
    w("  static __device__ __forceinline__ void betas(const double* D, double* beta, double& betaK) {")
    for tag, (a, b) in stencils:
        first = a + K // 2 - 1  # index of the first difference of this stencil
        n = b - a
        dn = [f"D[{first + j}]" for j in range(n)]
        if literal:
            rows = [(ints, wq * scale) for ints, wq in trows[tag]]
            ys = [linear_form(ints, dn) for ints, _ in rows]
            wts = [wq for _, wq in rows]
        else:
            Q = diff_quadratic(a, b)
            L, wts = ldl(Q)
            ys = [linear_form([L[j][q] if j >= q else Fr(0) for j in range(n)], dn) for q in range(n)]
        w("    {")
        for q in range(n):
            w(f"      const double y{q} = {ys[q]};")
        expr = f"{lit(wts[0])} * (y0 * y0)"
        for q in range(1, n):
            expr = f"fma({lit(wts[q])} * y{q}, y{q}, {expr})"
        target = "betaK" if tag == "K" else f"beta[{tag}]"
        w(f"      {target} = {expr};")
        w("    }")
    w("  }")
    w("};")
    return "\n".join(lines)


def main(out=sys.stdout):
    out.write("// Generated by gen_tables.py: exact-rational constants of the TENO-M\n")
    out.write("// reconstruction in difference form.  Do not edit.\n")
    out.write("#pragma once\n\n")
    out.write("template <int K> struct TenoTables;\n\n")
    # six points: the exact rationals as they come (the six-point kernels
    # run at three or more wavefronts per SIMD, which hide the scalar moves
    # of non-literal constants); eight points: literal-friendly forms (their
    # kernels run at one wavefront per SIMD, where every constant moved into
    # a scalar register costs an issue slot)
    out.write(emit(6, literal=False) + "\n\n")
    out.write(emit(8, literal=True) + "\n")


if __name__ == "__main__":
    main()
