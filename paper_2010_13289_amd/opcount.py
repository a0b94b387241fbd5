"""Algorithmic FP64 operation counts of the TENO-M path, item by item.

These are the counts the roofline fractions of the benchmark divide by: the
operations the method as formulated computes per unit of work, not what any
kernel happens to execute.  Counting rules: add, subtract, multiply,
divide, square root, abs, min, max and compare count 1; a fused
multiply-add counts 2; selects, loads and stores count 0.  The limiter acts
only on nonsmooth candidates (Eq. mp_flux), so its work depends on the
data: with rough = nonsmooth = None every candidate is counted (the bound
on the method's work); given the measured share of the data, its bounds
(or TVD flux) are counted once per reconstruction with a nonsmooth
candidate (a fraction `rough` of the reconstructions) and the clamp once
per nonsmooth candidate (`nonsmooth` per reconstruction on average).  The
roofline fractions use the measured counts.

Every item is a formula in the structure of the scheme (number of points K,
candidate stencil widths, fields, dimensions), written next to the step it
counts.  tests/test_opcount.py pins the structural inputs (stencil widths
from Table 1, the rank and density of the smoothness-indicator quadratic
forms) and the totals.
"""
from __future__ import annotations

from fractions import Fraction

# points r_k of the candidate stencils S_0 .. S_{K-3} (Table 1)
STENCIL_POINTS = {6: (3, 3, 3, 4), 8: (3, 3, 3, 4, 4, 5)}

# limiter IDs of the C ABI
LIM_TENO, LIM_MP, LIM_TVD_MINMOD, LIM_TVD5, LIM_VA = 0, 1, 2, 3, 4
LIM_MP_M4_B2, LIM_MP_MM_B4, LIM_MP_MM_B2, LIM_MP_MM_B1 = 5, 6, 7, 8
MP_M4 = (LIM_MP, LIM_MP_M4_B2)
MP_MM = (LIM_MP_MM_B4, LIM_MP_MM_B2, LIM_MP_MM_B1)


def linear_form_ops(terms: int) -> int:
    """sum of `terms` coefficient * value products: one multiply, then one
    fused multiply-add per further term."""
    return 0 if terms <= 0 else 1 + 2 * (terms - 1)


def beta_ops(points: int) -> int:
    """Eq. measureTENO's beta on an r-point stencil: a positive definite
    quadratic form in the r - 1 adjacent differences, evaluated as a
    weighted sum of squares (LDL^T): y_l = x_l + sum_{m>l} L_ml x_m costs
    n - 1 - l fused multiply-adds, and each of the n squares one multiply
    for the square, one for its weight and, after the first, the addition
    fused: n^2 + 2n - 1 with n = r - 1."""
    n = points - 1
    return n * n + 2 * n - 1


def mp_bounds_ops(limiter: int) -> int:
    """Eqs. curvature .. value_min_max relative to f_i: three curvatures
    (differences of differences); the interface curvatures (d^M4: two
    minmods of four arguments, two of them formed by a multiply-add each;
    d^MM: two minmods of two); UL, MD, LC; the min/max bounds."""
    curv = 3
    if limiter in MP_M4:
        measures = 4 * 2 + 2 * 9   # 4 arguments 4 d - d; minmod4 = 3 min, 3 max, clamp, clamp, add
    else:
        measures = 2 * 5           # minmod2 = min, max, clamp, clamp, add
    ul = 1                         # 1.25 (f_i - f_{i-1})
    md = 3                         # (f_{i+1} - f_i)/2 - d/2: multiply + fused multiply-add
    lc = 3                         # (f_i - f_{i-1})/2 + beta/3 d: multiply + fused multiply-add
    bounds = 2 * 5                 # max(min(min(.,.),.), min(min(.,.),.)) and its mirror
    return curv + measures + ul + md + lc + bounds


def adaptive_cutoff_ops() -> int:
    """Sec. 2.4: the Ren-type indicator at four points (|2ab| + eps over
    a^2 + b^2 + eps: 2 multiplies, abs, add, 2 fused multiply-adds, divide),
    their minimum, m, g(m) = (1-m)^4 (1+4m), beta, the floor and the three
    comparisons that pick C_T."""
    eta = 4 * (2 + 1 + 1 + 4 + 1) + 3
    m = 3            # eta / C_r, min(1, .), 1 - .
    g = 6            # 1 - m, square, square, 1 + 4m (fused), product
    beta = 3         # 1 - g, fused multiply-add
    return eta + m + g + beta + 1 + 3


def reconstruction_items(K: int, limiter: int, adaptive: bool = False, rough: float | None = None,
                         nonsmooth: float | None = None) -> dict:
    """Operations of one scalar TENO-M reconstruction (one side, one field);
    with rough and nonsmooth the limiter's share as measured (module
    docstring), else every candidate limited."""
    pts = STENCIL_POINTS[K]
    nk = len(pts)
    if (rough is None) != (nonsmooth is None):
        raise ValueError("give both rough and nonsmooth, or neither")
    if rough is None:
        rough, nonsmooth = 1, nk
    elif not (0 <= rough <= 1 and 0 <= nonsmooth <= nk * rough):
        raise ValueError(f"shares out of range: rough {rough}, nonsmooth {nonsmooth}")
    it = {
        "differences": K - 1,                                   # D_j = v_{j+1} - v_j
        "candidates": sum(linear_form_ops(r - 1) for r in pts),  # Table 1 in differences
        "betas": sum(beta_ops(r) for r in pts) + beta_ops(K),   # beta_k and beta_K
        "tau": 6,                                               # |beta_K - (beta_1 + beta_2 + 4 beta_0)/6|
        "gamma": 6 * nk,                                        # beta+eps, divide, 1+, ^2, ^4, ^6
        "cutoff": (nk - 1) + 1 + nk,                            # sum, C_T * sum, compares
    }
    if adaptive:
        it["adaptive_cutoff"] = adaptive_cutoff_ops()
    if limiter in MP_M4 or limiter in MP_MM:
        it["mp_bounds"] = rough * mp_bounds_ops(limiter)
        it["medians"] = 2 * nonsmooth                           # clamp of each nonsmooth candidate
    elif limiter == LIM_TVD_MINMOD:
        it["tvd_flux"] = rough * (5 + 1)                        # minmod2, halving
    elif limiter == LIM_TVD5:
        it["tvd_flux"] = rough * (8 + 2 + 3 + 3 + 2 + 1)        # B, 2d-, 2d+, two clamps, sign tests, halving
    elif limiter == LIM_VA:
        it["tvd_flux"] = rough * (3 + 1 + 1 + 3 + 1 + 7)        # d+^2 + d-^2, floor, divide, 2 d+ d- phi, phi/3, flux
    elif limiter != LIM_TENO:
        raise ValueError(f"unknown limiter {limiter}")
    if limiter == LIM_TENO:
        it["assembly"] = 2 * nk + nk + 1 + 1                    # sum d_k f_k, sum d_k, divide, + f_i
    else:
        it["assembly"] = 2 * nk                                 # sum d_k f^M_k (mul, fmas), + f_i
    return it


def reconstruction_ops(K: int, limiter: int, adaptive: bool = False, rough=None, nonsmooth=None) -> float:
    return sum(reconstruction_items(K, limiter, adaptive, rough, nonsmooth).values())


# --- per face vector ------------------------------------------------------

def cell_ops(ndim: int) -> dict:
    """Per-cell Euler physics, once per cell: primitives and normal flux,
    signal speed, and the Roe-average inputs (sqrt rho, velocity, H)."""
    nd = ndim
    prim = 1 + 1 + linear_form_ops(nd) + 3 + 1        # 1/rho, u_n, |m|^2, e, p
    flux = 2 + (nd - 1) + 3                           # F_m_n, transverse momenta, energy flux
    speed = 5                                         # |u_n| + sqrt(gamma p / rho)
    roe_in = 1 + nd + linear_form_ops(nd) + 3 + 3 + 1  # 1/rho, u, |u|^2, e, H, sqrt(rho)
    return {"cell_primitives_flux": prim + flux, "cell_speed": speed, "cell_roe_input": roe_in}


def projection_ops(ndim: int) -> int:
    """Left eigenvectors at the Roe state applied to one conservative vector
    (closed form): u~.m, A, B, the acoustic pair, entropy, shear waves."""
    nd = ndim
    return linear_form_ops(nd) + 4 + 2 + 3 + 1 + 2 * (nd - 1) + 3


def roe_ops(ndim: int) -> int:
    """Roe average of cells i, i+1 (weights, velocity, enthalpy, sound
    speed) and the eigenvector constants 1/c, b1, b2."""
    nd = ndim
    return 2 + 4 * nd + 4 + linear_form_ops(nd) + 4 + 5


def back_projection_ops(ndim: int) -> int:
    nd = ndim
    return 2 + 1 + 3 + 5 + 3 + 4 * (nd - 1)


def update_ops(nf: int, ndim: int) -> Fraction:
    """Per face vector: the divergence of one face pair (2 per field) plus
    this axis' share of the per-cell work of a stage: accumulating the axes
    (ndim - 1 adds per field) and the SSP-RK3 update U_s + dt R (fused) and
    a U^n + b (.) (1 in stage 1, 3 in stages 2 and 3), averaged over the
    three stages."""
    per_cell = nf * (Fraction(ndim - 1) + 2 + Fraction(1 + 3 + 3, 3))
    return 2 * nf + per_cell / ndim


def face_vector_items(system: str, ndim: int, K: int, limiter: int, adaptive: bool = False, rough=None,
                      nonsmooth=None) -> dict:
    """Operations per face vector (all fields, both split sides) of one
    SSP-RK3 stage sweep: system "euler" or "scalar"; rough and nonsmooth
    as for reconstruction_items."""
    rec = reconstruction_ops(K, limiter, adaptive, rough, nonsmooth)
    if system == "scalar":
        nf = 1
        it = {"flux_and_split": K * (1 + 3) / K,   # f = a u and the split, once per cell
              "reconstructions": 2 * rec, "combine": 2}
    elif system == "euler":
        nf = ndim + 2
        it = dict(cell_ops(ndim))
        it.update({
            "rusanov_alpha": K - 1,                  # max of |u_n| + c over the K cells
            "roe_average": roe_ops(ndim),
            "projections": 2 * K * projection_ops(ndim),  # U and F of the K cells
            "splits": 3 * nf * K,                    # alpha W, G + alpha W, G - alpha W
            "reconstructions": 2 * nf * rec,
            "combine": 2 * nf,                       # (f+ + f-) / 2
            "back_projection": back_projection_ops(ndim),
        })
    else:
        raise ValueError(system)
    it["divergence_and_update"] = update_ops(nf, ndim)
    return it


def face_vector_ops(system: str, ndim: int, K: int, limiter: int, adaptive: bool = False, rough=None,
                    nonsmooth=None) -> float:
    return float(sum(face_vector_items(system, ndim, K, limiter, adaptive, rough, nonsmooth).values()))


# --- adjoint (frozen decisions) --------------------------------------------

def adjoint_face_vector_items(ndim: int, K: int, limiter: int, adaptive: bool = False, rough=None,
                              nonsmooth=None) -> dict:
    """Operations per Euler face vector of the frozen-branch vector-Jacobian
    product: the forward face evaluated again (its decisions and
    intermediates are needed), then the reverse.  The reverse of a step
    linear in its inputs costs its forward count (a transpose); of a
    bilinear step (projection and back-projection with state-dependent
    eigenvectors, the Rusanov split) twice its forward count; of the
    nonlinear per-cell physics and Roe average three times.  Decisions
    (indicators, cutoff, limiter choices) have no reverse: with them frozen
    the reconstruction is linear in the split values, and its reverse is
    the transpose of the selected coefficients (differences, candidates,
    bounds' curvature terms and assembly); with measured shares the bounds'
    reverse is counted where the forward's are."""
    fwd = face_vector_items("euler", ndim, K, limiter, adaptive, rough, nonsmooth)
    rec = reconstruction_items(K, limiter, adaptive, rough, nonsmooth)
    nf = ndim + 2
    linear_rec = rec["differences"] + rec["candidates"] + rec["assembly"] + rec.get("mp_bounds", 0)
    it = {"forward_" + k: v for k, v in fwd.items()}
    it.update({
        "rev_divergence_and_update": fwd["divergence_and_update"],
        "rev_back_projection": 2 * fwd["back_projection"],
        "rev_combine": fwd["combine"],
        "rev_reconstructions": 2 * nf * linear_rec,
        "rev_splits": 2 * fwd["splits"],
        "rev_projections": 2 * fwd["projections"],
        "rev_roe_average": 3 * fwd["roe_average"],
        "rev_rusanov_alpha": fwd["rusanov_alpha"],
        "rev_cell": 3 * (fwd["cell_primitives_flux"] + fwd["cell_speed"] + fwd["cell_roe_input"]),
    })
    return it


def adjoint_face_vector_ops(ndim: int, K: int, limiter: int, adaptive: bool = False, rough=None,
                            nonsmooth=None) -> float:
    return float(sum(adjoint_face_vector_items(ndim, K, limiter, adaptive, rough, nonsmooth).values()))


def limiter_share(flags, nk: int) -> tuple[float, float]:
    """(rough, nonsmooth) of a set of reconstructions from their smoothness
    flags (bit k set = candidate k smooth, as the library's
    reconstruct_faces returns them): the fraction with a nonsmooth
    candidate and the mean number of nonsmooth candidates.  `flags` is a
    numpy or torch integer array; every element is one reconstruction."""
    full = (1 << nk) - 1
    rough = nonsmooth = 0
    total = 0
    for k in range(nk):
        bad = ((flags >> k) & 1) == 0
        nonsmooth += int(bad.sum())
    rough = int(((flags & full) != full).sum())
    total = int(flags.numel() if hasattr(flags, "numel") else flags.size)
    return rough / total, nonsmooth / total


# --- bytes ---------------------------------------------------------------

def rk3_bytes_per_cell(nf: int) -> int:
    """HBM bytes of one SSP-RK3 step per cell that the method must move:
    every stage reads its stage state and writes the next one, and stages 2
    and 3 also read U^n (8 bytes per value)."""
    return 8 * nf * (2 + 3 + 3)


if __name__ == "__main__":
    import json
    for name, args in {"euler3d_K6_MP": ("euler", 3, 6, LIM_MP), "euler1d_K8_MP": ("euler", 1, 8, LIM_MP),
                       "euler2d_K6_MP": ("euler", 2, 6, LIM_MP)}.items():
        items = {k: float(v) for k, v in face_vector_items(*args).items()}
        print(name, json.dumps(items), "total", face_vector_ops(*args))
    print("adjoint euler2d_K6_MP", adjoint_face_vector_ops(2, 6, LIM_MP))
