"""Reference adjoint of the TENO-M flux divergence and of one SSP-RK3 step.

Test infrastructure only: the test suite, the smoke check and the CPU leg
of the benchmark may use it; the library never does.  It shares no code
with the HIP library.

The forward method is written again in plain PyTorch CPU float64
operations, in the value form of ``tenom_oracle.c``:
  - Table 1 candidate fluxes (Sec. 3.1);
  - indicators beta_k, beta_K as quadratic forms of the stencil values,
    tau_K and gamma_k, and the cutoff (Eqs. measureTENO, taukTENO,
    normalize, cut-off; Sec. 2.4 for TENO8A);
  - the limiters of Sec. 3.2 and assembly with the optimal weights
    (Eq. reconstuction), or classic TENO's renormalisation
    (Eq. weight_renormalize);
  - Rusanov splitting and the characteristic projection on the Roe
    eigenvectors of Sec. 4 (L = R^-1 by a numeric inverse, as in the
    oracle), the divergence, and the SSP-RK3 stages.
The constants (Table 1 rows, the optimal weights, the indicator quadratic
forms) come from the C oracle.

Every piecewise choice is a comparison evaluated on the values
(``torch.where``), so ``torch.autograd`` returns the derivative of the
forward map with all of them frozen at the evaluation point:
  - the smoothness decisions;
  - the limiter branches, with min/max passing the derivative to the
    first argument on ties and a minmod passing it to its
    smallest-magnitude argument only when all its arguments share a
    strict sign;
  - the Rusanov alpha, at its first maximising cell, with |u_n| passing
    sgn(u_n) (0 at u_n = 0, torch.abs's convention).
That is the derivative the GPU adjoint computes.  The time step is a
parameter.  Pinned in ``tests/test_oracle_adjoint.py`` against the C oracle's
values and against central differences of the C oracle.
"""
from __future__ import annotations

import functools

import numpy as np
import torch

from . import LIM_MP, LIM_MP_M4_B2, LIM_MP_MM_B1, LIM_MP_MM_B2, LIM_MP_MM_B4, LIM_TENO, LIM_TVD5, LIM_TVD_MINMOD
from . import LIM_VA, SCHEME_ADAPTIVE, beta, poly_face, weights

DT = torch.float64
EPS = 1e-40          # Eq. measureTENO
Q = 6                # Eq. measureTENO
MP_ALPHA = 1.25      # Eq. upper_limiter
VA_KAPPA = 1.0 / 3.0  # Eq. vAflux
REN_XI, REN_CR = 1e-3, 0.23       # Eq. shock_indicator
ADAPT_A1, ADAPT_A2 = 10.5, 3.5    # Eq. cut-off_adjust
# candidate stencils S_k as offsets from i (Table 1)
CAND = [(-1, 1), (0, 2), (-2, 0), (0, 3), (-3, 0), (0, 4)]


@functools.lru_cache(maxsize=None)
def _quadratic_form(lo: int, hi: int) -> np.ndarray:
    """beta = D^T Q D in the differences D_j = v_{j+1} - v_j of the stencil
    [lo, hi] (beta is a quadratic form of the values that vanishes on
    constants), Q by polarisation of the oracle's beta on stencils whose
    differences are unit vectors.  A constant stencil gets beta = 0 exactly."""
    r = hi - lo
    steps = [np.concatenate([np.zeros(j + 1), np.ones(r - j)]) for j in range(r)]
    Qm = np.zeros((r, r))
    b = [beta(lo, hi, steps[i]) for i in range(r)]
    for i in range(r):
        Qm[i, i] = b[i]
        for j in range(i + 1, r):
            Qm[i, j] = Qm[j, i] = 0.5 * (beta(lo, hi, steps[i] + steps[j]) - b[i] - b[j])
    return Qm


@functools.lru_cache(maxsize=None)
def _scheme(K: int):
    nk = K - 2
    cands = [np.asarray(poly_face(*CAND[k])) for k in range(nk)]
    d = np.asarray(weights(K))
    full = (-(K // 2) + 1, K // 2)
    return cands, d, [_quadratic_form(*CAND[k]) for k in range(nk)], _quadratic_form(*full)


# ---------------------------------------------------------------------------
# piecewise choices (the derivative goes to the chosen argument)
# ---------------------------------------------------------------------------

def fmin(a, b):
    return torch.where(a <= b, a, b)


def fmax(a, b):
    return torch.where(a >= b, a, b)


def minmod(*args):
    """Eqs. minmod222 / minmod444: the smallest-magnitude argument when all
    share a strict sign, else 0."""
    if len(args) == 2:
        lo, hi = fmin(args[0], args[1]), fmax(args[0], args[1])
    else:
        lo = fmin(fmin(args[0], args[1]), fmin(args[2], args[3]))
        hi = fmax(fmax(args[0], args[1]), fmax(args[2], args[3]))
    zero = torch.zeros_like(lo)
    return torch.where(lo > 0, lo, torch.where(hi < 0, hi, zero))


# ---------------------------------------------------------------------------
# one TENO-M reconstruction on the last axis (K values each)
# ---------------------------------------------------------------------------

def _adaptive_ct(vd: torch.Tensor, K: int) -> torch.Tensor:
    """Eqs. shock_indicator and cut-off_adjust on detached values."""
    c0 = K // 2 - 1
    eps = 0.9 * REN_CR / (1.0 - 0.9 * REN_CR) * REN_XI * REN_XI
    eta = None
    for j in range(-1, 3):
        dp = vd[..., c0 + j + 1] - vd[..., c0 + j]
        dm = vd[..., c0 + j] - vd[..., c0 + j - 1]
        e = (torch.abs(2.0 * dp * dm) + eps) / (dp * dp + dm * dm + eps)
        eta = e if eta is None else torch.minimum(eta, e)
    m = 1.0 - torch.clamp(eta / REN_CR, max=1.0)
    g = (1.0 - m) ** 4 * (1.0 + 4.0 * m)
    b = ADAPT_A1 - ADAPT_A2 * (1.0 - g)
    return torch.pow(10.0, -torch.floor(b))


def teno_m(v: torch.Tensor, scheme: int, lim: int, C_T: float):
    """Reconstruction at x_{i+1/2} from v[..., 0..K-1] = f_{i-K/2+1..i+K/2}.
    Returns (value, delta[..., K-2])."""
    K = scheme & 0xFF
    nk, c0 = K - 2, K // 2 - 1
    cands, d, Qk, QK = _scheme(K)
    cand = torch.stack([sum(float(cf[j]) * v[..., c0 + CAND[k][0] + j] for j in range(len(cf)))
                        for k, cf in enumerate(cands)], dim=-1)
    vd = v.detach()
    dd = vd[..., 1:] - vd[..., :-1]
    bk = []
    for k in range(nk):
        lo, hi = CAND[k]
        s = dd[..., c0 + lo:c0 + hi]
        bk.append(torch.einsum("...i,ij,...j->...", s, torch.as_tensor(Qk[k]), s))
    bK = torch.einsum("...i,ij,...j->...", dd, torch.as_tensor(QK), dd)
    tau = torch.abs(bK - (bk[1] + bk[2] + 4.0 * bk[0]) / 6.0)
    gam = torch.stack([(1.0 + tau / (b + EPS)) ** Q for b in bk], dim=-1)
    chi = gam / gam.sum(dim=-1, keepdim=True)
    ct = _adaptive_ct(vd, K)[..., None] if scheme & SCHEME_ADAPTIVE else C_T
    delta = ~(chi < ct)
    dk = torch.as_tensor(d)
    if lim == LIM_TENO:
        w = torch.where(delta, dk, torch.zeros_like(chi))
        return (w * cand).sum(-1) / w.sum(-1), delta
    fm2, fm1, f0, fp1, fp2 = (v[..., c0 + o] for o in (-2, -1, 0, 1, 2))
    if lim in (LIM_MP, LIM_MP_M4_B2, LIM_MP_MM_B4, LIM_MP_MM_B2, LIM_MP_MM_B1):
        bet = {LIM_MP: 4.0, LIM_MP_M4_B2: 2.0, LIM_MP_MM_B4: 4.0, LIM_MP_MM_B2: 2.0, LIM_MP_MM_B1: 1.0}[lim]
        d_im1, d_i, d_ip1 = f0 - 2.0 * fm1 + fm2, fp1 - 2.0 * f0 + fm1, fp2 - 2.0 * fp1 + f0
        if lim in (LIM_MP, LIM_MP_M4_B2):
            dR = minmod(4.0 * d_i - d_ip1, 4.0 * d_ip1 - d_i, d_i, d_ip1)
            dL = minmod(4.0 * d_im1 - d_i, 4.0 * d_i - d_im1, d_im1, d_i)
        else:
            dR, dL = minmod(d_i, d_ip1), minmod(d_im1, d_i)
        f_ul = f0 + MP_ALPHA * (f0 - fm1)
        f_md = 0.5 * (f0 + fp1) - 0.5 * dR
        f_lc = f0 + 0.5 * (f0 - fm1) + (bet / 3.0) * dL
        f_lo = fmax(fmin(fmin(f0, fp1), f_md), fmin(fmin(f0, f_ul), f_lc))
        f_hi = fmin(fmax(fmax(f0, fp1), f_md), fmax(fmax(f0, f_ul), f_lc))
        # median(f_k, f_min, f_max) with f_min <= f_i <= f_max is the clamp
        flim = fmin(fmax(cand, f_lo[..., None]), f_hi[..., None])
    else:
        dm, dp = f0 - fm1, fp1 - f0
        if lim == LIM_TVD_MINMOD:
            ftvd = f0 + 0.5 * minmod(dm, dp)
        elif lim == LIM_TVD5:
            # phi(r) delta^- of Eqs. high order TVD, TVDhighorder2, TVDbeta
            B = (-2.0 * (fm1 - fm2) + 11.0 * dm + 24.0 * dp - 3.0 * (fp2 - fp1)) / 30.0
            zero = torch.zeros_like(dm)
            up = fmax(zero, fmin(fmin(2.0 * dm, 2.0 * dp), B))
            dn = fmin(zero, fmax(fmax(2.0 * dm, 2.0 * dp), B))
            ftvd = f0 + 0.5 * torch.where(dm > 0, up, torch.where(dm < 0, dn, zero))
        elif lim == LIM_VA:
            # phi = 2 r / (r^2 + 1), r = dp / dm (Eqs. slop_ratio, van_Albada_limiter)
            den = dp * dp + dm * dm
            safe = torch.where(den > 0, den, torch.ones_like(den))
            phi = torch.where(den > 0, 2.0 * dp * dm / safe, torch.zeros_like(den))
            ftvd = f0 + 0.25 * phi * ((1.0 - VA_KAPPA * phi) * dm + (1.0 + VA_KAPPA * phi) * dp)
        else:
            raise ValueError(f"limiter {lim}")
        flim = ftvd[..., None].expand_as(cand)
    fM = torch.where(delta, cand, flim)
    return (dk * fM).sum(-1), delta


# ---------------------------------------------------------------------------
# Euler and scalar face fluxes along one axis
# ---------------------------------------------------------------------------

def _euler_flux(U: torch.Tensor, gamma: float, ax: int):
    """U[nf, ...] -> (F[nf, ...] along axis ax, |u_n| + c)."""
    nd = U.shape[0] - 2
    rho, E = U[0], U[nd + 1]
    vel = [U[1 + d] / rho for d in range(nd)]
    q2 = sum(v * v for v in vel)
    p = (gamma - 1.0) * (E - 0.5 * rho * q2)
    un = vel[ax]
    F = [rho * un] + [rho * vel[d] * un + (p if d == ax else 0.0) for d in range(nd)] + [(E + p) * un]
    return torch.stack(F), torch.abs(un) + torch.sqrt(gamma * p / rho)


def _roe_right(UL: torch.Tensor, UR: torch.Tensor, gamma: float, ax: int) -> torch.Tensor:
    """Right eigenvectors at the Roe average, [..., nf, nf] (columns u_n - c,
    entropy, shear waves in increasing axis order, u_n + c)."""
    nf = UL.shape[0]
    nd = nf - 2

    def prim(S):
        rho = S[0]
        vel = [S[1 + d] / rho for d in range(nd)]
        q2 = sum(v * v for v in vel)
        p = (gamma - 1.0) * (S[nf - 1] - 0.5 * rho * q2)
        return rho, vel, (S[nf - 1] + p) / rho

    rl, vl, Hl = prim(UL)
    rr, vr, Hr = prim(UR)
    sl, sr = torch.sqrt(rl), torch.sqrt(rr)
    u = [(sl * vl[d] + sr * vr[d]) / (sl + sr) for d in range(nd)]
    q2 = sum(x * x for x in u)
    H = (sl * Hl + sr * Hr) / (sl + sr)
    c = torch.sqrt((gamma - 1.0) * (H - 0.5 * q2))
    un = u[ax]
    one, zero = torch.ones_like(c), torch.zeros_like(c)
    cols = [[one] + [u[d] - (c if d == ax else 0.0) for d in range(nd)] + [H - un * c],
            [one] + [u[d] for d in range(nd)] + [0.5 * q2]]
    for t in range(nd):
        if t != ax:
            cols.append([zero] + [one if d == t else zero for d in range(nd)] + [u[t]])
    cols.append([one] + [u[d] + (c if d == ax else 0.0) for d in range(nd)] + [H + un * c])
    return torch.stack([torch.stack(col, dim=-1) for col in cols], dim=-1)  # [..., row, col]


def face_fluxes(S: torch.Tensor, gamma: float, ax: int, system: int, adv: float, scheme: int, lim: int,
                C_T: float):
    """S[nf, ..., K]: the K stencil states of each face.  Returns (Fhat[nf, ...],
    delta[2, nf, ..., K-2])."""
    K = scheme & 0xFF
    h = K // 2
    if system == 0:
        a = adv
        gp = 0.5 * (a * S + abs(a) * S)
        gm = 0.5 * (a * S - abs(a) * S)
        fp, dp_ = teno_m(gp[0], scheme, lim, C_T)
        fm, dm_ = teno_m(torch.flip(gm[0], dims=(-1,)), scheme, lim, C_T)
        return (fp + fm)[None], torch.stack([dp_[None], dm_[None]])
    nf = S.shape[0]
    Fc, lam = _euler_flux(S, gamma, ax)
    alpha = torch.zeros_like(lam[..., 0])
    for m in range(K):                              # the first maximum
        alpha = torch.where(lam[..., m] > alpha, lam[..., m], alpha)
    R = _roe_right(S[..., h - 1], S[..., h], gamma, ax)
    L = torch.linalg.inv(R)
    W = torch.einsum("...cr,r...k->c...k", L, S)
    G = torch.einsum("...cr,r...k->c...k", L, Fc)
    gp = 0.5 * (G + alpha[..., None] * W)
    gm = 0.5 * (G - alpha[..., None] * W)
    fc, dl = [], []
    for c in range(nf):
        fp, dp_ = teno_m(gp[c], scheme, lim, C_T)
        fm, dm_ = teno_m(torch.flip(gm[c], dims=(-1,)), scheme, lim, C_T)
        fc.append(fp + fm)
        dl.append((dp_, dm_))
    fcs = torch.stack(fc, dim=-1)
    Fh = torch.einsum("...rc,...c->r...", R, fcs)
    delta = torch.stack([torch.stack([d[0] for d in dl]), torch.stack([d[1] for d in dl])])
    return Fh, delta


def _stencil_index(n: int, K: int, bc: int, periodic_faces: bool) -> torch.Tensor:
    """[faces, K] cell indices of the stencils of faces 0..n (face j between
    cells j-1 and j)."""
    nfa = n if periodic_faces else n + 1
    j = torch.arange(nfa)[:, None] + torch.arange(K)[None, :] - K // 2
    return torch.remainder(j, n) if bc == 0 else torch.clamp(j, 0, n - 1)


def flux_divergence(U: torch.Tensor, grid: dict, scheme: int, lim: int, C_T: float, gamma: float,
                    return_flags: bool = False):
    """dU/dt = -sum_axis (F_{i+1/2} - F_{i-1/2}) / dx (Eq. approximateEq)."""
    nd = int(grid["ndim"])
    K = scheme & 0xFF
    out = torch.zeros_like(U)
    flags = []
    for ax in range(nd):
        n = int(grid["n"][ax])
        bc = int(grid["bc"][ax])
        dim = U.dim() - 1 - ax        # numpy axis of grid axis ax
        Um = U.movedim(dim, -1)       # [nf, ..., n]
        idx = _stencil_index(n, K, bc, periodic_faces=False)
        S = Um[..., idx]              # [nf, ..., n+1, K]
        adv = float(grid.get("adv", [0.0] * 3)[ax]) if int(grid.get("system", 1)) == 0 else 0.0
        Fh, delta = face_fluxes(S, gamma, ax, int(grid.get("system", 1)), adv, scheme, lim, C_T)
        div = -(Fh[..., 1:] - Fh[..., :-1]) / float(grid["dx"][ax])
        out = out + div.movedim(-1, dim)
        flags.append(delta)
    return (out, flags) if return_flags else out


def rk3_step(U: torch.Tensor, grid: dict, scheme: int, lim: int, C_T: float, gamma: float, dt: float):
    """One SSP-RK3 step (Sec. 4)."""
    L = lambda V: flux_divergence(V, grid, scheme, lim, C_T, gamma)  # noqa: E731
    U1 = U + dt * L(U)
    U2 = 0.75 * U + 0.25 * (U1 + dt * L(U1))
    return U / 3.0 + 2.0 / 3.0 * (U2 + dt * L(U2))


# ---------------------------------------------------------------------------
# numpy entry points
# ---------------------------------------------------------------------------

def _t(a) -> torch.Tensor:
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64))


def flux_divergence_np(U, grid, scheme, lim, C_T, gamma) -> np.ndarray:
    with torch.no_grad():
        return flux_divergence(_t(U), grid, scheme, lim, C_T, gamma).numpy()


def flux_divergence_vjp(U, Lbar, grid, scheme, lim, C_T, gamma) -> np.ndarray:
    """(dL/dU)^T Lbar with every piecewise choice frozen."""
    Ut = _t(U).requires_grad_(True)
    L = flux_divergence(Ut, grid, scheme, lim, C_T, gamma)
    (g,) = torch.autograd.grad(L, Ut, _t(Lbar))
    return g.numpy()


def rk3_step_vjp(U, Ubar, grid, scheme, lim, C_T, gamma, dt) -> np.ndarray:
    """(d step(U)/dU)^T Ubar with every piecewise choice frozen."""
    Ut = _t(U).requires_grad_(True)
    out = rk3_step(Ut, grid, scheme, lim, C_T, gamma, dt)
    (g,) = torch.autograd.grad(out, Ut, _t(Ubar))
    return g.numpy()
