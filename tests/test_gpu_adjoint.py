"""GPU parity of the adjoint (tenom_flux_divergence_vjp, tenom_rk3_step_vjp)
against the reference adjoint, element by element, and of the
checkpointed rollout gradient against the same computation without
checkpoints and against central differences of the GPU forward map."""
import numpy as np
import pytest

import workloads as W
from oracle import reference_adjoint as RA
from parity import assert_close_fields, band_faces, faces_to_cells, require_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu

GAMMA = 1.4

# name, shape (z, y, x), grid, scheme, limiter, C_T
CASES = [
    ("euler1d_mp6_trans", (40,), dict(ndim=1, n=[40], dx=[0.05], bc=[1], system=1), 6, 1, 1e-5),
    ("euler1d_tvdmm8_per", (36,), dict(ndim=1, n=[36], dx=[0.05], bc=[0], system=1), 8, 2, 1e-7),
    ("euler1d_teno6_trans", (30,), dict(ndim=1, n=[30], dx=[0.05], bc=[1], system=1), 6, 0, 1e-5),
    ("euler2d_mp6", (20, 23), dict(ndim=2, n=[23, 20], dx=[0.05, 0.06], bc=[0, 1], system=1), 6, 1, 1e-5),
    ("euler2d_tvd5_8", (14, 12), dict(ndim=2, n=[12, 14], dx=[0.05, 0.07], bc=[0, 1], system=1), 8, 3, 1e-7),
    ("euler2d_8a_va", (14, 12), dict(ndim=2, n=[12, 14], dx=[0.05, 0.07], bc=[1, 0], system=1), 8 | 0x100, 4, 0.0),
    ("euler2d_mpmm6", (12, 13), dict(ndim=2, n=[13, 12], dx=[0.06, 0.05], bc=[0, 0], system=1), 6, 6, 1e-5),
    ("scalar1d_mp8", (34,), dict(ndim=1, n=[34], dx=[0.05], bc=[0], system=0, adv=[-0.7]), 8, 1, 1e-7),
    ("scalar2d_va6", (15, 17), dict(ndim=2, n=[17, 15], dx=[0.05, 0.06], bc=[1, 0], system=0, adv=[0.6, -1.1]),
     6, 4, 1e-5),
    ("euler3d_mp6", (7, 8, 9), dict(ndim=3, n=[9, 8, 7], dx=[0.05, 0.06, 0.07], bc=[0, 1, 0], system=1), 6, 1, 1e-5),
    # lines as short as the stencil
    ("euler2d_min_mp6", (6, 6), dict(ndim=2, n=[6, 6], dx=[0.05, 0.06], bc=[0, 1], system=1), 6, 1, 1e-5),
    ("euler1d_min_mp8_per", (8,), dict(ndim=1, n=[8], dx=[0.05], bc=[0], system=1), 8, 1, 1e-7),
    ("scalar1d_min_tvd5_6_per", (6,), dict(ndim=1, n=[6], dx=[0.05], bc=[0], system=0, adv=[0.8]), 6, 3, 1e-5),
]
IDS = [c[0] for c in CASES]


def state(case, seed):
    """Mixed data with a 0.1 % random factor on every value (no
    characteristic field is zero up to rounding)."""
    shape, grid = case[1], case[2]
    if grid["system"] == 0:
        U = W.random_scalar_lines(shape, seed=seed, kind="mixed")
    else:
        U = W.random_euler_state(shape, seed=seed, kind="mixed")
    return U * (1.0 + 1e-3 * np.random.default_rng(seed + 1000).standard_normal(U.shape))


def band_cells(orc, U, grid, K, lim, C_T, reach):
    """Cells within `reach` of a face in the oracle's cutoff band."""
    nd = grid["ndim"]
    excl = np.zeros(U.shape[1:], dtype=bool)
    for axis in range(nd):
        _, _, bd = orc.reconstruct_faces(U, grid, K, lim, C_T, GAMMA, axis)
        excl |= faces_to_cells(band_faces(bd), nd - 1 - axis, grid["n"][axis], grid["bc"][axis] == 0, reach)
    return excl


@pytest.fixture(scope="module")
def T():
    require_gpu()
    import paper_2010_13289_amd as T
    return T


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_flux_divergence_vjp_matches_reference(T, orc, case):
    name, shape, grid, K, lim, C_T = case
    print(f"[vjp] {name}", flush=True)
    U = state(case, 4)
    Lbar = np.random.default_rng(5).standard_normal(U.shape)
    ref = RA.flux_divergence_vjp(U, Lbar, grid, K, lim, C_T, GAMMA)
    got = to_host(T.flux_divergence_vjp(to_dev(U), to_dev(Lbar), grid, K, lim, C_T, GAMMA))
    excl = band_cells(orc, U, grid, K, lim, C_T, K & 0xFF)
    assert excl.sum() <= excl.size // 10
    assert_close_fields(got, ref, exclude=excl, what=f"{name} VJP")


@pytest.mark.parametrize("K, lim, C_T", [(6, 1, 1e-5), (8, 1, 1e-7), (6, 3, 1e-5)], ids=["mp6", "mp8", "tvd5_6"])
def test_vjp_on_smooth_data_matches_reference(T, orc, K, lim, C_T):
    """Smooth 2D data, where almost every wavefront's reconstructions have
    all candidates smooth, so that the reverse skips the limiter's part (it
    would only add zeros): the VJP against the reference adjoint."""
    n = 48
    U, _ = _smooth_state(n)
    grid = dict(ndim=2, n=[n, n], dx=[1.0 / n, 1.0 / n], bc=[0, 0], system=1)
    print(f"[vjp smooth] K={K} lim={lim}", flush=True)
    nk = K - 2
    for axis in range(2):
        _, fl = T.reconstruct_faces(to_dev(U), grid, K, lim, C_T, GAMMA, axis, return_flags=True)
        rough = float(((fl & ((1 << nk) - 1)) != (1 << nk) - 1).double().mean())
        assert rough < 0.05, f"axis {axis}: {rough:.3f} of the reconstructions have a nonsmooth candidate"
    Lbar = np.random.default_rng(7).standard_normal(U.shape)
    ref = RA.flux_divergence_vjp(U, Lbar, grid, K, lim, C_T, GAMMA)
    got = to_host(T.flux_divergence_vjp(to_dev(U), to_dev(Lbar), grid, K, lim, C_T, GAMMA))
    excl = band_cells(orc, U, grid, K, lim, C_T, K)
    assert excl.sum() <= excl.size // 10
    assert_close_fields(got, ref, exclude=excl, what=f"smooth 2D VJP K={K} lim={lim}")


def test_vjp_scale_accumulate_and_determinism(T):
    case = CASES[3]
    name, shape, grid, K, lim, C_T = case
    U = state(case, 6)
    rng = np.random.default_rng(7)
    Lbar, base = rng.standard_normal(U.shape), rng.standard_normal(U.shape)
    Ud, Ld = to_dev(U), to_dev(Lbar)
    one = to_host(T.flux_divergence_vjp(Ud, Ld, grid, K, lim, C_T, GAMMA))
    again = to_host(T.flux_divergence_vjp(Ud, Ld, grid, K, lim, C_T, GAMMA))
    assert np.array_equal(one, again)
    out = to_dev(base)
    T.flux_divergence_vjp(Ud, Ld, grid, K, lim, C_T, GAMMA, out=out, scale=-0.5, accumulate=True)
    np.testing.assert_allclose(to_host(out), base - 0.5 * one, rtol=0, atol=1e-12 * np.abs(one).max())


@pytest.mark.parametrize("case", [CASES[0], CASES[1], CASES[3], CASES[5], CASES[7], CASES[9]],
                         ids=[IDS[0], IDS[1], IDS[3], IDS[5], IDS[7], IDS[9]])
def test_rk3_step_vjp_matches_reference(T, orc, case):
    name, shape, grid, K, lim, C_T = case
    print(f"[rk3 vjp] {name}", flush=True)
    U = state(case, 8)
    dt = 0.4 / orc.max_wave_speed(U, grid, GAMMA)
    Ubar = np.random.default_rng(9).standard_normal(U.shape)
    ref = RA.rk3_step_vjp(U, Ubar, grid, K, lim, C_T, GAMMA, dt)
    Bd = to_dev(Ubar)
    T.rk3_step_vjp(to_dev(U), Bd, grid, K, lim, C_T, GAMMA, dt)
    got = to_host(Bd)
    # the stage states' band faces, their cones through the three stages
    L0 = orc.flux_divergence(U, grid, K, lim, C_T, GAMMA)
    U1 = U + dt * L0
    U2 = 0.75 * U + 0.25 * (U1 + dt * orc.flux_divergence(U1, grid, K, lim, C_T, GAMMA))
    excl = np.zeros(U.shape[1:], dtype=bool)
    for S in (U, U1, U2):
        excl |= band_cells(orc, S, grid, K, lim, C_T, 3 * (K & 0xFF))
    assert excl.sum() <= excl.size // 5
    assert_close_fields(got, ref, exclude=excl, what=f"{name} RK3 VJP")


@pytest.mark.parametrize("case", [CASES[0], CASES[3], CASES[9]], ids=[IDS[0], IDS[3], IDS[9]])
def test_stage_entries_match_the_recomputing_ones(T, orc, case):
    """rk3_step(stages=...) updates U to the same bits and writes the stage
    states the step's adjoint recomputes: the adjoint given them equals the
    recomputing adjoint in every bit."""
    import torch
    name, shape, grid, K, lim, C_T = case
    U = state(case, 11)
    dt = 0.4 / orc.max_wave_speed(U, grid, GAMMA)
    Ud = to_dev(U)
    A, Bv = Ud.clone(), Ud.clone()
    S1, S2 = torch.empty_like(Ud), torch.empty_like(Ud)
    T.rk3_step(A, grid, K, lim, C_T, GAMMA, dt)
    T.rk3_step(Bv, grid, K, lim, C_T, GAMMA, dt, stages=(S1, S2))
    assert torch.equal(A, Bv)
    # U1 = U + dt L(U) up to the sweeps' rounding
    L0 = to_host(T.flux_divergence(Ud, grid, K, lim, C_T, GAMMA))
    np.testing.assert_allclose(to_host(S1), U + dt * L0, rtol=1e-13, atol=1e-13 * np.abs(U).max())
    Ubar = to_dev(np.random.default_rng(12).standard_normal(U.shape))
    g1, g2 = Ubar.clone(), Ubar.clone()
    T.rk3_step_vjp(Ud, g1, grid, K, lim, C_T, GAMMA, dt)
    T.rk3_step_vjp(Ud, g2, grid, K, lim, C_T, GAMMA, dt, stages=(S1, S2))
    assert torch.equal(g1, g2)


def _smooth_state(n):
    """Smooth 2D data with every field varying along both axes."""
    x = W.cell_centres(n, 0.0, 1.0)
    Y, X = np.meshgrid(x, x, indexing="ij")
    tp = 2 * np.pi
    rho = 1.0 + 0.2 * np.sin(tp * (X + 2 * Y) + 0.3)
    u = 0.3 * np.cos(tp * (2 * X - Y) + 1.1)
    v = 0.2 * np.sin(tp * (X + Y) + 2.0)
    p = 1.0 + 0.1 * np.cos(tp * (X - 3 * Y) + 0.7)
    target = 1.0 + 0.1 * np.cos(tp * (3 * X + Y))
    return W.conservative(rho, [u, v], p, GAMMA), target


def _rollout_loss(T, grid, K, lim, C_T, dt, steps, target):
    def loss(U, ck):
        Uf = T.rollout(U, grid, K, lim, C_T, GAMMA, dt, steps, checkpoint=ck)
        return 0.5 * ((Uf[0] - target) ** 2).sum()
    return loss


def test_rollout_gradient_checkpointing_is_exact(T):
    """12 fixed steps, TENO6-M-MP: the backward with a checkpoint every 5
    steps (replayed segments) equals the one-segment backward in every bit."""
    n = 40
    grid = dict(ndim=2, n=[n, n], dx=[1.0 / n] * 2, bc=[0, 0], system=1)
    U0, tgt = _smooth_state(n)
    dt = 0.3 / T.max_wave_speed(to_dev(U0), grid, GAMMA)
    loss = _rollout_loss(T, grid, 6, T.LIM_MP, 1e-5, dt, 12, to_dev(tgt))
    grads = []
    for ck in (5, 12, 1):
        U = to_dev(U0).requires_grad_(True)
        loss(U, ck).backward()
        grads.append(U.grad.detach().cpu().numpy())
    assert np.array_equal(grads[0], grads[1]) and np.array_equal(grads[0], grads[2])
    assert np.all(np.isfinite(grads[0])) and np.abs(grads[0]).max() > 0


def test_rollout_gradient_matches_differences(T):
    """With C_T = 0 every candidate is smooth (the K-point linear scheme with
    Rusanov splitting and the characteristic projection, no cutoff decision),
    so the 12-step rollout is smooth around the state and central
    differences of the GPU forward converge to the gradient.  (With the
    cutoff on, decisions at under-resolved extrema change within 1e-6 of
    the state; the per-step adjoint with frozen decisions is checked against
    the reference above.)"""
    import torch
    n = 40
    grid = dict(ndim=2, n=[n, n], dx=[1.0 / n] * 2, bc=[0, 0], system=1)
    U0, tgt = _smooth_state(n)
    dt = 0.3 / T.max_wave_speed(to_dev(U0), grid, GAMMA)
    loss = _rollout_loss(T, grid, 6, T.LIM_MP, 0.0, dt, 12, to_dev(tgt))
    U = to_dev(U0).requires_grad_(True)
    loss(U, 5).backward()
    g = U.grad.detach().cpu().numpy()
    rng = np.random.default_rng(34)
    scale = np.abs(U0).max(axis=(1, 2), keepdims=True)
    with torch.no_grad():
        for d in range(6):
            V = rng.standard_normal(U0.shape) * scale
            fd = []
            for h in (1e-5, 1e-6):
                lp = loss(to_dev(U0 + h * V), 12).item()
                lm = loss(to_dev(U0 - h * V), 12).item()
                fd.append((lp - lm) / (2 * h))
            ad = float(np.sum(g * V))
            print(f"[rollout grad] direction {d}: fd {fd} adjoint {ad}", flush=True)
            assert abs(fd[0] - fd[1]) <= 1e-6 * abs(fd[1])
            assert abs(fd[1] - ad) <= 1e-7 * abs(ad), (d, fd, ad)


def test_rollout_gradient_with_the_cutoff_on(T):
    """TENO6-M-MP with C_T = 1e-5 over 24 fixed steps (checkpoint 20, so
    two replayed segments) on a moving 2D state: 64 density modes (|k| <= 8)
    and a jump on a circle, set in motion by small velocity and pressure
    perturbations (|k| <= 4) so that every characteristic field carries a
    signal.  Directions are smooth and local (random-phase fields under a
    Gaussian window), so that a step along them moves the smoothness
    indicators by about the state's own relative amount.  A direction
    counts where the rollouts from U +- hV (h = 1e-8) take every smoothness
    decision of every stage as the rollout from U, and the differences at
    h and h/2 agree to 1e-6 (no limiter kink crossed, and rounding in the
    differences resolves 1e-6 along that direction); at least 8 must count,
    and on each the frozen-decision gradient equals the central difference
    at h to 1e-6.  The difference is taken on the final states,
    L(U+) - L(U-) = sum (rho+ - rho-)(rho+ + rho- - 2 rho_T) / 2."""
    import torch
    n, steps, ck, C_T = 128, 24, 20, 1e-5
    grid = dict(ndim=2, n=[n, n], dx=[1.0 / n] * 2, bc=[0, 0], system=1)
    U0h, _ = W.moving_density_modes_2d(n, seed=5, kmax=4.0, density_kmax=8)
    Th, _ = W.moving_density_modes_2d(n, seed=6, kmax=4.0, density_kmax=8)
    U0 = to_dev(U0h)
    dt = 0.4 / T.max_wave_speed(U0, grid, GAMMA)
    target = T.rollout(to_dev(Th), grid, 6, T.LIM_MP, C_T, GAMMA, dt, steps, checkpoint=steps).detach()[0].clone()
    U = U0.clone().requires_grad_(True)
    _rollout_loss(T, grid, 6, T.LIM_MP, C_T, dt, steps, target)(U, ck).backward()
    g = U.grad.detach()
    assert bool(torch.isfinite(g).all()) and float(g.abs().max()) > 0

    def final_rho(V):
        return T.rollout(V, grid, 6, T.LIM_MP, C_T, GAMMA, dt, steps, checkpoint=steps)[0]

    def central(V, h):
        with torch.no_grad():
            rp, rm = final_rho(U0 + h * V), final_rho(U0 - h * V)
            return float((0.5 * (rp - rm) * (rp + rm - 2.0 * target)).sum().item()) / (2.0 * h)

    ref = T.rollout_flags(U0, grid, 6, T.LIM_MP, C_T, GAMMA, dt, steps)
    scale = torch.from_numpy(np.abs(U0h).max(axis=(1, 2), keepdims=True)).to(U0.device)
    h = 1e-8
    usable, tried = 0, 0
    while usable < 8 and tried < 32:
        V = to_dev(W.local_direction_2d(U0h.shape, seed=tried)) * scale
        tried += 1
        same = (T.rollout_flags(U0 + h * V, grid, 6, T.LIM_MP, C_T, GAMMA, dt, steps, ref=ref)
                and T.rollout_flags(U0 - h * V, grid, 6, T.LIM_MP, C_T, GAMMA, dt, steps, ref=ref))
        fd, fd2 = central(V, h), central(V, h / 2)
        ad = float((g * V).sum().item())
        print(f"[rollout grad C_T=1e-5] direction {tried}: same decisions {same}, fd {fd:.12e} "
              f"(h/2: {fd2:.12e}), adjoint {ad:.12e}", flush=True)
        if not same or abs(fd - fd2) > 1e-6 * abs(fd):
            continue
        usable += 1
        assert abs(fd - ad) <= 1e-6 * abs(ad), (tried, fd, ad)
    assert usable >= 8, f"only {usable} of {tried} directions kept every decision"
