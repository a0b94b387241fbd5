"""The SSP-RK3 step with its size from the CFL condition on the device
(tenom_rk3_step_cfl): the same bits and the same dt as tenom_max_wave_speed
on the host followed by tenom_rk3_step, replays of a captured HIP graph of
several such steps, and a non-finite state."""
import numpy as np
import pytest

import workloads as W
from parity import require_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu

GAMMA = 1.4
CFL = 0.4

# name, shape (z, y, x order), system, bc (x, y, z order), scheme, limiter, C_T, adv
CASES = [
    ("euler3d_mp6", (10, 12, 33), 1, [0, 1, 0], 6, 1, 1e-5, None),
    ("euler2d_tvd5_8", (33, 65), 1, [1, 0], 8, 3, 1e-6, None),
    ("euler1d_8a_mp", (400,), 1, [1], 8 | 0x100, 1, 0.0, None),
    ("scalar2d_mp6", (20, 70), 0, [0, 1], 6, 1, 1e-5, [0.5, -1.2]),
    # more cells than 4096 blocks of 256 threads: every rate block covers several cells
    ("euler2d_1100x1000", (1000, 1100), 1, [0, 0], 6, 1, 1e-5, None),
]
IDS = [c[0] for c in CASES]


@pytest.fixture(scope="module")
def T():
    require_gpu()
    import paper_2010_13289_amd as T
    return T


def make(case, seed=0):
    name, shape, system, bc, K, lim, C_T, adv = case
    nd = len(shape)
    grid = dict(ndim=nd, n=list(reversed(shape)), dx=[0.05, 0.07, 0.06][:nd], bc=bc, system=system,
                adv=adv or [0.0] * nd)
    if system == 0:
        U = W.random_scalar_lines(shape, seed=seed + 300, kind="mixed")
    else:
        U = W.random_euler_state(shape, seed=seed + 400, kind="mixed")
    return grid, U, K, lim, C_T


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_cfl_step_matches_the_host_step_size(T, case):
    import torch
    grid, U, K, lim, C_T = make(case)
    print(f"[rk3_step_cfl] {case[0]}", flush=True)
    Ua, Ub = to_dev(U), to_dev(U)
    ws = T.Workspace(grid, K)
    dto = torch.zeros(1, dtype=torch.float64, device="cuda")
    for step in range(3):
        dt = CFL / T.max_wave_speed(Ua, grid, GAMMA)
        T.rk3_step(Ua, grid, K, lim, C_T, GAMMA, dt, workspace=ws)
        T.rk3_step_cfl(Ub, grid, K, lim, C_T, GAMMA, CFL, workspace=ws, dt_out=dto)
        assert dto.item() == dt, (step, dto.item(), dt)
        assert np.array_equal(to_host(Ub), to_host(Ua)), f"step {step}"


def test_cfl_steps_in_a_captured_graph(T):
    """Three CFL steps captured once and replayed four times, with eager
    work and synchronisations between the replays; every replay against the
    same steps taken eagerly."""
    import torch
    grid, U, K, lim, C_T = make(CASES[0], seed=5)
    Ug, Ue = to_dev(U), to_dev(U)
    wsg, wse = T.Workspace(grid, K), T.Workspace(grid, K)
    dtg = torch.zeros(1, dtype=torch.float64, device="cuda")
    dte = torch.zeros(1, dtype=torch.float64, device="cuda")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(3):
            T.rk3_step_cfl(Ug, grid, K, lim, C_T, GAMMA, CFL, workspace=wsg, dt_out=dtg)
    # capture records the launches without running them
    assert np.array_equal(to_host(Ug), U)
    for rep in range(4):
        print(f"[graph replay] {rep}", flush=True)
        g.replay()
        for _ in range(3):
            T.rk3_step_cfl(Ue, grid, K, lim, C_T, GAMMA, CFL, workspace=wse, dt_out=dte)
        torch.cuda.synchronize()
        assert np.array_equal(to_host(Ug), to_host(Ue)), f"replay {rep}"
        assert dtg.item() == dte.item()
        # unrelated eager work on the same device between the replays
        scratch = torch.randn(1 << 20, dtype=torch.float64, device="cuda")
        scratch.sum().item()
    del g


def test_nonfinite_state_gives_nonfinite_step(T):
    import torch
    grid, U, K, lim, C_T = make(CASES[0], seed=7)
    U = U.copy()
    U[0, 3, 4, 5] = np.nan
    Ud = to_dev(U)
    dto = torch.zeros(1, dtype=torch.float64, device="cuda")
    T.rk3_step_cfl(Ud, grid, K, lim, C_T, GAMMA, CFL, workspace=T.Workspace(grid, K), dt_out=dto)
    assert np.isnan(dto.item())
    assert not T.check_finite(Ud, grid)
