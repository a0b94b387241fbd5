"""The allocation-free SSP-RK3 step (tenom_rk3_step_cfl_noalloc, scratch in
the library's static device array) against tenom_rk3_step_cfl with a caller
workspace: the same kernels, so the same bits, on two calls in a row, the
second on a smaller grid (the array keeps the first call's contents)."""
import ctypes as C

import numpy as np
import pytest
import torch

import paper_2010_13289_amd as T
import workloads as W
from parity import require_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu
GAMMA = 1.4


def _cases():
    # a 2D grid that fills most of the 128 MiB scratch, then a small 3D one
    big = dict(ndim=2, n=[1024, 1000], dx=[1.0 / 1024, 1.0 / 1000], bc=[0, 1], system=1)
    small = dict(ndim=3, n=[24, 20, 18], dx=[0.1, 0.11, 0.12], bc=[0, 1, 0], system=1)
    return [(big, lambda: W.random_euler_state((1000, 1024), seed=3), 6, T.LIM_MP, 1e-5),
            (small, lambda: W.random_euler_state((18, 20, 24), seed=5), 8, T.LIM_TVD5, 1e-7)]


def test_noalloc_step_matches_the_workspace_step():
    require_gpu()
    assert T.static_scratch_bytes() == 128 << 20
    for grid, make, scheme, lim, ct in _cases():
        print(f"[no-alloc step] grid {grid['n']} K={scheme} limiter={lim}", flush=True)
        need = T.workspace_bytes(grid, scheme)
        assert 0 < need <= T.static_scratch_bytes()
        U0 = make()
        Ua, Ub = to_dev(U0), to_dev(U0)
        dta = torch.zeros(1, dtype=torch.float64, device="cuda")
        dtb = torch.zeros(1, dtype=torch.float64, device="cuda")
        ws = T.Workspace(grid, scheme)
        T.rk3_step_cfl(Ua, grid, scheme, lim, ct, GAMMA, W.CFL, workspace=ws, dt_out=dta)
        T.rk3_step_cfl_noalloc(Ub, grid, scheme, lim, ct, GAMMA, W.CFL, dt_out=dtb)
        torch.cuda.synchronize()
        assert to_host(dtb)[0] == to_host(dta)[0] and np.isfinite(to_host(dta)[0])
        a, b = to_host(Ua), to_host(Ub)
        assert np.all(np.isfinite(b))
        assert np.array_equal(a, b), np.abs(a - b).max()
        assert not np.array_equal(b, U0)


def test_noalloc_step_rejects_grids_beyond_the_scratch():
    require_gpu()
    grid = dict(ndim=3, n=[128, 128, 128], dx=[0.1] * 3, bc=[0, 0, 0], system=1)
    assert T.workspace_bytes(grid, 6) > T.static_scratch_bytes()
    U = torch.ones((5, 128, 128, 128), dtype=torch.float64, device="cuda")
    with pytest.raises(T.TenomError) as e:
        T.rk3_step_cfl_noalloc(U, grid, 6, T.LIM_MP, 1e-5, GAMMA, W.CFL)
    assert e.value.code == T.EWORKSPACE
