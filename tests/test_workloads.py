"""The seeded input generators: determinism, shapes and physical ranges."""
import math

import numpy as np

import workloads as W


def test_generators_are_deterministic():
    a, _ = W.tgv_3d(16)
    b, _ = W.tgv_3d(16)
    np.testing.assert_array_equal(a, b)
    assert W.riemann_states(3) == W.riemann_states(3)
    np.testing.assert_array_equal(W.random_euler_state((5, 6), 4), W.random_euler_state((5, 6), 4))


def test_tgv_3d_recipe():
    n = 32
    U, dx = W.tgv_3d(n)
    assert U.shape == (5, n, n, n) and U.flags.c_contiguous and dx == 2 * math.pi / n
    x = W.cell_centres(n, 0, 2 * math.pi)
    rho = U[0]
    np.testing.assert_array_equal(rho[:, :, x < math.pi], 1.0)
    np.testing.assert_array_equal(rho[:, :, x >= math.pi], 0.125)
    u = U[1] / rho
    base = np.sin(x)[None, None, :] * np.cos(x)[None, :, None] * np.cos(x)[:, None, None]
    assert abs(np.max(np.abs(u - base)) - 1e-2) < 1e-12  # perturbation amplitude
    w = U[3] / rho
    assert abs(np.max(np.abs(w)) - 1e-2) < 1e-12
    p = 0.4 * (U[4] - 0.5 * (U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / rho)
    assert 99.5 - 1e-9 <= p.min() and p.max() <= 100.25 + 1e-9  # 100 + [-1/2, 1/4]


def test_riemann_state_ranges():
    for s in range(50):
        (rl, ul, pl), (rr, ur, pr) = W.riemann_states(s)
        assert 0.1 <= rl <= 1 and 0.1 <= rr <= 1 and 0.1 <= pl <= 1 and 0.1 <= pr <= 1
        assert -1 <= ul <= 1 and -1 <= ur <= 1


def test_batched_sizes():
    n = W.batched_riemann_sizes()
    assert len(n) == 4096 and n.min() >= 256 and n.max() <= 16384
    assert 3000 < n.mean() < 4500


def test_random_euler_positive():
    for kind in ("smooth", "jumps", "mixed"):
        U = W.random_euler_state((7, 8, 9), 11, kind=kind)
        rho = U[0]
        p = 0.4 * (U[4] - 0.5 * (U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / rho)
        assert rho.min() > 0 and p.min() > 0
