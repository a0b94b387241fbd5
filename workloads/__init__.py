"""Seeded synthetic inputs for the TENO-M reconstruction path.

This module only builds input arrays: grids of cell-centre coordinates,
initial conditions and random states.  It holds none of the scheme's
arithmetic (no stencils, indicators, limiters, fluxes or time stepping), so
both the CPU oracle's tests and the GPU path's tests and benchmark can draw
identical inputs from it without sharing any of the method.

Conventions
-----------
* Point values at cell centres, x_i = a + (i + 1/2) * dx (the scheme is a
  finite-difference scheme on point values, Sec. 2).
* Arrays are float64, C-contiguous, structure of arrays ``[field][z][y][x]``
  with x fastest; 1D arrays are ``[field][x]`` and 2D ``[field][y][x]``.
* Euler fields are (rho, rho*u, [rho*v], [rho*w], E) with
  E = p/(gamma-1) + rho*|u|^2/2 (ideal gas).
* Every random draw goes through ``numpy.random.default_rng(seed)`` with the
  seed stated in the function.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "cell_centres",
    "conservative",
    "advection_sine_pulse",
    "gaussian_pulse",
    "multiwave",
    "square_wave",
    "riemann_states",
    "riemann_problem",
    "SOD",
    "LAX",
    "tgv_3d",
    "random_scalar_lines",
    "random_euler_state",
    "batched_riemann_sizes",
    "density_modes_2d",
]


def cell_centres(n: int, a: float, b: float) -> np.ndarray:
    """Cell-centre coordinates of n uniform cells on [a, b]."""
    dx = (b - a) / n
    return a + (np.arange(n, dtype=np.float64) + 0.5) * dx


def conservative(rho, vel, p, gamma: float) -> np.ndarray:
    """Stack primitive fields into conservative ones.

    ``vel`` is a sequence of ndim velocity arrays.  Returns
    ``[rho, rho*u_0, ..., rho*u_{ndim-1}, E]`` as one float64 array.
    """
    rho = np.asarray(rho, dtype=np.float64)
    vel = [np.broadcast_to(np.asarray(v, dtype=np.float64), rho.shape) for v in vel]
    p = np.broadcast_to(np.asarray(p, dtype=np.float64), rho.shape)
    ke = 0.5 * rho * sum(v * v for v in vel)
    out = [rho] + [rho * v for v in vel] + [p / (gamma - 1.0) + ke]
    return np.ascontiguousarray(np.stack(out))


# --------------------------------------------------------------------------
# 1D scalar advection inputs
# --------------------------------------------------------------------------

def advection_sine_pulse(n: int = 200, pulse: bool = True) -> tuple[np.ndarray, float]:
    """u0 = sin(pi x) on periodic [-1, 1], plus a unit square pulse on
    [-0.4, -0.2] when ``pulse`` (the smooth part alone serves order studies).

    Returns (u[1][n], dx).
    """
    x = cell_centres(n, -1.0, 1.0)
    u = np.sin(np.pi * x)
    if pulse:
        u = u + ((x >= -0.4) & (x <= -0.2)).astype(np.float64)
    return u[None, :].copy(), 2.0 / n


def gaussian_pulse(n: int) -> tuple[np.ndarray, float]:
    """Gaussian pulse exp(-300 (x - 0.5)^2) on periodic [0, 1] (Sec. 4.1.1)."""
    x = cell_centres(n, 0.0, 1.0)
    return np.exp(-300.0 * (x - 0.5) ** 2)[None, :].copy(), 1.0 / n


def multiwave(n: int = 200) -> tuple[np.ndarray, float]:
    """Jiang-Shu multi-wave initial condition on [0, 2] as stated in Sec. 4.1.2:
    Gaussians, a square wave, a triangle and a half ellipse."""
    x = cell_centres(n, 0.0, 2.0)
    a, z, theta, alpha = 0.5, -0.7, 0.005, 10.0
    beta = math.log(2.0) / (36.0 * theta * theta)

    def G(xx, b, zz):
        return np.exp(-b * (xx - zz) ** 2)

    def F(xx, al, aa):
        return np.sqrt(np.maximum(1.0 - al * al * (xx - aa) ** 2, 0.0))

    u = np.zeros(n)
    m = (x >= 0.2) & (x < 0.4)
    xs = x[m] - 1.0
    u[m] = (G(xs, beta, z - theta) + G(xs, beta, z + theta) + 4.0 * G(xs, beta, z)) / 6.0
    m = (x >= 0.6) & (x <= 0.8)
    u[m] = 1.0
    m = (x >= 1.0) & (x <= 1.2)
    u[m] = 1.0 - np.abs(10.0 * (x[m] - 1.1))
    m = (x >= 1.4) & (x < 1.6)
    xs = x[m] - 1.0
    u[m] = (F(xs, alpha, a - theta) + F(xs, alpha, a + theta) + 4.0 * F(xs, alpha, a)) / 6.0
    return u[None, :].copy(), 2.0 / n


def square_wave(n: int, lo: float = 0.25, hi: float = 0.5) -> tuple[np.ndarray, float]:
    """Unit square wave on periodic [0, 1] (value 1 on [lo, hi], else 0)."""
    x = cell_centres(n, 0.0, 1.0)
    return (((x >= lo) & (x <= hi)).astype(np.float64))[None, :].copy(), 1.0 / n


# --------------------------------------------------------------------------
# 1D Euler: Riemann problems
# --------------------------------------------------------------------------

# CFL number of every run (Sec. 4: CFL 0.4 with the SSP Runge-Kutta step;
# Sec. 3.2.2 chooses the MP alpha so that CFL <= 1/(1 + alpha) holds)
CFL = 0.4

# (rho, u, p) left and right states of the shock tubes (Sec. 4.2.1)
SOD = ((1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
LAX = ((0.445, 0.698, 3.528), (0.5, 0.0, 0.5710))


def riemann_states(seed: int) -> tuple[tuple[float, float, float], tuple[float, float, float]]:
    """Seeded Riemann states: rho in [0.1, 1], u in [-1, 1], p in [0.1, 1].

    One ``default_rng(seed).uniform`` call draws a (2, 3) array: row 0 is the
    left state (rho, u, p), row 1 the right one.
    """
    rng = np.random.default_rng(seed)
    s = rng.uniform([0.1, -1.0, 0.1], [1.0, 1.0, 1.0], size=(2, 3))
    return tuple(float(v) for v in s[0]), tuple(float(v) for v in s[1])


def riemann_problem(n: int, left, right, gamma: float = 1.4, x0: float = 0.5,
                    a: float = 0.0, b: float = 1.0) -> tuple[np.ndarray, float]:
    """Piecewise-constant 1D Euler state on [a, b] split at x0 (x < x0: left).

    Returns (U[3][n], dx)."""
    x = cell_centres(n, a, b)
    lm = x < x0
    rho = np.where(lm, left[0], right[0])
    u = np.where(lm, left[1], right[1])
    p = np.where(lm, left[2], right[2])
    return conservative(rho, [u], p, gamma), (b - a) / n


def batched_riemann_sizes(count: int = 4096, lo: int = 256, hi: int = 16384,
                          seed: int = 4096) -> np.ndarray:
    """Ragged problem sizes, log-uniform in [lo, hi] (``default_rng(seed)``)."""
    rng = np.random.default_rng(seed)
    e = rng.uniform(math.log(lo), math.log(hi), size=count)
    return np.clip(np.rint(np.exp(e)), lo, hi).astype(np.int64)


# --------------------------------------------------------------------------
# 3D Euler: Taylor-Green vortex with a density jump and seeded perturbations
# --------------------------------------------------------------------------

def _random_phase_field(n: int, kmax: float, seed: int, amp: float) -> np.ndarray:
    """Real periodic field on an n^3 grid: unit-magnitude modes with uniform
    random phase for integer wavevectors 1 <= |k|_2 <= kmax, scaled so that
    max|field| = amp.  Array order [z][y][x]."""
    rng = np.random.default_rng(seed)
    kz = np.fft.fftfreq(n, d=1.0 / n)[:, None, None]
    ky = np.fft.fftfreq(n, d=1.0 / n)[None, :, None]
    kx = np.fft.rfftfreq(n, d=1.0 / n)[None, None, :]
    kk = np.sqrt(kx * kx + ky * ky + kz * kz)
    phase = rng.uniform(0.0, 2.0 * math.pi, size=kk.shape)
    spec = np.where((kk >= 1.0) & (kk <= kmax), np.exp(1j * phase), 0.0)
    f = np.fft.irfftn(spec, s=(n, n, n), axes=(0, 1, 2))
    return f * (amp / np.max(np.abs(f)))


def tgv_3d(n: int = 256, gamma: float = 1.4, kmax: float | None = None,
           amp: float = 1e-2, seed_base: int = 201013289,
           rho_jump: tuple[float, float] = (1.0, 0.125)) -> tuple[np.ndarray, float]:
    """Inviscid Taylor-Green velocity and pressure (Sec. 4.3.1) on the periodic
    cube [0, 2 pi)^3, with density rho_jump[0] for x < pi and rho_jump[1] for
    x >= pi, plus random-phase perturbations of u, v, w.

    The perturbation of velocity component c (0, 1, 2 = u, v, w) uses
    ``default_rng(seed_base + c)`` and modes 1 <= |k| <= kmax with
    kmax = 16 (capped at n/4 for small test grids), scaled to max|du| = amp.
    Returns (U[5][n][n][n], dx).
    """
    if kmax is None:
        kmax = min(16.0, n / 4.0)
    x1 = cell_centres(n, 0.0, 2.0 * math.pi)
    z, y, x = np.meshgrid(x1, x1, x1, indexing="ij")
    u = np.sin(x) * np.cos(y) * np.cos(z)
    v = -np.cos(x) * np.sin(y) * np.cos(z)
    w = np.zeros_like(u)
    p = 100.0 + ((np.cos(2 * x) + np.cos(2 * y)) * (2.0 + np.cos(2 * z)) - 2.0) / 16.0
    rho = np.where(x < math.pi, rho_jump[0], rho_jump[1])
    for c, comp in enumerate((u, v, w)):
        comp += _random_phase_field(n, kmax, seed_base + c, amp)
    del z, y
    return conservative(rho, [u, v, w], p, gamma), 2.0 * math.pi / n


# --------------------------------------------------------------------------
# Generic random inputs for per-call parity tests
# --------------------------------------------------------------------------

def random_scalar_lines(shape, seed: int, kind: str = "mixed") -> np.ndarray:
    """Random scalar data of the given grid shape (z, y, x order, any ndim).

    kind: "smooth" (a few random Fourier modes), "noise" (iid normal),
    "steps" (piecewise constant with random jumps), or "mixed" (smooth +
    steps + a little noise).  Returns a float64 array of ``shape`` with a
    leading field axis of length 1.
    """
    rng = np.random.default_rng(seed)
    shape = tuple(int(s) for s in shape)
    grids = np.meshgrid(*[np.linspace(0.0, 2.0 * math.pi, s, endpoint=False) for s in shape],
                        indexing="ij")
    smooth = np.zeros(shape)
    for _ in range(4):
        ph = rng.uniform(0, 2 * math.pi)
        arg = sum(int(rng.integers(-3, 4)) * g for g in grids) + ph
        smooth += rng.uniform(0.2, 1.0) * np.sin(arg)
    steps = np.zeros(shape)
    for _ in range(3):
        axis = int(rng.integers(0, len(shape)))
        cut = int(rng.integers(1, max(2, shape[axis])))
        idx = [slice(None)] * len(shape)
        idx[axis] = slice(cut, None)
        steps[tuple(idx)] += rng.uniform(-2.0, 2.0)
    noise = rng.standard_normal(shape)
    if kind == "smooth":
        out = smooth
    elif kind == "noise":
        out = noise
    elif kind == "steps":
        out = steps + 0.5
    elif kind == "mixed":
        out = smooth + steps + 0.05 * noise
    else:
        raise ValueError(kind)
    return np.ascontiguousarray(out[None].astype(np.float64))


def random_euler_state(shape, seed: int, gamma: float = 1.4, kind: str = "mixed") -> np.ndarray:
    """Random positive-density, positive-pressure Euler state on a grid of the
    given shape (z, y, x order; ndim = len(shape)).

    kind: "smooth" (waves), "jumps" (waves plus density/pressure/velocity
    jumps) or "mixed" (jumps plus 1% cell noise).  Returns U[ndim+2][shape].
    """
    rng = np.random.default_rng(seed)
    shape = tuple(int(s) for s in shape)
    nd = len(shape)
    grids = np.meshgrid(*[np.linspace(0.0, 2.0 * math.pi, s, endpoint=False) for s in shape],
                        indexing="ij")

    def wave(scale):
        f = np.zeros(shape)
        for _ in range(3):
            ph = rng.uniform(0, 2 * math.pi)
            arg = sum(int(rng.integers(-2, 3)) * g for g in grids) + ph
            f += scale * rng.uniform(0.3, 1.0) * np.sin(arg)
        return f

    rho = 1.0 + wave(0.15)
    p = 1.0 + wave(0.15)
    vel = [wave(0.3) for _ in range(nd)]
    if kind in ("jumps", "mixed"):
        for _ in range(2):
            axis = int(rng.integers(0, nd))
            cut = int(rng.integers(1, max(2, shape[axis])))
            idx = [slice(None)] * nd
            idx[axis] = slice(cut, None)
            rho[tuple(idx)] *= rng.uniform(0.2, 0.9)
            p[tuple(idx)] *= rng.uniform(0.1, 0.9)
            vel[axis][tuple(idx)] += rng.uniform(-0.5, 0.5)
    if kind == "mixed":
        rho *= 1.0 + 0.01 * rng.standard_normal(shape)
        p *= 1.0 + 0.01 * rng.standard_normal(shape)
    elif kind not in ("smooth", "jumps"):
        raise ValueError(kind)
    return conservative(rho, vel, p, gamma)


def density_modes_2d(n: int = 1024, seed: int = 5, modes: int = 64, kmax: int = 32,
                     amp: float = 0.05, radius: float = 0.2,
                     gamma: float = 1.4) -> tuple[np.ndarray, float]:
    """2D periodic [0,1)^2 state: density 1 + a seeded sum of ``modes`` Fourier
    modes (integer 0 < |k| <= kmax, random phases) scaled so that the sum has
    max amplitude ``amp`` (so the density stays positive), times 0.5 inside a
    circle of the given radius at the centre; u = v = 0, p = 1.
    Returns (U[4][n][n], dx)."""
    rng = np.random.default_rng(seed)
    x1 = cell_centres(n, 0.0, 1.0)
    y, x = np.meshgrid(x1, x1, indexing="ij")
    pert = np.zeros((n, n))
    for _ in range(modes):
        while True:
            kx, ky = (int(k) for k in rng.integers(-kmax, kmax + 1, size=2))
            if 0 < kx * kx + ky * ky <= kmax * kmax:
                break
        pert += np.cos(2 * math.pi * (kx * x + ky * y) + rng.uniform(0, 2 * math.pi))
    rho = 1.0 + pert * (amp / np.max(np.abs(pert)))
    rho = np.where((x - 0.5) ** 2 + (y - 0.5) ** 2 < radius * radius, 0.5 * rho, rho)
    zero = np.zeros_like(rho)
    return conservative(rho, [zero, zero], 1.0, gamma), 1.0 / n


def smooth_direction_2d(shape, seed: int, kmax: float = 8.0) -> np.ndarray:
    """A random direction for difference checks on an [nf][n][n] state: per
    field a seeded random-phase field with modes 1 <= |k| <= kmax and max
    magnitude 1 (smooth, so that a small step along it changes the
    smoothness indicators by about the same relative amount as the state)."""
    nf, n = shape[0], shape[1]
    return np.stack([_random_phase_field_2d(n, min(kmax, n / 4.0), 7919 * seed + f, 1.0) for f in range(nf)])


def local_direction_2d(shape, seed: int, width: float = 1.0 / 16.0, kmax: float = 8.0) -> np.ndarray:
    """smooth_direction_2d(shape, seed) times a Gaussian window of the given
    width (a fraction of the periodic unit square) centred at a seeded
    random point: a smooth direction whose influence stays local."""
    n = shape[1]
    rng = np.random.default_rng(104729 + seed)
    cx, cy = rng.uniform(0.0, 1.0, size=2)
    x1 = cell_centres(n, 0.0, 1.0)
    dx_ = np.abs(x1 - cx)
    dy_ = np.abs(x1 - cy)
    dx_ = np.minimum(dx_, 1.0 - dx_)  # periodic distance
    dy_ = np.minimum(dy_, 1.0 - dy_)
    win = np.exp(-(dy_[:, None] ** 2 + dx_[None, :] ** 2) / (2.0 * width * width))
    return smooth_direction_2d(shape, seed, kmax) * win[None]


def _random_phase_field_2d(n: int, kmax: float, seed: int, amp: float) -> np.ndarray:
    """Real periodic field on an n^2 grid: unit-magnitude modes with uniform
    random phase for integer wavevectors 1 <= |k|_2 <= kmax, scaled so that
    max|field| = amp.  Array order [y][x]."""
    rng = np.random.default_rng(seed)
    ky = np.fft.fftfreq(n, d=1.0 / n)[:, None]
    kx = np.fft.rfftfreq(n, d=1.0 / n)[None, :]
    kk = np.sqrt(kx * kx + ky * ky)
    phase = rng.uniform(0.0, 2.0 * math.pi, size=kk.shape)
    spec = np.where((kk >= 1.0) & (kk <= kmax), np.exp(1j * phase), 0.0)
    f = np.fft.irfftn(spec, s=(n, n), axes=(0, 1))
    return f * (amp / np.max(np.abs(f)))


def moving_density_modes_2d(n: int = 1024, seed: int = 5, amp: float = 1e-2, kmax: float = 16.0,
                            density_kmax: int = 32, gamma: float = 1.4) -> tuple[np.ndarray, float]:
    """density_modes_2d(n, seed, kmax=density_kmax) set in motion: seeded
    random-phase velocity perturbations (max |u|, |v| = amp) and a pressure
    1 + a perturbation of max amp, modes 1 <= |k| <= kmax (capped at n/4),
    seeds 1000 seed + 1..3.  Every characteristic field then carries a
    signal far above rounding.  Returns (U[4][n][n], dx)."""
    U, dx = density_modes_2d(n, seed=seed, kmax=density_kmax, gamma=gamma)
    rho = U[0]
    km = min(kmax, n / 4.0)
    u = _random_phase_field_2d(n, km, 1000 * seed + 1, amp)
    v = _random_phase_field_2d(n, km, 1000 * seed + 2, amp)
    p = 1.0 + _random_phase_field_2d(n, km, 1000 * seed + 3, amp)
    return conservative(rho, [u, v], p, gamma), dx

