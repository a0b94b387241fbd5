"""Throughput benchmark of the TENO-M path on one MI355X.

One step = one SSP-RK3 step of the 3D Euler equations on a 256^3 periodic
cube (the Taylor-Green velocity and pressure of Sec. 4.3.1, a planar
density jump 1 -> 0.125 at x = pi, seeded random-phase velocity
perturbations), six-point TENO-M with the MP limiter, C_T = 1e-5,
gamma = 1.4, CFL 0.4: the wave-speed reduction and dt on the device
(tenom_rk3_step_cfl, no host round trip), then 3 stages x (x, y, z) sweeps
of face reconstructions, divergence and stage update.
Unit: one face vector (the full 5-component flux at one face, both split
sides), 3 stages x 3 axes x 256^3 = 150,994,944 per step.

Prints one JSON line.  Inputs are resident in HBM before timing starts.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
                    [--calibrate-copy]   (adds a plain 1 GiB device copy,
                                          the HBM-counter scale reference)
    python bench.py --variants [--steps K]
        one JSON line with the cost of the same RK3 step for every scheme
        (TENO6, TENO8, TENO8A) and limiter, relative to classic TENO of the
        same scheme, in the manner of the paper's Table 2
    python bench.py --adjoint [--adj-steps 200] [--fd-directions 16]
        one JSON line for the adjoint: 2D Euler 1024^2 periodic (density
        modes + circular jump, at rest), TENO6-M-MP, 200 fixed steps, loss =
        L2 density misfit against a target run; forward, checkpointed
        forward + backward (checkpoint every 20 steps), and central
        differences of the loss along random directions
    python bench.py --batched [--batch-steps 100] [--per-problem-steps 3]
        one JSON line for the batched path: 4096 independent 1D Euler
        Riemann problems, n log-uniform in [256, 16384] (15.9 M cells),
        TENO8-M-MP, C_T = 1e-7, CFL 0.4 with each problem's own step, 100
        SSP-RK3 steps as one replay of a captured graph after the tile
        autotuner, against one launch per problem
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402  (seeded inputs; no scheme arithmetic)
from paper_2010_13289_amd import opcount as O  # noqa: E402  (itemised operation counts)

METRIC = "face-reconstructions/s + % HBM roofline (fwd, fwd+adjoint, batched vs plain)"
N = 256
GAMMA = 1.4
C_T = 1e-5
SCHEME = 6
CFL = W.CFL

# MI355X published peaks
PEAK_FP64_TFLOPS = 78.6     # 256 CU x 4 SIMD x 16 FP64 lanes x 2 (FMA) x 2.4 GHz
PEAK_HBM_GBS = 8000.0

# Algorithmic FP64 operations per face vector, itemised in
# paper_2010_13289_amd/opcount.py (FMA = 2, every other arithmetic, min/max,
# compare, division or square root = 1) and pinned by tests/test_opcount.py:
# with every candidate limited (the bound on the method's work) here; the
# roofline fractions count the limiter where the timed state needs it
# (limiter_shares).
FLOPS_PER_FACE_VECTOR = O.face_vector_ops("euler", 3, SCHEME, O.LIM_MP)
# Algorithmic HBM bytes per cell and step: U^(s) read and U^(s+1) written in
# every stage, U^n also read in stages 2 and 3 (5 fields x 8 bytes each).
BYTES_PER_CELL_STEP = O.rk3_bytes_per_cell(5)

# HBM bytes per launch of each sweep kind at 256^3, averaged over the three
# stages, from two rocprofv3 --pmc runs of this benchmark (FETCH_SIZE scaled
# by 2.0 and WRITE_SIZE by 1.0, the factors a plain 1 GiB device copy reads
# as).  They describe the kernels built from the sources whose digest is
# TRAFFIC_SOURCE_DIGEST and are reported as null for any other build.
TRAFFIC_SOURCE_DIGEST = "1af54b998de4687b11c56218fb72441ef32ccbc249d679660a48fd7e8136fe72"
MEASURED_TRAFFIC = {"sweep_x": 1.4719e+09, "sweep_y": 2.0330e+09, "sweep_z": 2.5889e+09}
# batched sweep, 4096 problems, averaged over the stages, per tile shape
# (64x1, 128x1, 128x2, 256x1, 256x2, 512x1): smaller tiles re-read more halo
MEASURED_TRAFFIC_BATCH = (1.2754e9, 1.1488e9, 1.0866e9, 1.0863e9, 1.0554e9, 1.0551e9)
TRAFFIC_NOTE = ("recorded, not measured in this run: rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE of this benchmark "
                "on the kernel sources whose digest is TRAFFIC_SOURCE_DIGEST (null for any other build); "
                "see the profiles directory")


# sources of the adjoint only: the forward and batched sweeps whose traffic
# is recorded above do not include them
ADJOINT_ONLY_SOURCES = ("teno_adjoint.h", "tenom_vjp_inst.hip", "vjp_dispatch.h")


def kernel_source_digest() -> str:
    """sha256 over the sources of the forward and batched kernels (csrc/*.h,
    *.hip, the table generator; not the generated tables, not the adjoint)."""
    import hashlib
    d = os.path.join(ROOT, "paper_2010_13289_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        if name.endswith((".h", ".hip", ".py")) and name != "teno_tables.h" and name not in ADJOINT_ONLY_SOURCES:
            h.update(name.encode())
            with open(os.path.join(d, name), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def limiter_shares(T, U, grid, scheme, limiter, ct):
    """Per axis, (rough, nonsmooth) of the reconstructions of state U
    (opcount.limiter_share) from the smoothness flags of the library's
    reconstruct_faces (untimed; the flags are the kernels' own decisions)."""
    nk = (scheme & 0xFF) - 2
    shares = []
    for ax in range(grid["ndim"]):
        _, fl = T.reconstruct_faces(U, grid, scheme, limiter, ct, GAMMA, ax, return_flags=True)
        shares.append(O.limiter_share(fl, nk))
        del fl
    return shares


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=N)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--variants", action="store_true")
    ap.add_argument("--batched", action="store_true")
    ap.add_argument("--adjoint", action="store_true")
    ap.add_argument("--adj-steps", type=int, default=200)
    ap.add_argument("--adj-n", type=int, default=1024)
    ap.add_argument("--fd-directions", type=int, default=16)
    ap.add_argument("--batch-steps", type=int, default=100)
    ap.add_argument("--per-problem-steps", type=int, default=3)
    return ap.parse_args()


# Algorithmic FP64 operations per 1D Euler face vector, K = 8, MP limiter
# (the batched sweep), and per 2D face vector of the adjoint's VJP, K = 6, MP.
FLOPS_PER_FACE_VECTOR_1D_K8 = O.face_vector_ops("euler", 1, 8, O.LIM_MP)
FLOPS_PER_VJP_FACE_VECTOR_2D_K6 = O.adjoint_face_vector_ops(2, 6, O.LIM_MP)


def run_adjoint(args):
    """The adjoint workload; returns the JSON object.

    Timing: TENO6-M-MP (C_T = 1e-5) on the configured state.  The fluid is
    at rest at uniform pressure, so its acoustic characteristic fields carry
    only rounding-level signals whose cutoff decisions are set by rounding:
    the loss is not differentiable at any scale differences can resolve.
    Two difference checks stand beside the timing:
      * the same grid, state, steps and checkpointing with C_T = 0 (every
        candidate smooth, no decision), where the rollout is smooth;
      * the scheme as configured (C_T = 1e-5, MP) on the same grid with the
        state set in motion (small seeded velocity and pressure
        perturbations), over 24 steps with a checkpoint every 20: a
        direction counts where the perturbed rollouts take every smoothness
        decision of the unperturbed one and the differences at two step
        sizes agree."""
    import numpy as np
    import torch

    import paper_2010_13289_amd as T
    n, steps, ck = args.adj_n, args.adj_steps, 20
    U0h, dx = W.density_modes_2d(n, seed=5)
    T0h, _ = W.density_modes_2d(n, seed=6)
    grid = dict(ndim=2, n=[n, n], dx=[dx, dx], bc=[0, 0], system=1)
    scheme, lim = 6, T.LIM_MP
    U0 = torch.from_numpy(U0h).to("cuda")
    dt = CFL / T.max_wave_speed(U0, grid, GAMMA)
    ws = T.Workspace(grid, scheme, U0.device)

    def forward(U, ct):
        V = U.clone()
        for _ in range(steps):
            T.rk3_step(V, grid, scheme, lim, ct, GAMMA, dt, workspace=ws)
        return V

    def loss_fn(ct):
        rho_T = forward(torch.from_numpy(T0h).to("cuda"), ct)[0].clone()
        return lambda Uf: 0.5 * ((Uf[0] - rho_T) ** 2).sum() * dx * dx

    def grad(ct, loss_of):
        U = U0.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L = loss_of(T.rollout(U, grid, scheme, lim, ct, GAMMA, dt, steps, checkpoint=ck))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        T.profile_read()
        T.profile_enable(True)
        L.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        T.profile_enable(False)
        return U.grad.detach(), float(L.item()), t1 - t0, t2 - t1, T.profile_read()

    # timing on the configured scheme
    ct = 1e-5
    loss_mp = loss_fn(ct)
    U_end = forward(U0, ct)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    forward(U0, ct)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    grad(ct, loss_mp)  # warm-up: workspaces allocated, kernels loaded
    g_mp, L_mp, t_fwd_ck, t_bwd, prof = grad(ct, loss_mp)
    # difference check with C_T = 0
    loss0 = loss_fn(0.0)
    g0, L0, _, _, _ = grad(0.0, loss0)
    rng = np.random.default_rng(2010)
    scale = np.maximum(np.abs(U0h).max(axis=(1, 2)), 1.0)[:, None, None]
    rows = []
    with torch.no_grad():
        for d in range(args.fd_directions):
            V = torch.from_numpy(rng.standard_normal(U0h.shape) * scale).to("cuda")
            fd = []
            for h in (1e-5, 1e-6):
                lp = loss0(forward(U0 + h * V, 0.0)).item()
                lm = loss0(forward(U0 - h * V, 0.0)).item()
                fd.append((lp - lm) / (2 * h))
            ad = float((g0 * V).sum().item())
            rows.append({"fd_h1e-5": fd[0], "fd_h1e-6": fd[1], "adjoint": ad,
                         "rel_err": abs(fd[1] - ad) / max(abs(ad), 1e-300)})
    cutoff_check = fd_check_cutoff(T, n, args.fd_directions)
    vjp_n, vjp_ms = prof["vjp_axis"]
    faces = 2 * n * n
    vjp_avg_s = vjp_ms / 1e3 / max(vjp_n, 1)
    # the limiter counted where the states need it, averaged over the two
    # axes, on the rollout's last state: the fluid is at rest, and from the
    # first step on the decisions of its acoustic and shear fields follow
    # rounding noise (about half of their reconstructions have a nonsmooth
    # candidate, against 0.1 % on the initial state)
    shares = limiter_shares(T, U_end, grid, scheme, lim, ct)
    del U_end
    rough = sum(r for r, _ in shares) / len(shares)
    nonsm = sum(c for _, c in shares) / len(shares)
    vjp_flops = O.adjoint_face_vector_ops(2, 6, O.LIM_MP, rough=rough, nonsmooth=nonsm) * n * n  # n^2 faces per axis
    return {
        "metric": METRIC,
        "value": 3 * steps * faces / t_bwd,
        "unit": "face adjoints/s (backward pass, recomputation included)",
        "n_gpus": 1,
        "steps": steps,
        "warmup": 1,
        "ms_per_step": t_bwd / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"2D Euler {n}^2 periodic: density 1 + 64 seeded Fourier modes (|k| <= 32, amplitude "
                        "0.05), x0.5 inside a circle of radius 0.2, u = v = 0, p = 1; TENO6-M-MP, C_T=1e-5, "
                        f"gamma=1.4, {steps} SSP-RK3 steps of fixed dt (CFL 0.4 at t=0); loss = L2 density "
                        "misfit against the run from seed 6; adjoint checkpointed every 20 steps",
            "grid": [n, n],
        },
        "forward_s": t_fwd,
        "forward_with_checkpoints_s": t_fwd_ck,
        "backward_s": t_bwd,
        "backward_over_forward": t_bwd / t_fwd,
        "vjp_axis_avg_ms": vjp_avg_s * 1e3,
        "vjp_axis_launches": vjp_n,
        "roofline": {"bound": "alu", "kernel": "vjp_axis", "achieved": vjp_flops / vjp_avg_s / 1e12,
                     "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": vjp_flops / vjp_avg_s / 1e12 / PEAK_FP64_TFLOPS, "traffic": None,
                     "avg_launch_ms": vjp_avg_s * 1e3, "flops_per_launch": vjp_flops,
                     "flops_per_launch_every_candidate_limited": FLOPS_PER_VJP_FACE_VECTOR_2D_K6 * n * n},
        "limiter_share": {ax: {"reconstructions_with_a_nonsmooth_candidate": r,
                               "nonsmooth_candidates_per_reconstruction": c} for ax, (r, c) in zip("xy", shares)},
        "loss": L_mp,
        "mp_gradient_max_per_field": g_mp.abs().amax(dim=(1, 2)).cpu().tolist(),
        "fd_check_ct0": {"directions": len(rows), "loss": L0,
                         "max_rel_err": max(r["rel_err"] for r in rows) if rows else None, "rows": rows},
        "fd_check_cutoff": cutoff_check,
    }


def fd_check_cutoff(T, n, want, steps=24, ck=20, max_tries=32, h=1e-8):
    """Central differences of the TENO6-M-MP (C_T = 1e-5) rollout gradient on
    the moving 2D state along smooth local directions (random-phase fields
    under a Gaussian window of width 1/64).  Every direction tried is
    reported; a direction is "strict" where the rollouts from U +- hV take
    every smoothness decision of the unperturbed one and the differences at
    h and h/2 agree to 1e-6 (rounding in the differences resolves 1e-6).  The difference is taken on the final states:
    L(U+) - L(U-) = sum (rho+ - rho-)(rho+ + rho- - 2 rho_T) dx^2 / 2."""
    import numpy as np
    import torch
    ct = 1e-5
    U0h, dx = W.moving_density_modes_2d(n, seed=5)
    Th, _ = W.moving_density_modes_2d(n, seed=6)
    grid = dict(ndim=2, n=[n, n], dx=[dx, dx], bc=[0, 0], system=1)
    U0 = torch.from_numpy(U0h).to("cuda")
    dt = CFL / T.max_wave_speed(U0, grid, GAMMA)

    def final_rho(V):
        return T.rollout(V, grid, 6, T.LIM_MP, ct, GAMMA, dt, steps, checkpoint=steps)[0]

    target = final_rho(torch.from_numpy(Th).to("cuda")).detach().clone()
    U = U0.clone().requires_grad_(True)
    Uf = T.rollout(U, grid, 6, T.LIM_MP, ct, GAMMA, dt, steps, checkpoint=ck)
    (0.5 * ((Uf[0] - target) ** 2).sum() * dx * dx).backward()
    g = U.grad.detach()

    def central(V, hh):
        with torch.no_grad():
            rp, rm = final_rho(U0 + hh * V), final_rho(U0 - hh * V)
            return float((0.5 * (rp - rm) * (rp + rm - 2.0 * target)).sum().item()) * dx * dx / (2.0 * hh)

    ref = T.rollout_flags(U0, grid, 6, T.LIM_MP, ct, GAMMA, dt, steps)
    scale = torch.from_numpy(np.abs(U0h).max(axis=(1, 2), keepdims=True)).to("cuda")
    rows, strict = [], 0
    for d in range(max_tries):
        if strict >= want:
            break
        V = torch.from_numpy(W.local_direction_2d(U0h.shape, seed=d, width=1.0 / 64.0)).to("cuda") * scale
        same = (T.rollout_flags(U0 + h * V, grid, 6, T.LIM_MP, ct, GAMMA, dt, steps, ref=ref)
                and T.rollout_flags(U0 - h * V, grid, 6, T.LIM_MP, ct, GAMMA, dt, steps, ref=ref))
        fd, fd2 = central(V, h), central(V, h / 2)
        ad = float((g * V).sum().item())
        ok = same and abs(fd - fd2) <= 1e-6 * abs(fd)
        strict += ok
        rows.append({"fd": fd, "fd_half_h": fd2, "adjoint": ad, "same_decisions": bool(same), "strict": bool(ok),
                     "rel_err": abs(fd - ad) / max(abs(ad), 1e-300)})
    del ref
    errs = [r["rel_err"] for r in rows]
    serrs = [r["rel_err"] for r in rows if r["strict"]]
    return {"scheme": "TENO6-M-MP", "C_T": ct, "steps": steps, "checkpoint": ck, "h": h,
            "state": f"{n}^2 moving density modes (W.moving_density_modes_2d, seed 5; target seed 6)",
            "directions": "W.local_direction_2d(seed=d, width=1/64) times each field's max |U|",
            "directions_tried": len(rows), "directions_strict": strict,
            "max_rel_err_strict": max(serrs) if serrs else None,
            "directions_within_1e-6": sum(e <= 1e-6 for e in errs),
            "max_rel_err_all": max(errs) if errs else None, "median_rel_err_all": float(np.median(errs)),
            "gradient_max_per_field": g.abs().amax(dim=(1, 2)).cpu().tolist(), "rows": rows}


def run_batched(args):
    """The batched workload; returns the JSON object."""
    import numpy as np
    import torch

    import paper_2010_13289_amd as T
    sizes = W.batched_riemann_sizes()
    parts, dx = [], []
    for p, n in enumerate(sizes):
        left, right = W.riemann_states(p)
        Up, h = W.riemann_problem(int(n), left, right, gamma=GAMMA)
        parts.append(Up)
        dx.append(h)
    U_host = np.concatenate(parts, axis=1)
    plan = T.BatchPlan(sizes, dx, T.BC_TRANSMISSIVE)
    U0 = torch.from_numpy(U_host).to("cuda")
    U = U0.clone()
    scheme, lim, ct = 8, T.LIM_MP, 1e-7
    # limiter share of the initial state's reconstructions, from the flags of
    # the problems laid end to end as one transmissive line (untimed; the
    # 4,095 faces where two problems meet are 0.03 % of the faces)
    line = dict(ndim=1, n=[int(U_host.shape[1])], dx=[float(np.mean(dx))], bc=[T.BC_TRANSMISSIVE], system=1)
    (rough, nonsm), = limiter_shares(T, U0, line, scheme, lim, ct)
    best, tile_ms = plan.autotune(U, scheme, lim, ct, GAMMA, CFL, steps=2)
    steps = args.batch_steps
    faces_per_stage = plan.total + plan.count  # n + 1 faces per problem
    faces = 3 * steps * faces_per_stage
    # capture and one untimed replay, then the timed replay from the same state
    plan.rk3_graph(U, scheme, lim, ct, GAMMA, CFL, steps=steps)
    torch.cuda.synchronize()
    U.copy_(U0)
    plan.reset_times()
    torch.cuda.synchronize()
    T.profile_read()
    T.profile_enable(True)
    t0 = time.perf_counter()
    plan.rk3_graph(U, scheme, lim, ct, GAMMA, CFL, steps=steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    T.profile_enable(False)
    graph_ms = T.profile_read()["batch_graph"][1]
    ok = bool(torch.isfinite(U).all().item())
    U_graph = U.clone()
    # the same steps as one persistent kernel launch (untimed warm-up of one
    # step, then the timed launch from the same state); the same bits
    plan.rk3_persistent(U, scheme, lim, ct, GAMMA, CFL, steps=1)
    U.copy_(U0)
    plan.reset_times()
    torch.cuda.synchronize()
    T.profile_enable(True)
    plan.rk3_persistent(U, scheme, lim, ct, GAMMA, CFL, steps=steps)
    torch.cuda.synchronize()
    T.profile_enable(False)
    persist_ms = T.profile_read()["batch_persist"][1]
    persist_same = bool(torch.equal(U, U_graph))
    del U_graph
    # per-kernel averages from eager steps (kernels inside a graph are not
    # bracketed one by one)
    U.copy_(U0)
    torch.cuda.synchronize()
    T.profile_enable(True)
    plan.rk3(U, scheme, lim, ct, GAMMA, CFL, steps=5)
    torch.cuda.synchronize()
    T.profile_enable(False)
    prof = T.profile_read()
    sweep_n, sweep_ms = prof["batch_sweep"]
    dt_n, dt_ms = prof["batch_dt"]
    avg_s = sweep_ms / 1e3 / max(sweep_n, 1)
    flops_launch = O.face_vector_ops("euler", 1, 8, O.LIM_MP, rough=rough, nonsmooth=nonsm) * faces_per_stage
    achieved = flops_launch / avg_s / 1e12
    sec_per_step = graph_ms / 1e3 / steps
    # one launch per problem: the same kernels with first = p, count = 1
    pp = args.per_problem_steps
    per_problem = None
    if pp > 0:
        U.copy_(U0)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        p0 = time.perf_counter()
        e0.record()
        for p in range(plan.count):
            plan.rk3(U, scheme, lim, ct, GAMMA, CFL, steps=pp, first=p, count=1)
        e1.record()
        torch.cuda.synchronize()
        p1 = time.perf_counter()
        pp_wall = (p1 - p0) / pp
        per_problem = {
            "launches_per_step": 4 * plan.count,
            "ms_per_step_wall": pp_wall * 1e3,
            "ms_per_step_gpu": e0.elapsed_time(e1) / pp,
            "steps_timed": pp,
            "face_reconstructions_per_s": 3 * faces_per_stage / pp_wall,
            "batched_speedup": pp_wall / sec_per_step,
            "graph": per_problem_graph(plan, U, U0, scheme, lim, ct, pp, sec_per_step, faces_per_stage),
        }
    value = faces / (graph_ms / 1e3)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "face-reconstructions/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": 1,
        "ms_per_step": sec_per_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "batched 1D Euler: 4096 seeded Riemann problems, n log-uniform in [256, 16384], "
                        "TENO8-M-MP, C_T=1e-7, gamma=1.4, CFL 0.4 per problem, 100 SSP-RK3 steps in one "
                        "replay of a captured HIP graph",
            "problems": plan.count,
            "cells": plan.total,
            "face_vectors_per_step": 3 * faces_per_stage,
            "tile": {"id": best, "threads": T.batch_tile_shape(best)[0],
                     "faces_per_thread": T.batch_tile_shape(best)[1]},
            "autotune_ms_per_step": tile_ms,
        },
        "roofline": {
            "bound": "alu",
            "kernel": "batch_sweep",
            "achieved": achieved,
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_TFLOPS,
            "traffic": (MEASURED_TRAFFIC_BATCH[best] if kernel_source_digest() == TRAFFIC_SOURCE_DIGEST
                        else None),
            "traffic_source": TRAFFIC_NOTE,
            "avg_launch_ms": avg_s * 1e3,
            "flops_per_launch": flops_launch,
            "flops_per_launch_every_candidate_limited": FLOPS_PER_FACE_VECTOR_1D_K8 * faces_per_stage,
            "limiter_share": {"reconstructions_with_a_nonsmooth_candidate": rough,
                              "nonsmooth_candidates_per_reconstruction": nonsm},
        },
        "graph_wall_ms": (t1 - t0) * 1e3,
        "persistent": {"ms_per_step": persist_ms / steps, "launches": 1,
                       "face_reconstructions_per_s": faces / (persist_ms / 1e3),
                       "same_bits_as_graph": persist_same,
                       "note": "all steps of all problems in one kernel launch (tenom_batch_rk3_persistent)"},
        "step_size_kernel_avg_ms": dt_ms / max(dt_n, 1),
        "per_problem_launches": per_problem,
        "state_finite": ok,
    }
    plan.close()
    return out


def per_problem_graph(plan, U, U0, scheme, lim, ct, reps, sec_per_step, faces_per_stage):
    """One step of the per-problem launches (4 kernels for each problem)
    captured in one HIP graph and replayed `reps` times: the per-problem
    kernels' own cost without host launch overhead."""
    import torch
    U.copy_(U0)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up off the capture, as torch asks
        plan.rk3(U, scheme, lim, ct, GAMMA, CFL, steps=1, first=0, count=1)
    torch.cuda.current_stream().wait_stream(side)
    U.copy_(U0)
    torch.cuda.synchronize()
    with torch.cuda.graph(graph):
        for p in range(plan.count):
            plan.rk3(U, scheme, lim, ct, GAMMA, CFL, steps=1, first=p, count=1)
    graph.replay()  # untimed
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del graph
    return {"nodes_per_step": 4 * plan.count, "ms_per_step": ms,
            "face_reconstructions_per_s": 3 * faces_per_stage / (ms / 1e3),
            "batched_speedup": ms / 1e3 / sec_per_step}


# (name, scheme, limiter, C_T) of the variant report; classic TENO first in
# each group, the reference of the ratios.  The adaptive scheme ignores C_T.
VARIANTS = [
    ("TENO6", 6, 0, 1e-5), ("TENO6-M-MP", 6, 1, 1e-5), ("TENO6-M-TVD5", 6, 3, 1e-5),
    ("TENO6-M-VA", 6, 4, 1e-5), ("TENO6-M-TVD(minmod)", 6, 2, 1e-5), ("TENO6-M-MP(M4,b2)", 6, 5, 1e-5),
    ("TENO6-M-MP(MM,b4)", 6, 6, 1e-5), ("TENO6-M-MP(MM,b2)", 6, 7, 1e-5), ("TENO6-M-MP(MM,b1)", 6, 8, 1e-5),
    ("TENO8", 8, 0, 1e-7), ("TENO8-M-MP", 8, 1, 1e-7), ("TENO8-M-TVD5", 8, 3, 1e-7), ("TENO8-M-VA", 8, 4, 1e-7),
    ("TENO8A", 8 | 0x100, 0, 0.0), ("TENO8A-M-MP", 8 | 0x100, 1, 0.0), ("TENO8A-M-TVD5", 8 | 0x100, 3, 0.0),
    ("TENO8A-M-VA", 8 | 0x100, 4, 0.0),
]


def run_variants(T, U0, grid, n, steps, warmup):
    """Time one RK3 step of every variant from the same initial state."""
    import torch
    rows = []
    ref = {}
    for name, scheme, lim, ct in VARIANTS:
        U = U0.clone()
        ws = T.Workspace(grid, scheme, U.device)
        shares = limiter_shares(T, U, grid, scheme, lim, ct)

        def step():
            T.rk3_step_cfl(U, grid, scheme, lim, ct, GAMMA, CFL, workspace=ws)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        T.profile_read()
        T.profile_enable(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        T.profile_enable(False)
        prof = T.profile_read()
        ms = (t1 - t0) / steps * 1e3
        group = name.split("-")[0]
        ref.setdefault(group, ms)
        sweep_ms = {k: prof[k][1] / max(prof[k][0], 1) for k in ("sweep_x", "sweep_y", "sweep_z")}
        kind = max(sweep_ms, key=sweep_ms.get)  # the slowest sweep of the variant
        rough, nonsm = shares["xyz".index(kind[-1])]
        flops_launch = O.face_vector_ops("euler", 3, scheme & 0xFF, lim, bool(scheme & 0x100),
                                         rough=rough, nonsmooth=nonsm) * n ** 3
        achieved = flops_launch / (sweep_ms[kind] / 1e3) / 1e12
        rows.append({
            "variant": name, "scheme": scheme, "limiter": lim, "C_T": ct, "ms_per_step": ms,
            "face_vectors_per_s": 9 * n ** 3 / (ms / 1e3),
            "ratio_vs_classic": ms / ref[group],
            "sweep_avg_ms": sweep_ms,
            "roofline": {"bound": "alu", "kernel": kind, "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                         "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS, "flops_per_launch": flops_launch},
            "limiter_share": {ax: {"reconstructions_with_a_nonsmooth_candidate": r,
                                   "nonsmooth_candidates_per_reconstruction": c} for ax, (r, c) in zip("xyz", shares)},
            "state_finite": T.check_finite(U, grid),
        })
        print(f"# {name}: {ms:.3f} ms/step, {kind} {sweep_ms[kind]:.3f} ms, frac {achieved / PEAK_FP64_TFLOPS:.3f}",
              file=sys.stderr, flush=True)
        del ws, U
    return rows


def cpu_baseline(U, grid, seconds):
    """The oracle as it stands, on a bounded random sample of faces of the
    same state (all three axes), using the host's OpenMP threads."""
    import numpy as np

    import oracle
    rng = np.random.default_rng(7)
    nfaces = (grid["n"][0] + 1) * grid["n"][1] * grid["n"][2]

    def run(m):
        t0 = time.perf_counter()
        for ax in range(3):
            idx = rng.integers(0, nfaces, size=m)
            oracle.faces_points(U, grid, SCHEME, 1, C_T, GAMMA, ax, idx)
        return time.perf_counter() - t0

    m = 256
    t = run(m)
    while t < 0.5:
        m *= 4
        t = run(m)
    m = max(m, int(m * seconds / max(t, 1e-3)))
    t = run(m)
    cores = oracle.num_threads()
    # the same oracle on one thread, on a sample cut to about 5 s
    m1 = max(256, int(m * 5.0 / (t * cores)))
    oracle.set_num_threads(1)
    try:
        t1 = run(m1)
    finally:
        oracle.set_num_threads(cores)
    return {"value": 3 * m / t, "unit": "face-reconstructions/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{3 * m} random faces ({m} per axis) of the same {grid['n'][0]}^3 state, "
                      f"TENO6-M-MP, {t:.1f} s",
            "value_1core": 3 * m1 / t1,
            "sample_1core": f"{3 * m1} random faces, one thread, {t1:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU decomposition is not built", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2010_13289_amd as T

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    if args.batched:
        print(json.dumps(run_batched(args)), flush=True)
        return
    if args.adjoint:
        print(json.dumps(run_adjoint(args)), flush=True)
        return
    n = args.n
    U_host, dx = W.tgv_3d(n, gamma=GAMMA)
    grid = dict(ndim=3, n=[n, n, n], dx=[dx] * 3, bc=[0, 0, 0], system=1)
    U0 = torch.from_numpy(U_host).to(dev)
    if args.variants:
        rows = run_variants(T, U0, grid, n, args.steps, args.warmup)
        print(json.dumps({
            "report": "variants", "unit": "ms per SSP-RK3 step", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"3D Euler {n}^3 periodic TGV + density jump + seeded perturbations, "
                                   "gamma=1.4, CFL 0.4, one SSP-RK3 step per variant from the same state",
                       "grid": [n, n, n]},
            "rows": rows,
        }), flush=True)
        return
    U = U0.clone()
    ws = T.Workspace(grid, SCHEME, dev)

    # limiter share of the initial state's reconstructions, per axis (untimed)
    shares = limiter_shares(T, U, grid, SCHEME, T.LIM_MP, C_T)
    torch.cuda.synchronize()

    if args.calibrate_copy:
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    def step():
        # dt = CFL / (largest signal rate of U), taken on the device
        T.rk3_step_cfl(U, grid, SCHEME, T.LIM_MP, C_T, GAMMA, CFL, workspace=ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    T.profile_read()  # discard
    T.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    T.profile_enable(False)
    prof = T.profile_read()
    ok = T.check_finite(U, grid)

    cells = n ** 3
    faces_per_step = 3 * 3 * cells
    sec_per_step = (t1 - t0) / args.steps
    value = faces_per_step / sec_per_step

    # dominant kernel: the sweep kind with the largest summed time
    kind = max(("sweep_x", "sweep_y", "sweep_z"), key=lambda k: prof[k][1])
    launches, ms = prof[kind]
    avg_s = ms / 1e3 / max(launches, 1)
    rough, nonsm = shares["xyz".index(kind[-1])]
    flops_launch = O.face_vector_ops("euler", 3, SCHEME, O.LIM_MP, rough=rough, nonsmooth=nonsm) * cells
    achieved = flops_launch / avg_s / 1e12
    sweeps_ms = {k: (prof[k][1] / max(prof[k][0], 1)) for k in ("sweep_x", "sweep_y", "sweep_z")}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "face-reconstructions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec_per_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"3D Euler {n}^3 periodic TGV + density jump + seeded perturbations, "
                        "TENO6-M-MP, C_T=1e-5, gamma=1.4, CFL 0.4 (dt on the device), one SSP-RK3 step",
            "grid": [n, n, n],
            "scheme": "TENO6-M-MP",
            "face_vectors_per_step": faces_per_step,
        },
        "roofline": {
            "bound": "alu",
            "kernel": kind,
            "achieved": achieved,
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_TFLOPS,
            "traffic": (MEASURED_TRAFFIC.get(kind) if n == N and kernel_source_digest() == TRAFFIC_SOURCE_DIGEST
                        else None),
            "traffic_source": TRAFFIC_NOTE,
            "avg_launch_ms": avg_s * 1e3,
            "flops_per_launch": flops_launch,
            "flops_per_launch_every_candidate_limited": FLOPS_PER_FACE_VECTOR * cells,
            "frac_every_candidate_limited": FLOPS_PER_FACE_VECTOR * cells / avg_s / 1e12 / PEAK_FP64_TFLOPS,
        },
        "limiter_share": {ax: {"reconstructions_with_a_nonsmooth_candidate": r, "nonsmooth_candidates_per_reconstruction": c}
                          for ax, (r, c) in zip("xyz", shares)},
        "scalar_reconstructions_per_s": 10 * value,
        "sweep_avg_ms": sweeps_ms,
        "hbm_alg_frac": (BYTES_PER_CELL_STEP * cells / sec_per_step / 1e9) / PEAK_HBM_GBS,
        "nonsmooth_flag_fraction": sum(c for _, c in shares) / (4 * len(shares)),
        "state_finite": ok,
        "kernel_source_digest": kernel_source_digest(),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(U_host, grid, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
