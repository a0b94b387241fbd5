"""Throughput benchmark of the TENO-M path on one MI355X.

One step = one SSP-RK3 step of the 3D Euler equations on a 256^3 periodic
cube (the Taylor-Green velocity and pressure of Sec. 4.3.1, a planar
density jump 1 -> 0.125 at x = pi, seeded random-phase velocity
perturbations), six-point TENO-M with the MP limiter, C_T = 1e-5,
gamma = 1.4, CFL 0.4: the wave-speed reduction for dt, then 3 stages x
(x, y, z) sweeps of face reconstructions, divergence and stage update.
Unit: one face vector (the full 5-component flux at one face, both split
sides), 3 stages x 3 axes x 256^3 = 150,994,944 per step.

Prints one JSON line.  Inputs are resident in HBM before timing starts.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
                    [--calibrate-copy]   (adds a plain 1 GiB device copy,
                                          the HBM-counter scale reference)
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

METRIC = "face-reconstructions/s + % HBM roofline (fwd, fwd+adjoint, batched vs plain)"
N = 256
GAMMA = 1.4
C_T = 1e-5
SCHEME = 6
CFL = 0.4

# MI355X published peaks
PEAK_FP64_TFLOPS = 78.6     # 256 CU x 4 SIMD x 16 FP64 lanes x 2 (FMA) x 2.4 GHz
PEAK_HBM_GBS = 8000.0

# Algorithmic FP64 operations per Euler face vector (3D, K = 6, MP limiter),
# FMA counted as 2, every other arithmetic, min/max or compare as 1, a
# division or square root as 1.  Breakdown (per face vector):
#   cell primitives and physical flux, once per cell     22
#   Rusanov alpha (max over 6 cells)                       5
#   Roe average and eigenvector constants                 38
#   projection of 6 U and 6 F vectors on L               264
#   Rusanov split of 5 fields x 6 cells                  150
#   TENO-M, 10 scalar reconstructions x 193            1930
#   back-projection with R                                20
#   divergence and stage update, once per cell            20
FLOPS_PER_FACE_VECTOR = 2449
# Algorithmic HBM bytes per cell and step: U^(s) read and U^(s+1) written in
# every stage, U^n also read in stages 2 and 3 (5 fields x 8 bytes each).
BYTES_PER_CELL_STEP = 320

# HBM bytes per launch of each sweep kind at 256^3, averaged over the three
# stages, from two rocprofv3 --pmc runs of this benchmark (FETCH_SIZE scaled
# by 2.0 and WRITE_SIZE by 1.0, the factors a plain 1 GiB device copy reads
# as).  They describe the kernels built from the sources whose digest is
# TRAFFIC_SOURCE_DIGEST and are reported as null for any other build.
TRAFFIC_SOURCE_DIGEST = "dac703a37bf04cb3cea84ee29149123ff9da5a6314c1926f65f68df941227ea7"
MEASURED_TRAFFIC = {"sweep_x": 1.3425e9, "sweep_y": 2.0765e9, "sweep_z": 2.5239e9}


def kernel_source_digest() -> str:
    """sha256 over the kernel sources (csrc/*.h, *.hip, the table generator)."""
    import hashlib
    d = os.path.join(ROOT, "paper_2010_13289_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        if name.endswith((".h", ".hip", ".py")) and name != "teno_tables.h":
            h.update(name.encode())
            with open(os.path.join(d, name), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=N)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--calibrate-copy", action="store_true")
    return ap.parse_args()


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
    return {"value": 3 * m / t, "unit": "face-reconstructions/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{3 * m} random faces ({m} per axis) of the same {grid['n'][0]}^3 state, "
                      f"TENO6-M-MP, {t:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU decomposition is not built", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2010_13289_amd as T
    import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    n = args.n
    U_host, dx = W.tgv_3d(n, gamma=GAMMA)
    grid = dict(ndim=3, n=[n, n, n], dx=[dx] * 3, bc=[0, 0, 0], system=1)
    U0 = torch.from_numpy(U_host).to(dev)
    U = U0.clone()
    ws = T.Workspace(grid, SCHEME, dev)

    # fraction of nonsmooth candidate flags on the initial state (untimed)
    nonsmooth = 0
    total = 0
    for ax in range(3):
        _, fl = T.reconstruct_faces(U, grid, SCHEME, T.LIM_MP, C_T, GAMMA, ax, return_flags=True)
        bits = fl.to(torch.int32)
        ones = sum(((bits >> k) & 1).sum().item() for k in range(4))
        nonsmooth += fl.numel() * 4 - ones
        total += fl.numel() * 4
        del fl, bits
    torch.cuda.synchronize()

    if args.calibrate_copy:
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    def step():
        rate = T.max_wave_speed(U, grid, GAMMA)
        T.rk3_step(U, grid, SCHEME, T.LIM_MP, C_T, GAMMA, CFL / rate, workspace=ws)

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
    flops_launch = FLOPS_PER_FACE_VECTOR * cells
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
                        "TENO6-M-MP, C_T=1e-5, gamma=1.4, CFL 0.4, one SSP-RK3 step",
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
            "avg_launch_ms": avg_s * 1e3,
            "flops_per_launch": flops_launch,
        },
        "scalar_reconstructions_per_s": 10 * value,
        "sweep_avg_ms": sweeps_ms,
        "hbm_alg_frac": (BYTES_PER_CELL_STEP * cells / sec_per_step / 1e9) / PEAK_HBM_GBS,
        "nonsmooth_flag_fraction": nonsmooth / total,
        "state_finite": ok,
        "kernel_source_digest": kernel_source_digest(),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(U_host, grid, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
