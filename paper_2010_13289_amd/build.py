"""Build libtenom.so (HIP, gfx950) in-tree.

Steps: regenerate csrc/teno_tables.h from gen_tables.py, compile the eight
forward, the eight tile-sweep and the eight adjoint instantiation units
(fields x K), the six batched-path units (one per tile shape), the persistent
batched unit and the three C-ABI sources in parallel with hipcc, link them into
paper_2010_13289_amd/libtenom.so.

    python -m paper_2010_13289_amd.build [--verbose]
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libtenom.so")
ARCH = os.environ.get("TENOM_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-result",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no implicit contraction: every fused multiply-add is written in the
    # source, so each kernel instantiation (and each batched tile shape)
    # rounds the same way and gives the same bits
    "-ffp-contract=off",
]

# the tile sweeps: no machine-level loop-invariant code motion (the face's
# constants hoisted out of the chunk loop spill into vector-register lanes)
TILE_FLAGS = ["-DTENOM_TILE_UNIT", "-mllvm", "-disable-machine-licm"]

# the adjoint units: instructions scheduled to keep memory clauses together
# (the tile adjoint measured 1-2 % faster, the same bits; the forward sweeps
# measured slower and keep the default)
VJP_FLAGS = ["-mllvm", "-amdgpu-sched-strategy=max-memory-clause"]

UNITS = [(nf, k) for nf in (1, 3, 4, 5) for k in (6, 8)]
BATCH_TILES = 6  # tile shapes of the batched path (kTiles in teno_batch.h)


def _hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cand = os.path.join(rocm, "bin", "hipcc")
    return cand if os.path.exists(cand) else "hipcc"


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    if verbose and (r.stdout or r.stderr):
        print(r.stdout + r.stderr, flush=True)
    return r


def generate_tables():
    sys.path.insert(0, CSRC)
    try:
        import gen_tables  # noqa: WPS433
    finally:
        sys.path.pop(0)
    path = os.path.join(CSRC, "teno_tables.h")
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        gen_tables.main(fh)
    os.replace(tmp, path)


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile and link libtenom.so; returns its path.  Always rebuilds."""
    os.makedirs(BUILD, exist_ok=True)
    generate_tables()
    hipcc = _hipcc()
    cmds = []
    objs = []
    for nf, k in UNITS:
        for unit in ("inst", "vjp", "tile"):
            obj = os.path.join(BUILD, f"{unit}_nf{nf}_k{k}.o")
            objs.append(obj)
            extra = TILE_FLAGS if unit == "tile" else (VJP_FLAGS if unit == "vjp" else [])
            cmds.append([hipcc, *HIPCC_FLAGS, *extra, f"-DTENOM_NF={nf}", f"-DTENOM_K={k}", "-c",
                         os.path.join(CSRC, "tenom_vjp_inst.hip" if unit == "vjp" else "tenom_inst.hip"), "-o", obj])
    for t in range(BATCH_TILES):
        obj = os.path.join(BUILD, f"batch_tile{t}.o")
        objs.append(obj)
        cmds.append([hipcc, *HIPCC_FLAGS, f"-DTENOM_TILE={t}", "-c",
                     os.path.join(CSRC, "tenom_batch_inst.hip"), "-o", obj])
    obj = os.path.join(BUILD, "batch_persist.o")
    objs.append(obj)
    # the persistent kernel loops over problems, steps, stages and segments
    # around the face: no machine-level loop-invariant code motion, as for the
    # tile sweeps
    cmds.append([hipcc, *HIPCC_FLAGS, "-DTENOM_PERSIST", "-mllvm", "-disable-machine-licm", "-c",
                 os.path.join(CSRC, "tenom_batch_inst.hip"), "-o", obj])
    for src in ("tenom_abi.hip", "tenom_batch.hip", "tenom_noalloc.hip"):
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        objs.append(obj)
        cmds.append([hipcc, *HIPCC_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
    if jobs is None:
        jobs = int(os.environ.get("MAX_JOBS", "0") or 0) or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(lambda c: _run(c, verbose), cmds))
    tmp = LIB + ".tmp"
    _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="--verbose" in sys.argv))
