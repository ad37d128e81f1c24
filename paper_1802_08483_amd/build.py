"""Builds libmapdec.so in-tree with hipcc for gfx950.

Every translation unit goes through hipcc with packed-FP32 instruction
selection disabled; the shared library lands next to this file.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmapdec.so")
SOURCES = ["k_misc.hip", "k_lattice.hip", "k_chain.hip", "k_app.hip", "k_app_mfma.hip",
           "k_outer.hip", "scratch.hip", "mapdec.cpp", "outer.cpp"]
# k_chain_ring.hip is compiled once per (precision, workgroup shape); the
# shapes (waves, states per thread) match kRingShapes in csrc/kernels.h
RING_SHAPES = [(1, 1, 0), (2, 1, 0), (4, 1, 0), (4, 2, 0), (8, 2, 0), (16, 2, 0), (16, 2, 1)]
VARIANTS = [("k_chain_ring.hip", f"chain_ring_{tag}_{k}",
             [f"-DCHAIN_T={t}", f"-DCHAIN_NW={nw}", f"-DCHAIN_SPL={spl}",
              f"-DCHAIN_ONEROW={one}", f"-DCHAIN_FN=chain_ring_{tag}_{k}"])
            for tag, t in (("f32", "float"), ("f64", "double"))
            for k, (nw, spl, one) in enumerate(RING_SHAPES)]
# k_adjoint.hip is compiled once per precision
VARIANTS += [("k_adjoint.hip", f"adj_{tag}", [f"-DADJ_T={t}", f"-DADJ_FN=adj_{tag}"])
             for tag, t in (("f32", "float"), ("f64", "double"))]
# k_app_tile.hip is compiled once per precision
VARIANTS += [("k_app_tile.hip", f"app_tile_{tag}", [f"-DAPP_T={t}", f"-DAPP_FN=app_tile_{tag}"])
             for tag, t in (("f32", "float"), ("f64", "double"))]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _compile(job) -> str:
    src, name, defines = job
    obj = os.path.join(BUILD, name + ".o")
    cmd = [HIPCC] + FLAGS + defines + ["-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return obj


def _check_unique_kernels(objs) -> None:
    """Objects built from one source with different -D switches must not
    define the same kernel: the linker would keep one definition for both
    launchers.  Every kernel's host stub must come from one object."""
    seen = {}
    for obj in objs:
        r = subprocess.run(["nm", "-g", "--defined-only", obj], capture_output=True, text=True)
        for line in r.stdout.splitlines():
            sym = line.split()[-1]
            if "__device_stub__" not in sym:
                continue
            if sym in seen and seen[sym] != obj:
                raise RuntimeError(f"kernel {sym} defined in {seen[sym]} and {obj}")
            seen[sym] = obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = [(s, s, []) for s in SOURCES] + VARIANTS
    # longest compiles first
    jobs.sort(key=lambda j: 0 if j[0] in ("k_chain_ring.hip", "k_app_tile.hip",
                                         "k_adjoint.hip") else 1)
    workers = max(1, min(16, os.cpu_count() or 1, len(jobs)))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(_compile, jobs))
    _check_unique_kernels(objs)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
