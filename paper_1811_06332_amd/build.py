"""Build libctfmm.so for gfx950: run the operator generator, then hipcc.

    python -m paper_1811_06332_amd.build [--skip-gen]
"""
from __future__ import annotations

import os
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
GEN_DIR = os.path.join(CSRC, "generated")
LIB = os.path.join(PKG, "libctfmm.so")

SOURCES = ["ctfmm_api.hip", "ctfmm_kernels.hip", "ctfmm_adaptive.hip", "ctfmm_mlp.hip", "ctfmm_dual.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fno-gpu-rdc", "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-missing-braces",
]


def generate(verbose=True):
    t = time.time()
    subprocess.run([sys.executable, os.path.join(PKG, "gen", "gen_operators.py"), GEN_DIR], check=True)
    if verbose:
        print(f"[build] generator: {time.time() - t:.1f}s", flush=True)


def compile_lib(verbose=True):
    """Compile every source to an object in parallel, then link the library."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    obj_dir = os.path.join(ROOT, "_build")
    os.makedirs(obj_dir, exist_ok=True)
    t = time.time()
    flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(obj_dir, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc, *flags, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c", os.path.join(CSRC, src),
               "-o", obj]
        if verbose:
            print("[build] " + " ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd)))
        objs.append(obj)
    failed = [src for src, pr in procs if pr.wait() != 0]
    if failed:
        raise RuntimeError(f"hipcc failed on {', '.join(failed)}")
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", LIB + ".tmp"]
    if verbose:
        print("[build] " + " ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    if verbose:
        print(f"[build] hipcc: {time.time() - t:.1f}s -> {LIB}", flush=True)
    return LIB


def build(skip_gen=False, verbose=True):
    if not skip_gen or not os.path.exists(os.path.join(GEN_DIR, "ctfmm_gen.h")):
        generate(verbose)
    return compile_lib(verbose)


if __name__ == "__main__":
    build(skip_gen="--skip-gen" in sys.argv)
