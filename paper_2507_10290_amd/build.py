"""Build the HIP library libtop.so in-tree for gfx950 (hipcc, no JIT cache).

Usage: python -m paper_2507_10290_amd.build [--jobs N]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import re
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libtop.so")

SOURCES = ["sweep_f32.hip", "sweep_f64.hip", "sweep_axis.hip", "poly_f32.hip", "poly_f64.hip", "numeric_f32.hip", "numeric_f64.hip", "numeric_quad_f32.hip", "numeric_quad_f64.hip", "adjoint_f32.hip", "adjoint_f64.hip",
           "setup.hip",
           "finalize.hip", "grad.hip", "adapt.hip", "api.cpp", "solve_static.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SCRATCH_LIMIT = 8192   # kScratchLimit of csrc/common.h
# Packed FP32 VALU forms are kept out of the generated code.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-I" + INCLUDE, "-I" + CSRC,
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument"]


def _kernel_resources(remarks: str) -> list:
    """Parse the compiler's kernel-resource-usage remarks into one dict per kernel."""
    out, cur = [], None
    for line in remarks.splitlines():
        m = re.search(r"remark:\s+(.*?)\s*\[-Rpass-analysis", line)
        if not m:
            continue
        text = m.group(1)
        if text.startswith("Function Name:"):
            cur = {"name": text.split(":", 1)[1].strip()}
            out.append(cur)
        elif cur is not None and ":" in text:
            k, v = text.split(":", 1)
            cur[k.strip()] = v.strip()
    return out


def _compile(src: str):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + FLAGS + ["-Rpass-analysis=kernel-resource-usage", "-x", "hip", "-c",
                             os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile of {src} failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj, _kernel_resources(r.stderr)


def build(jobs: int = 0, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(_compile, SOURCES))
    objs = [o for o, _ in results]
    kernels = [k for _, ks in results for k in ks]
    # A kernel whose private stack depth the compiler cannot bound may overrun the scratch the
    # runtime gives it; refuse to produce such a library.
    dyn = [k["name"] for k in kernels if k.get("Dynamic Stack", "False") != "False"]
    with open(os.path.join(BUILD, "kernel_resources.txt"), "w") as f:
        for k in kernels:
            f.write(" ".join(f"{a}={b}" for a, b in k.items()) + "\n")
    if dyn:
        raise RuntimeError("kernels with a dynamic stack: " + ", ".join(dyn))
    # The library raises the runtime's per-lane stack limit to kScratchLimit (common.h) and relies
    # on every kernel's fixed scratch fitting under it.
    big = [k["name"] for k in kernels if int(k.get("ScratchSize [bytes/lane]", "0")) > SCRATCH_LIMIT]
    if big:
        raise RuntimeError(f"kernels with more than {SCRATCH_LIMIT} bytes of scratch per lane: " + ", ".join(big))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=0)
    a = ap.parse_args()
    build(a.jobs, verbose=True)
    sys.exit(0)
