"""Build libsmc_mpc.so (HIP kernels for gfx950 + C++ host orchestrator).

Usage: python -m paper_1506_02869_amd.build [--jobs N]
Objects go to _build/ at the repository root, the library next to this file.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(PKG, "libsmc_mpc.so")
BUILD = os.path.join(ROOT, "_build")

SOURCES = ["kernels_rng.hip", "kernels_wind.hip", "kernels_rollout.hip", "kernels_rollout_pw.hip", "kernels_rollout_pt.hip",
           "kernels_rollout_wm.hip", "kernels_rollout_wm_tv.hip", "kernels_rollout_batch.hip",
           "kernels_grad.hip",
           "kernels_smc.hip", "kernels_batch.hip", "kernels_plant.hip", "smc_mpc.cpp",
           "smc_batch.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         # packed FP32 instructions stay disabled (see the design notes)
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # a*b+c is fused only within one source expression, so kernels that
         # share arithmetic (single-scenario and batched) round identically
         "-ffp-contract=on",
         # bitwise | and & on comparisons are deliberate (no short-circuit branches)
         "-Wall", "-Wno-unused-function", "-Wno-bitwise-instead-of-logical",
         "-I", INCLUDE, "-I", CSRC]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    lang = ["-x", "hip"]
    cmd = [HIPCC, *lang, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    warn = "\n".join(l for l in r.stderr.splitlines()
                     if "packed-fp32-ops" not in l and l.strip())
    if "warning" in warn:
        sys.stderr.write(warn + "\n")
    return obj


def build(jobs: int | None = None, verbose: bool = True) -> str:
    if not os.path.exists(HIPCC) and shutil.which("hipcc") is None:
        raise RuntimeError("hipcc not found")
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 4, 8)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}")
    return OUT


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    a = ap.parse_args()
    build(a.jobs)
