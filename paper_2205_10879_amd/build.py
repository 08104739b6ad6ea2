"""Compile the HIP sources of the FastMuyGPs library for gfx950 into
paper_2205_10879_amd/libfastmuygps.so (in-tree, so it travels with the repo).

    python -m paper_2205_10879_amd.build      # or build() from Python
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libfastmuygps.so")

SOURCES = ["fmg_api.hip", "fmg_prep.hip", "fmg_exact.hip", "fmg_screen.hip", "fmg_rerank.hip",
           "fmg_precompute.hip", "fmg_precompute32.hip", "fmg_precompute_wide.hip", "fmg_predict.hip",
           "fmg_server.hip", "fmg_loss.hip", "fmg_grad.hip", "fmg_prune.hip", "fmg_noalloc.hip"]

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed FP32 instructions are switched off for every device function.
CFLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", INCLUDE, "-I", CSRC,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument"]


# Per-file additions.  The precompute keeps its MFMA accumulators in
# ordinary VGPRs (no copies between accumulation and vector registers in its
# loops, and no AGPR allocation on top of the VGPRs).
# fmg_screen.hip runs without IEEE mode (no sNaN quieting), so min/max of MFMA
# results need no canonicalisation; every value it screens is finite.
EXTRA = {"fmg_precompute32.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
         "fmg_screen.hip": ["-mno-amdgpu-ieee", "-fno-honor-nans"]}


def _compile(src: str) -> str:
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + CFLAGS + EXTRA.get(src, []) + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr[-8000:]))
    return obj


def build(jobs: int = 8, verbose: bool = False) -> str:
    """Compile every source and link the shared library.  Always rebuilds."""
    if shutil.which(HIPCC) is None and not os.path.exists(HIPCC):
        raise RuntimeError("hipcc not found at %s" % HIPCC)
    os.makedirs(OBJDIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=max(1, min(jobs, len(SOURCES)))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr[-8000:]))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
