"""Build ``libirfilter.so`` (HIP kernels + C ABI) for gfx950 with hipcc, in-tree.

The translation units compile in parallel (the kernels of each pixel type sit in
their own unit) and are linked into one shared library."""

from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB_PATH = os.path.join(PKG, "libirfilter.so")
BUILD_DIR = os.path.join(PKG, "_build")
SOURCES = [os.path.join(CSRC, n) for n in ("batch_cl_a.hip", "batch_cl_b.hip", "stack_u16.hip", "stack_u8.hip",
                                          "stack_large_u16.hip", "stack_large_u8.hip", "stack_huge_u16.hip",
                                          "stack_huge_u8.hip", "batch_c0.hip",
                                          "batch_c1.hip", "batch.hip", "irfilter.hip", "server.hip", "fused.hip")]
ARCH = os.environ.get("IRF_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    # never emit packed-fp32 VALU instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise subprocess.CalledProcessError(res.returncode, cmd, res.stdout, res.stderr)


def build(force: bool = True, verbose: bool = False) -> str:
    """Compile the library; returns its path.  Raises CalledProcessError on failure."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    os.makedirs(BUILD_DIR, exist_ok=True)
    objs = [os.path.join(BUILD_DIR, os.path.splitext(os.path.basename(s))[0] + ".o") for s in SOURCES]
    jobs = max(1, min(len(SOURCES), os.cpu_count() or 1))
    with cf.ThreadPoolExecutor(jobs) as ex:
        futs = [ex.submit(_run, ["hipcc", *HIPCC_FLAGS, "-c", "-o", o, s], verbose) for s, o in zip(SOURCES, objs)]
        for f in futs:
            f.result()
    tmp = LIB_PATH + ".tmp"
    _run(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs], verbose)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose=True))
