"""Build the gfx950 HIP library (libpic.so) in-tree with hipcc.

Every kernel source compiles to its own object, then they link into one
shared library that exports the C ABI of include/pic.h.  Packed-FP32
instructions are disabled for all device code.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libpic.so")
ARCH = os.environ.get("PIC_OFFLOAD_ARCH", "gfx950")

CFLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-munsafe-fp-atomics",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall", "-Wno-unused-function"]


# Per-source extra flags.  The surrogate's kernels consume every MFMA result
# on the VALU (bias, SiLU, BF16 packing); keeping MFMA operands and results
# in VGPRs saves the accumulator-register copies.
FILE_FLAGS = {"k_mlp.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src)[:-4] + ".o")
    cmd = ["hipcc", *CFLAGS, *FILE_FLAGS.get(os.path.basename(src), []), "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


PROBE_SRC = os.path.join(HERE, "probe", "probes.hip")
PROBE_LIB = os.path.join(HERE, "libprobes.so")


def build_probes(verbose: bool = False) -> str:
    """The benchmark's measurement probes (LDS bandwidth, a dword copy for the
    HBM counter calibration) as their own small library."""
    tmp = PROBE_LIB + ".tmp"
    cmd = ["hipcc", *CFLAGS, "-shared", "-o", tmp, PROBE_SRC]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {PROBE_SRC}:\n{r.stderr}")
    os.replace(tmp, PROBE_LIB)
    if verbose:
        print(f"built {PROBE_LIB}")
    return PROBE_LIB


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, sources()))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    build_probes(verbose)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
