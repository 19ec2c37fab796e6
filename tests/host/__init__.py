"""Host builds of product code for CPU tests (test infrastructure).

`deposit_host.hip` drives the particle kernel's deposit arithmetic on the CPU;
build() compiles it with hipcc (host code only runs; the device part is empty).
`asan_plugin` points the CPU tests at AddressSanitizer builds of the host code.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
BUILD = os.path.join(HERE, "_build")
SO = os.path.join(BUILD, "libdeposit_host.so")
CSRC = os.path.join(os.path.dirname(os.path.dirname(HERE)), "paper_1606_02862_amd", "csrc")
SOURCES = [os.path.join(HERE, "deposit_host.hip")] + [
    os.path.join(CSRC, f) for f in ("pic_deposit.hpp", "pic_device.hpp", "pic_internal.hpp")]


def build(force: bool = False, so: str = SO, extra: tuple = ()) -> str:
    """Compile libdeposit_host.so (or `so`, with the extra hipcc flags `extra`)
    if it is missing or older than its sources."""
    if not force and os.path.exists(so):
        t = os.path.getmtime(so)
        if all(os.path.getmtime(s) <= t for s in SOURCES):
            return so
    os.makedirs(os.path.dirname(so), exist_ok=True)
    tmp = so + ".tmp"
    subprocess.check_call(["hipcc", "-O2", "-std=c++17", "--offload-arch=gfx950", "-shared", "-fPIC", *extra,
                           "-o", tmp, SOURCES[0]], stderr=subprocess.DEVNULL)
    os.replace(tmp, so)
    return so
