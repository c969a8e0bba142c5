"""Build libmertens.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_1108_0135_amd.build   (or __graft_entry__.build()).
"""
from __future__ import annotations

import hashlib
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libmertens.so")
SOURCES = ["mertens_kernels.hip", "mertens_runtime.hip"]
ARCH = os.environ.get("MERTENS_OFFLOAD_ARCH", "gfx950")


KERNEL_SOURCES = ("mertens_kernels.hip", "mertens_internal.h")


def kernel_source_sha256() -> str:
    """SHA-256 over the kernel sources; compiled in so that a stored tuning
    (tuned_<arch>.json) is applied only to the kernels it was measured on."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def hipcc_command(out: str = LIB) -> list[str]:
    return [
        "hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
        f'-DMERTENS_KERNEL_SHA256="{kernel_source_sha256()}"', f'-DMERTENS_ARCH_NAME="{ARCH}"',
        "-ldl",
        # keep the compiler from forming packed fp32 instructions
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-function",
        "-I", os.path.join(ROOT, "include"), "-I", CSRC,
        *[os.path.join(CSRC, s) for s in SOURCES],
        "-o", out,
    ]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = hipcc_command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        sys.stderr.write(proc.stdout + proc.stderr)
        raise RuntimeError("hipcc failed building libmertens.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
