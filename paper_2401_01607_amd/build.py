"""Build libtaches.so (HIP, gfx950) in-tree.

Every .hip source under csrc/ is compiled separately with hipcc, then linked
into ``paper_2401_01607_amd/libtaches.so``.  Packed-FP32 instructions are
disabled for the device code (``-packed-fp32-ops``): the kernels are written
for plain v_fma_f32.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD_DIR = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libtaches.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=off", "-Wall", "-Wno-unused-result",
    "-I", INCLUDE, "-I", CSRC,
]
LDFLAGS = [f"--offload-arch={ARCH}", "-shared", "-fPIC", "-Wl,-rpath,/opt/rocm/lib"]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src: str) -> str:
    obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
    cmd = [HIPCC, *CFLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {os.path.basename(src)}")
    errs = [l for l in r.stderr.splitlines() if "error" in l]
    if errs:
        sys.stderr.write("\n".join(errs) + "\n")
    return obj


def build(jobs: int = 8, verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    srcs = sources()
    with ThreadPoolExecutor(max_workers=min(jobs, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *LDFLAGS, "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link of libtaches.so failed")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def asm(src_name: str, out: str) -> None:
    """Write the gfx950 assembly of one source (for inspection)."""
    cmd = [HIPCC, *CFLAGS, "--cuda-device-only", "-S", os.path.join(CSRC, src_name), "-o", out]
    subprocess.run(cmd, check=True)


if __name__ == "__main__":
    build(verbose=True)
