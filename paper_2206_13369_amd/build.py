"""Builds libmlpcp.so (the HIP kernels and the C ABI) for gfx950, in-tree.

    python -m paper_2206_13369_amd.build      # or build() from Python

Every HIP source is compiled with hipcc for gfx950 only, packed-FP32 ops
disabled, and linked into a shared library next to this file.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libmlpcp.so")
ARCH = "gfx950"

SOURCES = ["operators.hip", "eig.hip", "gram.hip", "dense.hip", "solver.hip", "fwt.hip", "profile.hip", "spectral.hip",
           "subspace.hip", "msvt.hip"]


def _hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the ROCm toolchain is required to build libmlpcp")


def _flags():
    return ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include")]


def build(verbose: bool = False, jobs: int = 8) -> str:
    os.makedirs(BUILD, exist_ok=True)
    cc = _hipcc()
    objs = []

    def compile_one(src):
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        cmd = [cc, *_flags(), "-c", os.path.join(CSRC, src), "-o", obj]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{res.stdout}\n{res.stderr}")
        msgs = [ln for ln in res.stderr.splitlines() if ln.strip() and "packed-fp32-ops" not in ln]
        if verbose and msgs:
            print("\n".join(msgs), file=sys.stderr)
        return obj

    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


# Host-code sanitizers for the argument-validation checks (tests/abi_host_check.c): each
# -fsanitize option applies to the host compilation only (the device code is built as
# usual and never runs in these checks).
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def build_host_sanitized(out_dir: str, jobs: int = 8) -> str:
    """Builds libmlpcp_san.so (host code under AddressSanitizer and UndefinedBehaviorSanitizer)
    and the validation driver tests/abi_host_check.c linked against it, in out_dir; returns
    the driver's path.  For the host-only checks of the C ABI: no GPU is needed to run it."""
    os.makedirs(out_dir, exist_ok=True)
    cc = _hipcc()
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), *SAN_FLAGS]

    def compile_one(src):
        obj = os.path.join(out_dir, src.replace(".hip", ".o"))
        res = subprocess.run([cc, *flags, "-c", os.path.join(CSRC, src), "-o", obj], capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{res.stderr}")
        return obj

    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    lib = os.path.join(out_dir, "libmlpcp_san.so")
    res = subprocess.run([cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *SAN_FLAGS, "-o", lib, *objs],
                         capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stderr}")
    clang = os.path.join(os.path.dirname(os.path.realpath(cc)), "..", "llvm", "bin", "clang")
    if not os.path.exists(clang):
        clang = "/opt/rocm/llvm/bin/clang"
    exe = os.path.join(out_dir, "abi_host_check")
    res = subprocess.run([clang, "-g", "-O1", "-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-I",
                          os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "abi_host_check.c"),
                          "-L", out_dir, "-lmlpcp_san", f"-Wl,-rpath,{out_dir}", "-lm", "-o", exe],
                         capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"driver build failed:\n{res.stderr}")
    return exe


if __name__ == "__main__":
    build(verbose=True)
