"""Build the HIP library libpowersort_hip.so for gfx950 with hipcc.

Usage: python -m paper_1805_04154_amd.build [--jobs N]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
BUILD_DIR = os.path.join(ROOT, "_build")
LIB_NAME = "libpowersort_hip.so"
LIB_PATH = os.path.join(HERE, LIB_NAME)
SOURCES = ["partition.hip", "tree.hip", "merge.hip", "api.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# -packed-fp32-ops: no packed fp32 instructions anywhere in device code.
CFLAGS = ["-std=c++17", "-O3", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-function",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(ROOT, "include")]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *CFLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int = 4, verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB_PATH + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB_PATH)
    if verbose:
        print(f"built {LIB_PATH}")
    return LIB_PATH


# Host-side sanitizers (AddressSanitizer + UndefinedBehaviorSanitizer) for
# the C ABI's host code in api.hip; each flag applies to the host pass only.
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
SAN_LIB_PATH = os.path.join(BUILD_DIR, "san", "libpowersort_hip_san.so")


def build_host_sanitized() -> str:
    """A copy of the library whose api.hip host code (argument checks,
    workspace layout, pool, status strings) is built with AddressSanitizer
    and UndefinedBehaviorSanitizer, linked with the regular objects of the
    other sources (built by build() first).  Load it with clang's ASan
    runtime preloaded (asan_runtime()) and POWERSORT_HIP_LIB pointing at it."""
    objs = [os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o") for src in SOURCES if src != "api.hip"]
    if not all(os.path.exists(o) for o in objs):
        build()
    os.makedirs(os.path.dirname(SAN_LIB_PATH), exist_ok=True)
    api_o = os.path.join(os.path.dirname(SAN_LIB_PATH), "api_san.o")
    flags = [f for f in CFLAGS if f != "-O3"] + ["-O1"]
    r = subprocess.run([HIPCC, *flags, *HOST_SANITIZE, "-c", os.path.join(CSRC, "api.hip"), "-o", api_o],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for the sanitized api.hip:\n{r.stderr}")
    r = subprocess.run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-shared-libsan", *HOST_SANITIZE,
                        "-o", SAN_LIB_PATH, api_o, *objs], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link of the sanitized library failed:\n{r.stderr}")
    return SAN_LIB_PATH


def asan_runtime() -> str:
    """clang's shared AddressSanitizer runtime (for LD_PRELOAD)."""
    import glob
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        raise FileNotFoundError("clang's libclang_rt.asan-x86_64.so not found under /opt/rocm/llvm")
    return hits[-1]


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=4)
    a = ap.parse_args()
    build(a.jobs, verbose=True)
    sys.exit(0)
