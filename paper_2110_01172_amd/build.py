"""Build ``libdctx.so`` (HIP kernels + C ABI) for gfx950 with hipcc.

Every source is compiled to an object under ``_build/`` (in parallel), then
linked into ``paper_2110_01172_amd/libdctx.so``.  Run ``python -m
paper_2110_01172_amd.build``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libdctx.so")
ARCH = os.environ.get("DCTX_OFFLOAD_ARCH", "gfx950")

SOURCES = ["capi.cpp", "plan.cpp", "noalloc.hip", "dct1d.hip", "dct1d_long.hip", "dct2d.hip", "fast2d.hip", "split2d.hip", "dct3d.hip", "poisson.hip", "batch.hip", "small_mfma.hip", "rowcol.hip", "server.cpp"]

# Packed-FP32 instructions are switched off for all device code; -O3 with
# ordinary FP32 arithmetic, FMA contraction allowed, no fast-math.
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(HERE, "..", "include")]


def _hipcc() -> str:
    cand = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(cand):
        raise RuntimeError("hipcc not found")
    return cand


# Host-side AddressSanitizer / UndefinedBehaviorSanitizer build of the same
# sources (a test aid: the device code is compiled as usual, every sanitizer
# flag applies to the host pass only).
SAN_BUILD = os.path.join(HERE, "_build_san")
SAN_LIB = os.path.join(HERE, "libdctx_san.so")
SAN_FLAGS = ["-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def _compile(src: str, build_dir: str = BUILD, extra=()) -> str:
    obj = os.path.join(build_dir, os.path.basename(src) + ".o")
    cmd = [_hipcc(), "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj] + COMMON + list(extra)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{res.stdout}\n{res.stderr}")
    # hipcc's host pass warns about the device-only target feature; keep other warnings
    lines = [ln for ln in (res.stdout + res.stderr).splitlines()
             if "packed-fp32-ops" not in ln and ln.strip()]
    if lines:
        sys.stderr.write(f"[{src}]\n" + "\n".join(lines) + "\n")
    return obj


def build(jobs: int = 8) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", "-pthread", f"--offload-arch={ARCH}", "-o", tmp] + objs
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    return LIB


# Write-count build: the same sources with every final output store also
# counted per output word (a test aid; see dctx_debug_write_count).
WC_BUILD = os.path.join(HERE, "_build_wc")
WC_LIB = os.path.join(HERE, "libdctx_wc.so")


def build_write_count(jobs: int = 8) -> str:
    """libdctx_wc.so: the library with output-store counting compiled in."""
    os.makedirs(WC_BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda src: _compile(src, WC_BUILD, ["-DDCTX_WRITE_COUNT"]), SOURCES))
    tmp = WC_LIB + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", "-pthread", f"--offload-arch={ARCH}", "-o", tmp] + objs
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, WC_LIB)
    return WC_LIB


def build_sanitized(jobs: int = 8) -> str:
    """libdctx_san.so: the library with ASan + UBSan on its host code."""
    os.makedirs(SAN_BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda src: _compile(src, SAN_BUILD, SAN_FLAGS), SOURCES))
    tmp = SAN_LIB + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", "-pthread", f"--offload-arch={ARCH}", "-o", tmp] + SAN_FLAGS + objs
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"sanitized link failed:\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, SAN_LIB)
    return SAN_LIB


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "--sanitize":
        print(build_sanitized())
    elif len(sys.argv) > 1 and sys.argv[1] == "--write-count":
        print(build_write_count())
    else:
        print(build())
