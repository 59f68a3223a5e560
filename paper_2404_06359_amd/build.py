"""Builds ``libgtsr.so`` (HIP kernels for gfx950 + host C ABI) in this package.

Host C++ goes through g++, the HIP translation unit through hipcc with
``--offload-arch=gfx950``; objects land in ``_build/`` at the repository root.
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
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libgtsr.so")

ARCH = os.environ.get("GTSR_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CXX = os.environ.get("CXX", "g++")

HOST_SOURCES = ["encode.cpp", "capi.cpp", "tune.cpp", "serve.cpp", "quant.cpp", "cones.cpp", "gtsrfile.cpp"]
HIP_SOURCES = ["decode.hip", "attrs.hip", "calib.hip"]

COMMON = ["-O3", "-std=c++17", "-fPIC", "-I", INCLUDE, "-I", CSRC]
# Host files that call the HIP runtime API (autotuner, server) compile with g++.
HIP_HOST = ["-D__HIP_PLATFORM_AMD__", "-isystem", "/opt/rocm/include"]
# Packed FP32 instructions are kept out of all device code.
HIP_FLAGS = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError(f"build step failed: {os.path.basename(cmd[-1])}")
    return r


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    objs = []
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        jobs.append([CXX, *COMMON, *HIP_HOST, "-Wall", "-Wextra", "-pthread", "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        jobs.append([HIPCC, *COMMON, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    with ThreadPoolExecutor(len(jobs)) as ex:
        for r in ex.map(_run, jobs):
            if verbose and (r.stdout or r.stderr):
                sys.stderr.write(r.stdout + r.stderr)
    tmp = f"{LIB}.{os.getpid()}.tmp"   # private per process: test workers may build at once
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


SANITIZE_DIR = os.path.join(BUILD, "sanitize")
SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]


def build_sanitized(verbose: bool = False) -> str:
    """A host-sanitized copy of the library for CPU test runs:
    ``_build/sanitize/libgtsr.so``.  The host C++ (encoder, validator,
    planner, quantizer, cones, tuner, server, .gtsr files) is compiled by g++ with
    AddressSanitizer and UndefinedBehaviorSanitizer; the HIP translation
    units keep their normal build (no sanitizer reaches device code).  Load
    it by setting GTSR_LIBRARY to its path, with the sanitizer runtime
    preloaded into the Python process."""
    os.makedirs(SANITIZE_DIR, exist_ok=True)
    jobs, objs = [], []
    for src in HOST_SOURCES:
        obj = os.path.join(SANITIZE_DIR, src + ".o")
        jobs.append([CXX, "-O1", "-std=c++17", "-fPIC", "-I", INCLUDE, "-I", CSRC, *HIP_HOST, *SANITIZE,
                     "-pthread", "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for src in HIP_SOURCES:
        obj = os.path.join(SANITIZE_DIR, src + ".o")
        jobs.append([HIPCC, *COMMON, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    with ThreadPoolExecutor(len(jobs)) as ex:
        for r in ex.map(_run, jobs):
            if verbose and (r.stdout or r.stderr):
                sys.stderr.write(r.stdout + r.stderr)
    out = os.path.join(SANITIZE_DIR, "libgtsr.so")
    _run([CXX, "-shared", "-fPIC", "-pthread", *SANITIZE, *objs, "-L/opt/rocm/lib", "-lamdhip64",
          "-Wl,-rpath,/opt/rocm/lib", "-o", f"{out}.{os.getpid()}.tmp"])
    os.replace(f"{out}.{os.getpid()}.tmp", out)
    return out


if __name__ == "__main__":
    print(build_sanitized(verbose=True) if "--sanitize" in sys.argv else build(verbose=True))
