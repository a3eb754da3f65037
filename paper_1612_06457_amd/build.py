"""Build libcvamx.so for gfx950 with hipcc (in-tree, no JIT cache).

    python -m paper_1612_06457_amd.build        # or build() from Python
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
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libcvamx.so")

HIP_SOURCES = ["k_labels.hip", "k_moments.hip", "k_project.hip", "k_project_u16.hip", "k_soft.hip", "k_class.hip",
               "k_mfma.hip", "k_stretch.hip", "k_cluster.hip", "k_bands.hip", "k_scratch.hip", "k_roof.hip"]
HOST_SOURCES = ["api.cpp", "finisher.cpp", "pipeline.cpp"]

ARCH = os.environ.get("CVAMX_ARCH", "gfx950")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-I", os.path.join(ROOT, "include"), "-I", CSRC]
# Packed FP32 instructions are disabled for all device code (see the build
# notes in the design document); hipcc's host pass warns that it does not
# know the feature, which is harmless.
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + r.stdout)
    return r.stdout


def build(verbose: bool = False) -> str:
    """Compile every source and link libcvamx.so; returns its path."""
    hipcc = _hipcc()
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    for src in HIP_SOURCES:
        path = os.path.join(CSRC, src)
        if not os.path.exists(path):
            continue
        obj = os.path.join(BUILD, src + ".o")
        jobs.append([hipcc, "-x", "hip", *DEVICE, *COMMON, "-c", path, "-o", obj])
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(hipcc)))
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        jobs.append(["g++", *COMMON, "-Wall", "-D__HIP_PLATFORM_AMD__", "-I",
                     os.path.join(rocm, "include"), "-c", os.path.join(CSRC, src), "-o", obj])
    with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        outs = list(ex.map(_run, jobs))
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    objs = [j[-1] for j in jobs]
    tmp = LIB + ".tmp"
    _run([hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


def build_host_sanitized(out_dir: str) -> str:
    """The library with its host code (argument checks, scratch management,
    the FP64 finisher, the page pipeline) built by g++ with AddressSanitizer
    and UndefinedBehaviorSanitizer, linked with the device objects of the
    regular build (built first if missing).  Returns the path of
    libcvamx_asan.so in out_dir; load it with CVAMX_LIB_PATH pointing at it
    and the sanitizer runtime preloaded."""
    if not all(os.path.exists(os.path.join(BUILD, s + ".o")) for s in HIP_SOURCES):
        build()
    hipcc = _hipcc()
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(hipcc)))
    os.makedirs(out_dir, exist_ok=True)
    san = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined"]
    objs = []
    jobs = []
    for src in HOST_SOURCES:
        obj = os.path.join(out_dir, src + ".asan.o")
        jobs.append(["g++", "-O1", "-g", "-std=c++17", "-fPIC", *san, "-Wall", "-D__HIP_PLATFORM_AMD__",
                     "-I", os.path.join(rocm, "include"), "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                     "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        list(ex.map(_run, jobs))
    lib = os.path.join(out_dir, "libcvamx_asan.so")
    _run(["g++", "-shared", *san, "-o", lib, *objs, *[os.path.join(BUILD, s + ".o") for s in HIP_SOURCES],
          "-L", os.path.join(rocm, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(rocm, "lib")])
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
