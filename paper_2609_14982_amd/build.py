"""Build libfmbtf.so in place: host setup and C ABI with g++, kernels with
hipcc for gfx950.  Run through __graft_entry__.build() or `python -m
paper_2609_14982_amd.build`."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libfmbtf.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]
# -ffp-contract=off keeps the setup's FP64 upwind decisions free of fused
# multiply-adds, so they are reproducible bit for bit
HOST_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall", "-Wno-unused-function"]
HIP_SOURCES = ("device.hip", "krylov.hip", "model_map.hip", "eikonal.hip", "setup_gpu.hip")
# the first-arrival update and the GPU setup pass round every product and
# sum as written (compared with a NumPy evaluation of the same formulas, and
# with the host setup bit for bit)
HIP_EXTRA = {"eikonal.hip": ["-ffp-contract=off"], "setup_gpu.hip": ["-ffp-contract=off"]}


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


SANITIZE_FLAGS = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined",
                  "-g"]
LIB_SANITIZE = os.path.join(PKG, "_build_sanitize", "libfmbtf_sanitize.so")


def build_sanitize(verbose: bool = False) -> str:
    """The host setup and C ABI (setup.cpp, capi.cpp) built with the address
    and undefined-behaviour sanitizers, linked with the kernels of an
    ordinary build, for host-side checks on the CPU: load it with the
    sanitizer runtimes preloaded and FMBTF_LIB pointing at it."""
    hip_objs = [src.replace(".hip", ".o") for src in HIP_SOURCES]
    if not all(os.path.exists(os.path.join(BUILD, o)) for o in hip_objs):
        build(verbose)
    out_dir = os.path.dirname(LIB_SANITIZE)
    os.makedirs(out_dir, exist_ok=True)
    objs = []
    for src in ("setup.cpp", "capi.cpp"):
        obj = os.path.join(out_dir, src.replace(".cpp", ".o"))
        _run(["g++", *HOST_FLAGS, *SANITIZE_FLAGS, "-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, src), "-o",
              obj], verbose)
        objs.append(obj)
    objs += [os.path.join(BUILD, o) for o in hip_objs]
    gcc_lib = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", LIB_SANITIZE, *objs, "-pthread",
          "-L", os.path.dirname(gcc_lib), "-lasan", "-lubsan"], verbose)
    return LIB_SANITIZE


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    for src in ("setup.cpp", "capi.cpp"):
        obj = os.path.join(BUILD, src.replace(".cpp", ".o"))
        jobs.append((["g++", *HOST_FLAGS, "-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj], obj))
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        jobs.append(([HIPCC, *HIP_FLAGS, *HIP_EXTRA.get(src, []), "-I", INCLUDE, "-I", CSRC, "-c",
                      os.path.join(CSRC, src), "-o", obj], obj))
    # the translation units compile independently (device.hip, the largest,
    # first so that it overlaps the rest)
    from concurrent.futures import ThreadPoolExecutor
    workers = max(1, min(len(jobs), os.cpu_count() or 1, 8))
    with ThreadPoolExecutor(workers) as pool:
        for f in [pool.submit(_run, cmd, verbose) for cmd, _ in sorted(jobs, key=lambda j: "device.hip" not in j[0][-3])]:
            f.result()
    objs = [obj for _, obj in jobs]
    tmp = LIB + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-pthread"], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
