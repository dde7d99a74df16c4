"""Compile the gfx950 HIP library ``libnucleus.so`` in place with hipcc.

Every ``csrc/*.hip`` file is compiled to an object for gfx950 only and linked
into one shared library next to this file. Packed FP32 instructions are
disabled (the library has no floating point on its paths anyway).
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libnucleus.so")
DRIVER = os.path.join(HERE, "nd_profile")
COPY = os.path.join(HERE, "nd_copy")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_FEATURES = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(os.path.dirname(HERE), "include"),
]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return obj


def _runtime_dirs() -> list[str]:
    """Where the HIP runtime is searched at load time when no process-wide
    copy is loaded yet. PyTorch ships its own libamdhip64.so.7 (same SONAME):
    the Python binding imports torch before loading this library, so in a
    torch process the library runs on torch's runtime; a process without
    torch (the profiling driver) uses /opt/rocm's."""
    return ["/opt/rocm/lib"]


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + f".tmp{os.getpid()}"
    rpath = ":".join(_runtime_dirs())
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs,
           f"-Wl,-rpath,{rpath}", "-Wl,--disable-new-dtags", "-Wl,-z,defs", "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc link failed")
    os.replace(tmp, LIB)
    # profiling driver: the C ABI from a plain C++ program (no Python/torch)
    drv_tmp = DRIVER + f".tmp{os.getpid()}"
    cmd = ["g++", "-O2", "-std=c++17", "-I" + os.path.join(os.path.dirname(HERE), "include"),
           os.path.join(HERE, "nd_profile.cpp"), "-L" + HERE, "-lnucleus",
           f"-Wl,-rpath,{HERE}:/opt/rocm/lib", "-o", drv_tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("driver build failed")
    os.replace(drv_tmp, DRIVER)
    # counter calibration: a plain copy kernel of known size
    copy_tmp = COPY + f".tmp{os.getpid()}"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-O3", "-std=c++17", *HIP_FEATURES,
           os.path.join(HERE, "nd_copy.hip"), f"-Wl,-rpath,{rpath}", "-o", copy_tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("copy tool build failed")
    os.replace(copy_tmp, COPY)
    if verbose:
        print("built", LIB, ",", DRIVER, "and", COPY)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
