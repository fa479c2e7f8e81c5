"""Build step for the HIP libraries (gfx950), run by ``__graft_entry__.build``.

Compiles the ``csrc/*.hip`` sources with hipcc, and the host-only ``csrc/*.cpp`` (the
search planner) with g++, into ``libswmi.so``, which exports the C ABI of
``include/swmi.h``, and ``csrc/calib.hip`` alone into ``libswmi_calib.so`` (the
VALU calibration of ``include/swmi_calib.h``).  The libraries are written next to this
file so that they travel with the source tree.
"""
from __future__ import annotations

import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libswmi.so")
CALIB_LIB = os.path.join(HERE, "libswmi_calib.so")
CALIB_SRC = os.path.join(HERE, "csrc", "calib.hip")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-fvisibility=hidden", "-Wall",
    # keep the compiler from forming packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def sources():
    return sorted(s for s in glob.glob(os.path.join(HERE, "csrc", "*.hip")) if s != CALIB_SRC)


def host_sources():
    """Host-only C++ (the search planner), compiled by the host compiler."""
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.cpp")))


HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-fvisibility=hidden", "-Wall", "-Wextra",
              "-I", os.path.join(ROOT, "include")]


def _link(objs, lib, verbose):
    tmp = lib + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-Wl,--no-undefined", *objs,
           "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, capture_output=not verbose)
    os.replace(tmp, lib)


def build(verbose: bool = False, extra=None) -> str:
    objs = []
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    for src in sources() + [CALIB_SRC]:
        obj = os.path.join(bdir, os.path.basename(src) + ".o")
        cmd = [HIPCC, *FLAGS, *(extra or []), "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
        objs.append(obj)
    host_objs = []
    for src in host_sources():
        obj = os.path.join(bdir, os.path.basename(src) + ".o")
        cmd = ["g++", *HOST_FLAGS, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"g++ failed for {src}:\n{r.stderr}")
        host_objs.append(obj)
    _link(objs[:-1] + host_objs, LIB, verbose)
    _link(objs[-1:], CALIB_LIB, verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
