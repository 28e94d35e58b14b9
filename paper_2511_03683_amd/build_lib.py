"""Compile the HIP sources of this package into libephbte.so for gfx950.

Usage: python -m paper_2511_03683_amd.build_lib  (or build() from Python).
The library is written next to this file and loaded by the ctypes binding.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libephbte.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 VALU ops are switched off for all device code.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-munsafe-fp-atomics", "-Wno-unused-command-line-argument"]


def build(verbose: bool = False, jobs: int = 4) -> str:
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    objs, procs = [], []
    for src in ("api.hip", "layout.cpp"):
        obj = os.path.join(bdir, src + ".o")
        if src.endswith(".hip"):
            cmd = [HIPCC, *DEVICE_FLAGS, *inc, "-c", os.path.join(CSRC, src), "-o", obj]
        else:
            cmd = [HIPCC, "-x", "c++", "-O3", "-std=c++17", "-fPIC", *inc, "-c",
                   os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        objs.append(obj)
    if any(p.wait() != 0 for p in procs):
        raise RuntimeError("HIP compilation failed")
    link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", OUT + ".tmp",
            "-lpthread"]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.check_call(link)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
