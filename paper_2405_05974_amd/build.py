"""Build libchem.so (host C ABI + gfx950 kernels) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libchem.so")
PROBE_LIB = os.path.join(HERE, "libchem_probe.so")
ARCH = os.environ.get("CHEM_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
    # packed FP32 forms are kept out of generated code on this target
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unknown-warning-option",
]
SOURCES = [os.path.join(CSRC, "chem_kernels.hip"), os.path.join(CSRC, "chem_host.cpp"),
           os.path.join(CSRC, "chem_server.cpp"), os.path.join(CSRC, "chem_jit.cpp")]


def build(verbose: bool = False) -> str:
    """Compile every source into paper_2405_05974_amd/libchem.so, and the measurement
    probes into libchem_probe.so (always rebuilds)."""
    objs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, os.path.basename(src) + ".o")
        cmd = ["hipcc", "-c", *HIP_FLAGS]
        if src.endswith(".cpp"):
            cmd += ["-x", "hip"]
        cmd += [src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp, "-lhiprtc", "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    # measurement probes (FP64 FMA rate, cost of one exp), a library of their own
    probe_src = os.path.join(CSRC, "chem_probe.cpp")
    tmp = PROBE_LIB + ".tmp"
    cmd = ["hipcc", *HIP_FLAGS, "-x", "hip", "-shared", probe_src, "-o", tmp, "-lhiprtc"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, PROBE_LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
