"""Build libfwr.so (HIP, gfx950) in-tree.

    python -m paper_1705_04298_amd.build [--verbose]

Every build compiles from source; there is no cache.  The shared library is
written next to this file, where the ctypes binding looks for it.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfwr.so")
SOURCES = ["gerchberg_onchip.hip", "gerchberg_multipass.hip", "gerchberg_fourier.hip", "gen_screens.hip", "ext_hudgin.hip",
           "cnn.hip", "fallback.hip", "fwr_api.cpp", "cnn_api.cpp"]
ARCH = "gfx950"

# Packed FP32 VALU instructions are disabled for all device code.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libfwr)")


def build(verbose: bool = False, resource_usage: bool = False, defines=(), out: str = LIB) -> str:
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++20", "-fPIC", "-shared",
           "-Wall", "-Wno-unused-function", *DEVICE_FLAGS, *[f"-D{d}" for d in defines]]
    if resource_usage:
        cmd += ["-Rpass-analysis=kernel-resource-usage"]
    cmd += [os.path.join(CSRC, s) for s in SOURCES]
    tmp = out + ".tmp"
    cmd += ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    log = res.stdout + res.stderr
    # the host pass does not know the packed-fp32 feature; that warning is expected
    noise = "not a recognized feature for this target"
    shown = "\n".join(l for l in log.splitlines() if noise not in l and "ignoring feature" not in l)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{shown}")
    if verbose and shown.strip():
        print(shown)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    defs = [a[2:] for a in sys.argv[1:] if a.startswith("-D")]
    outs = [a.split("=", 1)[1] for a in sys.argv[1:] if a.startswith("--out=")]
    print(build(verbose="--verbose" in sys.argv, resource_usage="--resources" in sys.argv,
                defines=defs, out=outs[0] if outs else LIB))
