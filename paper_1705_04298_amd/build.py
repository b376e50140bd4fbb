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
# (source, extra define): the on-chip kernel file is compiled once per group of grid sizes
SOURCES = [("gerchberg_onchip.hip", f"FWR_ONCHIP_UNIT={u}") for u in range(5)] + ["gerchberg_multipass.hip", "gerchberg_fourier.hip", "gerchberg_fourier_mp.hip", "gen_screens.hip", "ext_hudgin.hip",
           "cnn.hip", "fallback.hip", "fwr_api.cpp", "cnn_api.cpp"]
ARCH = "gfx950"

# Packed FP32 VALU instructions are disabled for all device code.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libfwr)")


def _compile(cmd, verbose):
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


def build(verbose: bool = False, resource_usage: bool = False, defines=(), out: str = LIB, jobs: int = 0) -> str:
    """Compile every source to an object in parallel, then link the shared library."""
    from concurrent.futures import ThreadPoolExecutor

    base = [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++20", "-fPIC",
            "-Wall", "-Wno-unused-function", *DEVICE_FLAGS, *[f"-D{d}" for d in defines]]
    if resource_usage:
        base += ["-Rpass-analysis=kernel-resource-usage"]
    tag = f"{os.getpid()}_{abs(hash((out, tuple(defines)))) % 10**8}"
    objdir = os.path.join(os.path.dirname(out), f"_build_{tag}")
    os.makedirs(objdir, exist_ok=True)
    units = [s if isinstance(s, tuple) else (s, None) for s in SOURCES]
    objs = [os.path.join(objdir, f"{os.path.splitext(s)[0]}{'' if d is None else '_' + d.split('=')[1]}.o")
            for s, d in units]
    cmds = [base + ([] if d is None else [f"-D{d}"]) + ["-c", os.path.join(CSRC, s), "-o", o]
            for (s, d), o in zip(units, objs)]
    jobs = jobs or min(len(cmds), max(1, len(os.sched_getaffinity(0))), 16)
    try:
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            for f in [ex.submit(_compile, c, verbose) for c in cmds]:
                f.result()
        tmp = out + ".tmp"
        _compile([hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp], verbose)
        os.replace(tmp, out)
    finally:
        shutil.rmtree(objdir, ignore_errors=True)
    return out


if __name__ == "__main__":
    defs = [a[2:] for a in sys.argv[1:] if a.startswith("-D")]
    outs = [a.split("=", 1)[1] for a in sys.argv[1:] if a.startswith("--out=")]
    print(build(verbose="--verbose" in sys.argv, resource_usage="--resources" in sys.argv,
                defines=defs, out=outs[0] if outs else LIB))
