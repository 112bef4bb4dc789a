"""Builds the HIP library ``libpdd.so`` in-tree for gfx950 (hipcc cross-compiles
without a GPU). Run as ``python -m paper_1512_02818_amd.build``."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libpdd.so")
SOURCES = ["path_kernel.hip", "reduce_kernel.hip", "pdd_runtime.hip", "pdd_server.hip", "pdd_fit.hip", "grid_kernel.hip", "pdd_noalloc.hip"]
HEADERS = ["pdd_internal.hpp", "host_runtime.hpp"]

# Packed FP32 instructions are switched off: hipcc -O3 would otherwise form
# them from plain float code. Contraction is off so that every fused
# multiply-add is written in the source and all kernels round alike.
FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-parameter", "-Wno-unused-command-line-argument",
    "-I" + os.path.join(ROOT, "include"),
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    raise RuntimeError("hipcc not found")


PROBE_LIB = os.path.join(HERE, "libpdd_probe.so")
PROBE_SOURCES = ["issue_probe.hip"]


def build_probe(verbose: bool = False) -> str:
    """Compile the VALU issue-rate probe (the benchmark's --issue-rates mode)
    into its own library, libpdd_probe.so."""
    srcs = [os.path.join(HERE, "csrc", s) for s in PROBE_SOURCES]
    tmp = PROBE_LIB + ".tmp"
    cmd = [hipcc()] + FLAGS + srcs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed (probe)")
    os.replace(tmp, PROBE_LIB)
    return PROBE_LIB


def build(verbose: bool = False) -> str:
    """Compile every HIP source into libpdd.so (always recompiles), and the
    issue-rate probe into libpdd_probe.so."""
    srcs = [os.path.join(HERE, "csrc", s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [hipcc()] + FLAGS + srcs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed")
    # the host pass warns about the GPU-only target feature; drop only that line
    noise = [l for l in (res.stdout + res.stderr).splitlines()
             if l.strip() and "packed-fp32-ops" not in l and "warning generated" not in l]
    if verbose and noise:
        print("\n".join(noise))
    os.replace(tmp, LIB)
    build_probe(verbose)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
