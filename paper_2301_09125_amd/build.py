"""Build the HIP library liblpa.so for gfx950 (in-tree, next to this file)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB_PATH = os.path.join(HERE, "liblpa.so")
SOURCES = ["csrc/lpa_prep.hip", "csrc/lpa_vote.hip", "csrc/lpa_mod.hip", "csrc/lpa_batch.hip", "csrc/lpa_learned.hip",
           "csrc/lpa_runtime.hip", "csrc/lpa_noalloc.hip",
           "csrc/lpa_copra.hip"]
ARCH = os.environ.get("LPA_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 instructions are disabled for all device code.
FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result"]


PROBE_SRC = os.path.join(ROOT, "bench_gather_probe.hip")
PROBE_LIB = os.path.join(ROOT, "libgather_probe.so")


def build_probe(verbose: bool = False) -> str:
    """The bench-only random-gather probe (libgather_probe.so at the repo
    root, loaded by bench.py --gather-ceiling); not part of liblpa.so."""
    tmp = PROBE_LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-o", tmp, PROBE_SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, PROBE_LIB)
    return PROBE_LIB


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    tmp = LIB_PATH + ".tmp"
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
           "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose=True))
