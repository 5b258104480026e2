"""Build libeeid.so (gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = os.path.join(PKG, "csrc", "eeid.hip")
DEPS = [os.path.join(PKG, "csrc", f) for f in ("eeid.hip", "eeid_tridiag.hpp", "eeid_tridiag_c.hpp", "eeid_band.hpp", "eeid_identity.hpp", "eeid_latency.hpp")]
LIB = os.path.join(PKG, "libeeid.so")
ARCH = "gfx950"

HIPCC_FLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-shared",
    # never emit packed FP32 arithmetic (v_pk_*_f32)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    return "hipcc"


PHASE_LIB = os.path.join(PKG, "libeeid_phase.so")   # instrumented with per-phase timers


def build(force: bool = True, extra=(), phase_timers: bool = False) -> str:
    lib = PHASE_LIB if phase_timers else LIB
    if not force and os.path.exists(lib) and all(os.path.getmtime(lib) >= os.path.getmtime(d) for d in DEPS):
        return lib
    tmp = lib + ".tmp"
    flags = ["-DEEID_PHASE_TIMERS"] if phase_timers else []
    cmd = [hipcc(), *HIPCC_FLAGS, *flags, *extra, "-o", tmp, SRC]
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(force="--lazy" not in sys.argv, phase_timers="--phase-timers" in sys.argv))
