"""Build libmpcpcg.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libmpcpcg.so")
SOURCES = [os.path.join(CSRC, "mpcpcg.hip")]
HEADERS = [os.path.join(CSRC, f) for f in ("pcg_kernel.h", "lane_ops.h")] + [
    os.path.join(ROOT, "include", "mpcpcg.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"


def flags():
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
            # no packed FP32 (v_pk_*_f32) instructions anywhere in the device code
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC]


FLOORS_LIB = os.path.join(PKG, "libmpcpcg_floors.so")
FLOORS_SOURCES = [os.path.join(CSRC, "floors.hip")]
# debug build: LDS filled with NaN at the start of every task of the fused kernel
POISON_LIB = os.path.join(PKG, "libmpcpcg_poison.so")


def _compile(sources, lib, verbose, extra):
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + flags() + list(extra) + sources + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in res.stderr.splitlines() if noise not in l)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + err)
    if verbose and err.strip():
        print(err, file=sys.stderr)
    os.replace(tmp, lib)
    return lib


def build(verbose: bool = False, extra=()) -> str:
    """Compile libmpcpcg.so, its LDS-poisoning debug build libmpcpcg_poison.so and the
    benchmark's floor probes, libmpcpcg_floors.so (always recompiles all three)."""
    _compile(FLOORS_SOURCES, FLOORS_LIB, verbose, extra)
    _compile(SOURCES, POISON_LIB, verbose, list(extra) + ["-DMPC_LDS_POISON=1"])
    return _compile(SOURCES, LIB, verbose, extra)


if __name__ == "__main__":
    print(build(verbose=True))
