"""Builds libtpkmc.so for gfx950 with hipcc, in-tree.

The FP64 kernels and the host unit are compiled without FMA contraction
(bit-exact FP64 path, compensated sums); packed-FP32 instructions are
disabled for all device code.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libtpkmc.so")
ARCH = os.environ.get("TPKMC_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}", f"-I{INCLUDE}", f"-I{CSRC}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-munsafe-fp-atomics",
          "-Wall", "-Wno-unused-result", "-Wno-unused-value"]
UNITS = {
    "tpkmc_host.hip": ["-ffp-contract=off"],
    "tpkmc_f64.hip": ["-ffp-contract=off"],
    "tpkmc_f32.hip": ["-ffp-contract=fast-honor-pragmas"],
}


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    return "hipcc"


def build(verbose: bool = False) -> str:
    """Compile every unit and link libtpkmc.so next to this file."""
    cc = _hipcc()
    with tempfile.TemporaryDirectory(prefix="tpkmc_build_") as tmp:
        objs = []
        for unit, extra in UNITS.items():
            obj = os.path.join(tmp, unit.replace(".hip", ".o"))
            cmd = [cc, *COMMON, *extra, "-c", os.path.join(CSRC, unit), "-o", obj]
            if verbose:
                print(" ".join(cmd), file=sys.stderr)
            subprocess.check_call(cmd)
            objs.append(obj)
        out_tmp = LIB + ".tmp"
        cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", out_tmp, *objs]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        subprocess.check_call(cmd)
        os.replace(out_tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
