"""Build libdvm.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdvm.so")
SOURCES = [os.path.join(CSRC, f) for f in ("dvm_kernels.hip", "dvm_sens.hip", "dvm_so.hip", "dvm_macro.hip", "dvm_rbf.hip",
                                                 "dvm_host.cpp", "dvm_shape.cpp")]

# -packed-fp32-ops: keep the compiler from emitting packed FP32 VALU ops.
# -ffp-contract=off: every a*b+c is rounded as written, so a kernel body gives
# the same bits whichever kernel inlines it (single solve vs batch) and the
# velocity-face products v.S that decide upwinding round like the oracle's.
FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument"]


# the streaming reference kernels of the benchmark's roofline (not part of libdvm)
STREAM_LIB = os.path.join(HERE, "libdvm_stream.so")
STREAM_SOURCES = [os.path.join(CSRC, "dvm_stream.hip")]


def _hipcc(out: str, sources, verbose: bool) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = out + ".tmp"
    cmd = [hipcc, *FLAGS, "-o", tmp, *sources]
    res = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (res.stdout + res.stderr).splitlines()
                     if "packed-fp32-ops" not in l and "not a recognized feature" not in l)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{msgs}")
    if verbose and msgs.strip():
        print(msgs, file=sys.stderr)
    os.replace(tmp, out)
    return out


def build(verbose: bool = False) -> str:
    _hipcc(STREAM_LIB, STREAM_SOURCES, verbose)
    return _hipcc(LIB, SOURCES, verbose)


if __name__ == "__main__":
    print(build(verbose=True))
