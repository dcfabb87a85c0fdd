"""Build libmpm.so (gfx950) in-tree with hipcc, and the hbm_probe and
valu_probe programs (plain kernels that measure the GPU's achievable HBM
bandwidth and VALU issue rate)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmpm.so")
PROBE = os.path.join(HERE, "hbm_probe")
VALU_PROBE = os.path.join(HERE, "valu_probe")
SOURCES = ["mpm_api.hip", "mpm_fit.hip", "mpm_map.hip", "mpm_serve.hip", "k_voxel.hip", "k_map.hip",
           "k_proj.hip"]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # keep packed-FP32 instructions out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-Wno-unused-value",
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    cmd = [hipcc] + FLAGS + ["-o", LIB + ".tmp"] + srcs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd, cwd=CSRC)
    os.replace(LIB + ".tmp", LIB)
    pflags = [f for f in FLAGS if f not in ("-fPIC", "-shared")]
    for out, src in ((PROBE, "hbm_probe.hip"), (VALU_PROBE, "valu_probe.hip")):
        cmd = [hipcc] + pflags + ["-o", out + ".tmp", os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd, cwd=CSRC)
        os.replace(out + ".tmp", out)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
