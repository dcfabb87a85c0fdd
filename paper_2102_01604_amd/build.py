"""Build libmpm.so (gfx950) in-tree with hipcc."""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmpm.so")
OBJ_DIR = os.path.join(HERE, "_build")
SOURCES = ["mpm_api.hip", "mpm_fit.hip", "mpm_map.hip", "mpm_serve.hip", "mpm_noise.hip", "mpm_tune.hip",
           "mpm_noalloc.hip",
           "k_voxel.hip", "k_map.hip", "k_proj.hip", "k_noise.hip"]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # keep packed-FP32 instructions out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-Wno-unused-value",
]


def build(verbose: bool = False) -> str:
    """Compile every source to an object (in parallel, one hipcc per file),
    then link libmpm.so."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ_DIR, exist_ok=True)
    cflags = [f for f in FLAGS if f != "-shared"]
    objs = [os.path.join(OBJ_DIR, os.path.splitext(s)[0] + ".o") for s in SOURCES]

    def compile_one(src, obj):
        cmd = [hipcc] + cflags + ["-c", "-o", obj, os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        return subprocess.run(cmd, cwd=CSRC, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)

    jobs = max(1, min(len(SOURCES), os.cpu_count() or 1, 8))
    with concurrent.futures.ThreadPoolExecutor(jobs) as pool:
        results = list(pool.map(compile_one, SOURCES, objs))
    for src, r in zip(SOURCES, results):
        out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
        if out.strip():
            print(out, file=sys.stderr, flush=True)
        if r.returncode:
            raise subprocess.CalledProcessError(r.returncode, f"hipcc -c {src}")
    cmd = [hipcc] + FLAGS + ["-o", LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd, cwd=CSRC)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
