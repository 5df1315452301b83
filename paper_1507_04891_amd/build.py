"""Build of the gfx950 library liblbmix.so (hipcc, in-tree)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "liblbmix.so")
SOURCES = [os.path.join(HERE, "csrc", name)
           for name in ("lbmix_step_f64.hip", "lbmix_step_f32.hip", "lbmix_step_f32x.hip", "lbmix_step_bf16.hip", "lbmix_step_f16.hip",
                        "lbmix_step.hip", "lbmix_poisson.hip", "lbmix_net.hip", "lbmix_net_runtime.hip",
                        "lbmix_runtime.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # no packed FP32 instructions in generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-result",
]


def build(verbose: bool = False) -> str:
    """Compile the sources in parallel into objects under _build/, then link the library."""
    out = os.path.join(HERE, "_build")
    os.makedirs(out, exist_ok=True)
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(out, os.path.basename(src) + ".o")
        cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-c", "-o", obj, src]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), src))
        objs.append(obj)
    failed = [src for p, src in procs if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, "hipcc " + " ".join(failed))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
