"""Build libdrc_cae.so (HIP, gfx950) in-tree with hipcc.

Each translation unit is compiled to an object in parallel, then linked
into one shared library next to this file.
"""
from __future__ import annotations

import os
import subprocess
import sys
import time
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libdrc_cae.so")
SOURCES = ["drc_cae.hip", "net.hip", "plan.hip", "gemm_f32.hip", "gemm_bf16.hip", "gemm_fp8.hip", "fused_fwd.hip",
           "envmap.hip", "interp.hip", "augment.hip", "unet.hip", "layer_bands.hip", "static_ws.hip", "fused_fp8.hip", "unet_train.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

CFLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # keep the compiler from forming packed-FP32 VALU instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-Wno-unused-function",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
]


# Per-source flags. The whole-network BF16 kernels (fused_fwd.hip) are
# scheduled for long LDS load clauses: their inner loops keep more operand
# reads in flight that way (same instructions and results, about 2 % faster).
# The FP8 kernel is left on the default schedule, which keeps it free of
# register spills.
SRC_FLAGS = {
    "fused_fwd.hip": ["-mllvm", "-amdgpu-sched-strategy=max-memory-clause"],
}


def _compile(src: str) -> str:
    obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + CFLAGS + SRC_FLAGS.get(src, []) + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(OBJ, exist_ok=True)
    t0 = time.time()
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), 8)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    if verbose:
        print(f"[build] {LIB} ({time.time() - t0:.1f} s)", flush=True)
    return LIB


if __name__ == "__main__":
    build()
