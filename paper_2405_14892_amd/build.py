"""Build the HIP library libmvn.so in-tree for gfx950 with hipcc.

Every source under csrc/ is compiled to an object, then linked into
paper_2405_14892_amd/libmvn.so.  ``python -m paper_2405_14892_amd.build``
rebuilds unconditionally.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
OBJ = os.path.join(ROOT, "_build", "obj")
LIB = os.path.join(HERE, "libmvn.so")
ARCH = os.environ.get("MVN_OFFLOAD_ARCH", "gfx950")

SOURCES = ["api.cpp", "kernels_chol.hip", "kernels_sov.hip", "kernels_sov_wide.hip", "kernels_sov_quad.hip",
           "kernels_sov_narrow.hip", "kernels_grad.hip",
           "kernels_tlr.hip", "kernels_tlr_sweep.hip", "kernels_mc.hip", "kernels_post.hip"]

# Per-file extra flags.  The sweep inlines the FP64 conditioning step into
# its row loop; machine loop-invariant code motion would hoist the step's
# ~60 materialised 64-bit constants out of that loop and spill registers.
EXTRA_FLAGS = {"kernels_sov.hip": ["-mllvm", "-disable-machine-licm"],
               "kernels_sov_wide.hip": ["-mllvm", "-disable-machine-licm"],
               "kernels_sov_quad.hip": ["-mllvm", "-disable-machine-licm"],
               "kernels_sov_narrow.hip": ["-mllvm", "-disable-machine-licm"],
               "kernels_grad.hip": ["-mllvm", "-disable-machine-licm"],
               "kernels_tlr_sweep.hip": ["-mllvm", "-disable-machine-licm"],
               "kernels_mc.hip": ["-mllvm", "-disable-machine-licm"]}

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions off for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found; the HIP library cannot be built")


def _compile(src: str) -> str:
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    cmd = [_hipcc(), *HIPCC_FLAGS, *EXTRA_FLAGS.get(src, []), "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj,
           f"-I{os.path.join(ROOT, 'include')}"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
