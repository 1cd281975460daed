"""Build librka.so for gfx950 with hipcc (in-tree, no JIT cache).

Every HIP translation unit is compiled with packed-FP32 instructions
disabled; the sampler unit (norms, running sum, row stream) is also compiled
with FP contraction off so that its arithmetic is one rounded IEEE operation
per written operation.
"""
from __future__ import annotations

import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB_PATH = os.path.join(PKG, "librka.so")

ARCH = os.environ.get("RKA_OFFLOAD_ARCH", "gfx950")
SOURCES = {
    "rka_setup.hip": ["-ffp-contract=off"],
    "rka_iter.hip": [],
    "rka_sstep.hip": [],
    "rka_blk.hip": [],
    "rka_rkab.hip": [],
    "rka_dense.hip": [],
    "rka_batch.hip": [],
    "rka_spectral.hip": [],
    "rka_api.hip": [],
}


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _common_flags():
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I" + INCLUDE, "-I" + CSRC, "-Wall", "-Wno-unused-result"]


def build(verbose: bool = False) -> str:
    """Compile every HIP source and link librka.so.  Always recompiles."""
    os.makedirs(BUILD, exist_ok=True)
    cc = hipcc()

    def compile_one(item):
        src, extra = item
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        cmd = [cc, *_common_flags(), *extra, "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-6000:]}")
        if verbose and r.stderr.strip():
            print(r.stderr)
        return obj

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(compile_one, SOURCES.items()))
    tmp = LIB_PATH + ".tmp"
    cmd = [cc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-6000:]}")
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose=True))
