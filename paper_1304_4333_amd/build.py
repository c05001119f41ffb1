"""Build libsps.so (HIP, gfx950) in-tree from paper_1304_4333_amd/csrc.

Every translation unit is compiled by hipcc for gfx950 only, in parallel,
then linked into paper_1304_4333_amd/libsps.so.  `incremental=True` reuses
objects whose inputs (source, headers, flags) are unchanged.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libsps.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

CFLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are kept off: the compiler must not form them
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-but-set-variable",
    "-I", os.path.join(ROOT, "include"),
]


# MFMA results in VGPRs instead of AGPRs: removes the accumulator copies that
# the default heuristic inserts around the epilogue.  Measured faster for the
# FP32 and BF16 kernels; the FP64 unit stays on the default assignment (the
# compiler fails on some FP64 instantiations with the flag).
# The pipelined BF16x3 kernels take it where it measured faster: the forward
# kernels for C >= 4 (multi6 17.3 against 19.0 ms) and the binary adjoint
# kernel (ar100 3.03 against 3.15 ms), not the binary forward kernel (ar100
# 1.41 ms without, 1.60 ms with).
FILE_FLAGS = {
    "loglik_fp32.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
    "loglik_bf16.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
    "loglik_bf16_wide.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
    "loglik_pipe_fwd_b.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
    "loglik_pipe_fwd_c.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
    "loglik_pipe_fwd_d.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
    "loglik_pipe_grad.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
}


def _flags(src: str) -> list:
    return CFLAGS + FILE_FLAGS.get(os.path.basename(src), [])


def _sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def _digest(src: str) -> str:
    h = hashlib.sha256()
    h.update(" ".join(_flags(src)).encode())
    for f in [src] + sorted(glob.glob(os.path.join(CSRC, "*.h"))) + [os.path.join(ROOT, "include", "sps.h")]:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _compile(src: str, incremental: bool) -> str:
    base = os.path.splitext(os.path.basename(src))[0]
    obj = os.path.join(BUILD, f"{base}.{_digest(src)}.o")
    if incremental and os.path.exists(obj):
        return obj
    tmp = obj + ".tmp"
    # one set of flags per unit: a failure is a build error, never a silent
    # rebuild with other options (the object digest names the flags used)
    r = subprocess.run([HIPCC] + _flags(src) + ["-c", src, "-o", tmp], capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "not a recognized feature" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{err}")
    if err.strip():
        sys.stderr.write(err + "\n")
    os.replace(tmp, obj)
    return obj


def build(incremental: bool = False, jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = _sources()
    jobs = jobs or min(len(srcs), os.cpu_count() or 4, 16)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, incremental), srcs))
    tmp = LIB + ".tmp"
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs,
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(incremental="--incremental" in sys.argv))
