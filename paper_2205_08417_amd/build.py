"""Build libsnrt.so (HIP for gfx950) in-tree with hipcc.

Every translation unit is compiled with packed-FP32 instruction selection disabled
(``-target-feature -packed-fp32-ops``); the kernels are written for 64-wide wavefronts and
MFMA on CDNA4 only.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libsnrt.so")
# the longest compiles (the unrolled P_N kernel of degree 13, the products) first, so the
# pool starts them early
SOURCES = ["sn_pn13.hip", "sn_gemm_mfma.hip", "sn_step_fused.hip", "sn_step_fused_rho.hip",
           "sn_step_fused_dose.hip", "sn_step_fused_rho_dose.hip", "sn_step_fused_combine.hip",
           "sn_step_fused_adjoint.hip", "snrt_api.hip", "sn_step_f32.hip", "sn_step_f64.hip", "sn_adjoint.hip",
           "sn_reduce.hip", "sn_gemm_simple.hip", "sn_step2.hip", "sn_step_imex.hip",
           "sn_pn.hip", "snrt_pn_api.hip", "snrt_rollout.hip", "snrt_noalloc.hip",
           "snrt_eig.hip"]
ARCH = os.environ.get("SNRT_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

CFLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-function",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          # the compile-time operator tables of the larger P_N degrees (pn_pattern.h)
          "-fconstexpr-steps=500000000",
          "-I", os.path.join(ROOT, "include")]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *CFLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    # the host pass does not know the packed-FP32 feature and says so; drop that noise
    noise = "is not a recognized feature for this target"
    msgs = [ln for ln in (r.stdout + r.stderr).splitlines() if ln.strip() and noise not in ln]
    if msgs:
        sys.stderr.write("\n".join(msgs) + "\n")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 4)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
