"""Build libqcd.so (HIP kernels + C-ABI) for gfx950 with hipcc.

Every HIP file is compiled with packed-FP32 instructions disabled
(``-Xclang -target-feature -Xclang -packed-fp32-ops``); hipcc's host pass
warns that it does not know that feature, which is harmless.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libqcd.so")
# (source, object, extra flags): the Wilson operator is built once per storage
# precision so that its many kernel instantiations compile in parallel
SOURCES = [("dslash.hip", "dslash_f16.o", ["-DQCD_DSLASH_PREC=2"]),
           ("dslash.hip", "dslash_bf16.o", ["-DQCD_DSLASH_PREC=3"]),
           ("dslash.hip", "dslash_f32.o", ["-DQCD_DSLASH_PREC=1"]),
           ("dslash.hip", "dslash_f64.o", ["-DQCD_DSLASH_PREC=0"]),
           ("blas.hip", "blas.o", []), ("api.hip", "api.o", []), ("ptc.hip", "ptc.o", [])]
ARCH = os.environ.get("QCD_OFFLOAD_ARCH", "gfx950")

FLAGS = ["-O3", f"--offload-arch={ARCH}", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", INCLUDE, "-I", CSRC]


def _compile(spec) -> str:
    src, objname, extra = spec
    obj = os.path.join(BUILD, objname)
    cmd = ["hipcc", *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed for {src}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("link of libqcd.so failed")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
