"""Build libspi.so (HIP for gfx950 + host C++) in-tree with hipcc.

Usage: ``python -m paper_1305_5683_amd.build`` or ``build()`` from Python.
Objects go to ``paper_1305_5683_amd/_build/``; the shared library is
``paper_1305_5683_amd/libspi.so``.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libspi.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

HIP_SOURCES = ["k_gemm.hip", "k_dense.hip", "k_sparse.hip", "k_learned.hip",
               "k_model.hip", "api_noalloc.hip"]
CPP_SOURCES = ["analysis.cpp", "analysis_io.cpp", "api.cpp", "api_learned.cpp",
               "api_batch.cpp", "api_model.cpp"]

COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
          f"-I{os.path.join(PKG, '..', 'include')}"]
# Device code: gfx950 only; hardware FP64 atomics; packed FP32 ops disabled.
HIP_FLAGS = [f"--offload-arch={ARCH}", "-munsafe-fp-atomics",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(src: str, hip: bool) -> tuple[str, subprocess.Popen]:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + COMMON + (HIP_FLAGS if hip else [f"--offload-arch={ARCH}"])
    if not hip:  # host-only C++ against the HIP runtime headers
        cmd += ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"]
    cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
    p = subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                         text=True)
    return obj, p


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = [_compile(s, True) for s in HIP_SOURCES] + \
           [_compile(s, False) for s in CPP_SOURCES]
    objs, errors = [], []
    for obj, p in jobs:
        out, _ = p.communicate()
        if verbose and out:
            sys.stdout.write(out)
        if p.returncode != 0:
            errors.append(out)
        objs.append(obj)
    if errors:
        raise RuntimeError("libspi compile failed:\n" + "\n".join(errors))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                       text=True)
    if r.returncode != 0:
        raise RuntimeError("libspi link failed:\n" + r.stdout)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
