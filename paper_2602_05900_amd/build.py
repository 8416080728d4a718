"""Build the HOTRG HIP library in-tree: paper_2602_05900_amd/libhotrg.so,
and the stand-alone unit-ceiling microbenchmark paper_2602_05900_amd/peak_bench.

Every source is compiled for gfx950 with hipcc and linked against the HIP
runtime that PyTorch ships, so a process that has imported torch holds
exactly one HIP runtime (loading the system ROCm runtime beside torch's would
put two in one process).  No other ROCm library is linked.

    python -m paper_2602_05900_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libhotrg.so")
PEAK = os.path.join(PKG, "peak_bench")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

SOURCES = ["gemm.hip", "tensor_ops.hip", "eig.hip", "hotrg.cpp", "itebd.hip", "noalloc.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-mcode-object-version=5",
    # keep the compiler from emitting packed-FP32 vector ops
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
    "-Wno-unused-command-line-argument",
]


def torch_lib_dir() -> str:
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec is None or not spec.submodule_search_locations:
        raise RuntimeError("torch is not importable; its HIP runtime is the one the library links against")
    return os.path.join(list(spec.submodule_search_locations)[0], "lib")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd[:3])} ...")
    return r


def build(verbose: bool = False) -> str:
    """Compile every HIP source and link libhotrg.so; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    include = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs = []
    for src in SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        lang = ["-x", "hip"]
        _run([hipcc, *lang, *HIPCC_FLAGS, *include, "-c", os.path.join(CSRC, src), "-o", obj], verbose)
        objs.append(obj)
    tlib = torch_lib_dir()
    clang = os.path.join(ROCM, "llvm", "bin", "clang++")
    tmp = LIB + ".tmp"
    _run([clang, "-shared", "-fPIC", "-o", tmp, *objs,
          "-L", tlib, "-l:libamdhip64.so",
          f"-Wl,-rpath,{tlib}", "-Wl,--no-undefined", "-lstdc++", "-lm"], verbose)
    os.replace(tmp, LIB)
    # the microbenchmark is its own program (no torch in its process): plain hipcc link
    tmp = PEAK + ".tmp"
    _run([hipcc, "-x", "hip", *[f for f in HIPCC_FLAGS if f != "-fPIC"], os.path.join(CSRC, "peak.hip"), "-o", tmp],
         verbose)
    os.replace(tmp, PEAK)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
