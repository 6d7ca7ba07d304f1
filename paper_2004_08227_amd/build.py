"""Builds libmplpxx.so in-tree with hipcc for gfx950.

Every HIP translation unit is compiled with packed FP32 instructions disabled
and FP contraction off (each entry of a min-plus pass must be exactly one IEEE
add followed by a minimum).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmplpxx.so")
# The same objects linked against /opt/rocm's HIP runtime only, for processes
# that do not load PyTorch (profiling under rocprofv3, whose tool library
# brings /opt/rocm's HSA runtime: with PyTorch's bundled HIP runtime next to
# it the process would hold two HSA runtimes).
LIB_ROCM = os.path.join(HERE, "libmplpxx_rocm.so")

SOURCES = ["solver.cpp", "batch.cpp", "schedule.cpp", "handshake.hip", "dual.hip", "batch.hip", "adjoint.hip",
           "rules.hip", "noalloc.hip", "probe.hip"]
ARCH = os.environ.get("MPLPXX_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wno-unused-command-line-argument",
          f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(ROOT, "include")]


# The handshake kernels see no NaN: inputs are validated finite (FP32:
# |cost| <= 1e18), padded tile entries are +inf (per-matching engine) or
# 2^126 (mailbox and wave engines), padded labels of the structured passes
# +inf, and no pass can form inf - inf.  Telling the compiler so lets min
# reductions skip the quieting of their operands and fold into DPP forms;
# on non-NaN operands the results are bitwise the same.
EXTRA = {"handshake.hip": ["-fno-honor-nans"], "batch.hip": ["-fno-honor-nans"], "rules.hip": ["-fno-honor-nans"]}


def _compile(src: str, build_dir: str = BUILD, defines=()) -> str:
    obj = os.path.join(build_dir, os.path.basename(src) + ".o")
    cmd = [HIPCC, *COMMON, *EXTRA.get(src, []), *defines, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def hip_runtime_dir() -> str:
    """Directory of the HIP runtime the library links against: PyTorch's
    bundled copy when present, so that a process using both PyTorch and this
    library runs one HIP runtime and can share device pointers and streams
    between them; /opt/rocm/lib otherwise."""
    try:
        import importlib.util
        spec = importlib.util.find_spec("torch")
        if spec and spec.origin:
            d = os.path.join(os.path.dirname(spec.origin), "lib")
            if os.path.exists(os.path.join(d, "libamdhip64.so")):
                return d
    except Exception:
        pass
    return "/opt/rocm/lib"


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    """Compiles and links the library to `out`; `defines` (e.g. a
    diagnostics macro) go to every translation unit."""
    build_dir = BUILD if out == LIB else out + "_build"
    os.makedirs(build_dir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda src: _compile(src, build_dir, defines), SOURCES))
    _link(objs, out, hip_runtime_dir())
    if out == LIB:
        _link(objs, LIB_ROCM, "/opt/rocm/lib")
    if verbose:
        print(f"built {out}")
    return out


def _link(objs, out, rt):
    tmp = out + ".tmp"
    rpath = [f"-Wl,-rpath,{rt}"] + (["-Wl,-rpath,/opt/rocm/lib"] if rt != "/opt/rocm/lib" else [])
    cmd = ["g++", "-shared", "-fPIC", "-o", tmp, *objs, f"-L{rt}", "-lamdhip64", *rpath, "-Wl,--no-undefined"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
