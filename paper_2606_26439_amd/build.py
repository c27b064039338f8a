"""Builds libmaxsim.so (the gfx950 HIP kernels and the C ABI) in-tree with hipcc.

Every HIP translation unit is compiled for gfx950 only, with packed-FP32
instruction selection disabled, then linked into one shared library that
resolves the HIP runtime already loaded by the host process.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libmaxsim.so")
BUILD_DIR = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# (source, object name, extra flags); the fused scorer is compiled once per
# element type so the four instantiation sets build in parallel.
# Token values are finite, so no NaN reaches the fused scorer's maxima: they
# need no quieting of each matrix-core result before the max (the overlong-
# query NaN is written as a bit pattern). Measured 3-5% faster for grouped
# queries and FP8; the FP32 form (type 0) measured 1% slower and keeps the
# default.
SOURCES = [("fused_inst.hip", f"fused_dt{t}",
            [f"-DFUSED_DT={t}"] + (["-fno-honor-nans"] if t != 0 else []))
           for t in range(4)] + [
    ("fused_dispatch.cpp", "fused_dispatch", []),
    # NaN never reaches the PQ maxima (every table entry and every decoded
    # dot product is finite), so the maxima need no NaN canonicalisation
    ("pq.hip", "pq", ["-fno-honor-nans"]),
    ("pq_mfma.hip", "pq_mfma", ["-fno-honor-nans"]),
    # the same holds for the residual scorer (finite table entries and codes)
    ("residual.hip", "residual", ["-fno-honor-nans"]),
    ("topk.hip", "topk", []),
    ("quantize.hip", "quantize", []),
    ("probe.hip", "probe", []),
    ("validate.hip", "validate", []),
    ("api.cpp", "api", []),
]

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-result", "-I", os.path.join(HERE, "..", "include")]


def _deps(src):
    """Files an object depends on: its source and the headers it can include
    (the fused scorer's implementation header only for its own unit)."""
    hdrs = [os.path.join(CSRC, h) for h in ("device_common.h", "kernels.h")]
    hdrs.append(os.path.join(HERE, "..", "include", "maxsim.h"))
    if src == "fused_inst.hip":
        hdrs.append(os.path.join(CSRC, "fused_impl.h"))
    if src in ("fused_inst.hip", "topk.hip"):
        hdrs.append(os.path.join(CSRC, "select_impl.h"))
    return [os.path.join(CSRC, src)] + hdrs + [os.path.abspath(__file__)]


def _stale(spec) -> bool:
    src, name, _ = spec
    obj = os.path.join(BUILD_DIR, name + ".o")
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(d) > t for d in _deps(src))


def _compile(spec) -> str:
    src, name, extra = spec
    obj = os.path.join(BUILD_DIR, name + ".o")
    cmd = [HIPCC, *COMMON, *extra, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False, only_changed: bool = False) -> str:
    """Compiles every source (only_changed: only objects older than their
    source or headers) and links the library."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    todo = [sp for sp in SOURCES if not only_changed or _stale(sp)]
    workers = min(max(1, len(todo)), max(1, min(8, os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(workers) as ex:
        list(ex.map(_compile, todo))
    objs = [os.path.join(BUILD_DIR, name + ".o") for _, name, _ in SOURCES]
    tmp = OUT + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}")
    return OUT


if __name__ == "__main__":
    build(verbose=True, only_changed="--changed" in sys.argv[1:])
    sys.exit(0)
