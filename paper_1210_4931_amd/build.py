"""Build the HIP library ``libmfwf.so`` for gfx950 in-tree.

Each ``csrc/*.hip`` file is compiled with hipcc; the objects are linked against the HIP
runtime that PyTorch ships, so that the library and PyTorch share one HIP/HSA runtime in
a process (PyTorch's device pointers and streams are then valid in the library).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmfwf.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["api.hip", "pixel.hip", "ringfft.hip", "legendre.hip", "harmonic.hip", "batched.hip",
           "polar.hip", "server.hip", "polbatched.hip", "templates.hip"]

HIPFLAGS = [
    "-std=c++17", "-O3", "-fPIC", "--offload-arch=gfx950",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def torch_lib_dir() -> str:
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec is None or spec.origin is None:
        raise RuntimeError("PyTorch is required: the library links against its HIP runtime")
    return os.path.join(os.path.dirname(spec.origin), "lib")


# The ring transforms run in several kernels that must round alike (the per-map forward and
# inverse transforms, the chained ring steps on the matrix-core columns, the split
# transforms): no floating-point contraction there, only the fused multiply-adds the code
# writes out.
FILE_FLAGS = {"ringfft.hip": ["-ffp-contract=off"]}


def source_hash() -> str:
    """SHA-256 (first 16 hex digits) of the library sources: keys the autotuner's cache, so
    that choices timed on other kernels are not reused."""
    import hashlib
    h = hashlib.sha256()
    files = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".h")))
    for f in files:
        h.update(f.encode())
        h.update(open(os.path.join(CSRC, f), "rb").read())
    h.update(open(os.path.join(INCLUDE, "mfwf.h"), "rb").read())
    h.update(repr((HIPFLAGS, FILE_FLAGS)).encode())  # the compile flags shape the kernels too
    return h.hexdigest()[:16]


def _compile(src: str, src_hash: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *HIPFLAGS, *FILE_FLAGS.get(src, []), "-I", INCLUDE, "-I", CSRC,
           "-DMFWF_SRC_HASH=\"%s\"" % src_hash,
           "-c", os.path.join(CSRC, src), "-o", obj, "-Rpass-analysis=kernel-resource-usage"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr))
    # per-kernel register, LDS and scratch figures of the compiler, kept next to the objects
    with open(os.path.join(BUILD, os.path.splitext(src)[0] + ".resources.txt"), "w") as f:
        f.write("\n".join(l for l in r.stderr.splitlines() if "remark:" in l))
    return obj


def resource_usage() -> dict:
    """{kernel symbol: {field: value}} from the last build's compiler remarks."""
    out = {}
    for src in SOURCES:
        path = os.path.join(BUILD, os.path.splitext(src)[0] + ".resources.txt")
        if not os.path.exists(path):
            continue
        cur = None
        for line in open(path):
            body = line.split("remark:", 1)[1].strip()
            if body.startswith("Function Name:"):
                cur = body.split(":", 1)[1].strip().split()[0]
                out[cur] = {}
            elif cur and ":" in body:
                k, v = body.split(":", 1)
                out[cur][k.strip()] = v.strip().split()[0]
    return out


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    src_hash = source_hash()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda f: _compile(f, src_hash), SOURCES))
    tl = torch_lib_dir()
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["g++", "-shared", "-o", tmp, *objs, "-L" + tl, "-l:libamdhip64.so",
           "-Wl,-rpath," + tl, "-Wl,--no-undefined", "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
