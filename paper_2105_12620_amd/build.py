"""Build the gfx950 shared library ``libbnlat.so`` in-tree with hipcc.

Each source is compiled to an object in its own hipcc process (in parallel),
then the objects are linked into the shared library."""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["csrc/count.hip", "csrc/kernels.hip", "csrc/swap.hip", "csrc/sampler.hip", "csrc/mfma.hip",
           "csrc/noalloc.hip", "csrc/peaks.hip", "csrc/api.cpp"]
LIB = os.path.join(HERE, "libbnlat.so")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=off",
    # never generate packed FP32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]
NOISE = "is not a recognized feature for this target"


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in res.stderr.splitlines() if NOISE not in l)
    return res.returncode, err


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    with tempfile.TemporaryDirectory(prefix="bnlat_build_") as tmpd:
        objs = [os.path.join(tmpd, os.path.basename(s) + ".o") for s in srcs]
        cmds = [[hipcc, *FLAGS, "-c", os.path.join(HERE, s), "-o", o] for s, o in zip(srcs, objs)]
        jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            results = list(ex.map(_run, cmds))
        errs = []
        for src, (rc, err) in zip(srcs, results):
            if rc != 0:
                raise RuntimeError(f"hipcc failed on {src} ({rc}):\n{err}")
            if err.strip():
                errs.append(err)
        tmp = LIB + ".tmp"
        rc, err = _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp])
        if rc != 0:
            raise RuntimeError(f"hipcc link failed ({rc}):\n{err}")
    if verbose and errs:
        print("\n".join(errs), file=sys.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
