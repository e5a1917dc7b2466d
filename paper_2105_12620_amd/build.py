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
           "csrc/noalloc.hip", "csrc/peaks.hip",
           "csrc/spectrum.hip", "csrc/api.cpp"]
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


# Host-side AddressSanitizer and UndefinedBehaviorSanitizer for the C-ABI
# host code (api.cpp only: it holds no device code); the sanitizer runtime is
# preloaded by the process that loads such a build (asan_runtime()).
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def asan_runtime() -> str:
    """Path of the compiler's shared AddressSanitizer runtime (it carries the
    UndefinedBehaviorSanitizer handlers too)."""
    clang = os.environ.get("BNLAT_CLANG", "/opt/rocm/llvm/bin/clang")
    res = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    return res.stdout.strip()


def build(verbose: bool = False, sanitize_host: bool = False, out: str | None = None) -> str:
    """Compile every source for gfx950 and link libbnlat.so (or `out`).  With
    sanitize_host the host code of the C ABI is instrumented (a test build)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    lib = out or LIB
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    with tempfile.TemporaryDirectory(prefix="bnlat_build_") as tmpd:
        objs = [os.path.join(tmpd, os.path.basename(s) + ".o") for s in srcs]
        cmds = [[hipcc, *FLAGS, *(HOST_SANITIZE if sanitize_host and s.endswith(".cpp") else []), "-c",
                 os.path.join(HERE, s), "-o", o] for s, o in zip(srcs, objs)]
        jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            results = list(ex.map(_run, cmds))
        errs = []
        for src, (rc, err) in zip(srcs, results):
            if rc != 0:
                raise RuntimeError(f"hipcc failed on {src} ({rc}):\n{err}")
            if err.strip():
                errs.append(err)
        tmp = lib + ".tmp"
        rc, err = _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp])
        if rc != 0:
            raise RuntimeError(f"hipcc link failed ({rc}):\n{err}")
    if verbose and errs:
        print("\n".join(errs), file=sys.stderr)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
