"""Builds the HIP library libmr.so in-tree for gfx950 (hipcc cross-compiles; no GPU needed).

Each source is compiled to an object of its own (in parallel) under _build/, then the objects
are linked into the shared library.
"""
from __future__ import annotations

import glob
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libmr.so")
OBJDIR = os.path.join(ROOT, "_build")

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + res.stdout + res.stderr)


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every HIP source and link libmr.so (always recompiles). Returns the library path."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = sources()
    objs = [os.path.join(OBJDIR, os.path.basename(s)[:-4] + ".o") for s in srcs]
    cmds = [[hipcc, *HIPCC_FLAGS, "-I", INCLUDE, "-I", CSRC, "-c", s, "-o", o] for s, o in zip(srcs, objs)]
    jobs = jobs or max(1, min(len(cmds), os.cpu_count() or 1, 8))
    with ThreadPoolExecutor(jobs) as ex:
        for f in [ex.submit(_run, c, verbose) for c in cmds]:
            f.result()
    tmp = LIB + ".tmp"
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


# The host half of every source instrumented by AddressSanitizer and UndefinedBehaviorSanitizer
# (the device code is not instrumented: each flag is for the host compilation only).
SANITIZE_HOST = [
    "-Xarch_host", "-fsanitize=address",
    "-Xarch_host", "-fsanitize=undefined",
    "-Xarch_host", "-fno-sanitize-recover=undefined",
    "-Xarch_host", "-fno-omit-frame-pointer",
]


def build_host_check(outdir: str, verbose: bool = False, jobs: int | None = None) -> str:
    """Build tests/host_check.cpp against every HIP source with the host sanitizers into outdir;
    returns the executable's path (run it with ASAN_OPTIONS=detect_leaks=0: the HIP runtime keeps
    allocations until exit)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(outdir, exist_ok=True)
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *SANITIZE_HOST, "-I", INCLUDE, "-I", CSRC]
    srcs = sources() + [os.path.join(ROOT, "tests", "host_check.cpp")]
    objs = [os.path.join(outdir, os.path.basename(s).rsplit(".", 1)[0] + ".o") for s in srcs]
    cmds = [[hipcc, *flags, "-x", "hip", "-c", s, "-o", o] for s, o in zip(srcs, objs)]
    jobs = jobs or max(1, min(len(cmds), os.cpu_count() or 1, 8))
    with ThreadPoolExecutor(jobs) as ex:
        for f in [ex.submit(_run, c, verbose) for c in cmds]:
            f.result()
    exe = os.path.join(outdir, "host_check")
    _run([hipcc, "--offload-arch=gfx950", *SANITIZE_HOST, *objs, "-o", exe], verbose)
    return exe


if __name__ == "__main__":
    print(build(verbose=True))
