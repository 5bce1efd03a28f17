"""Build the gfx950 shared library ``libs3cmtf.so`` from ``csrc/`` with hipcc.

Usage: ``python -m paper_1708_08640_amd.build`` (or ``build()`` from Python).
The host entry points and each group of kernel sets are separate translation
units, compiled in parallel and linked into one library written in-tree next
to this file.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libs3cmtf.so")
SOURCES = ["s3cmtf.hip", "sets_f32_3.hip", "sets_f32_4.hip", "sets_f64.hip", "sets_cp.hip",
           "sets_naive.hip", "sets_mx.hip"]
HEADERS = ["common.hpp", "contract.hpp", "kernels.hpp", "lockfree.hpp", "mfma.hpp", "qr.hpp", "plan.hpp", "sort.hpp"]
ARCH = os.environ.get("S3_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC",
    f"--offload-arch={ARCH}",
    "-munsafe-fp-atomics",
    # no packed-FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES] + [os.path.join(CSRC, h) for h in HEADERS] + [
        os.path.join(INCLUDE, "s3cmtf.h")]


# host code of the entry points (s3cmtf.hip) under AddressSanitizer and
# UndefinedBehaviorSanitizer; device code is built as usual.  A process that
# loads such a build must preload the compiler's shared ASan runtime.
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]


def asan_runtime() -> str:
    """Path of the shared ASan runtime of the compiler hipcc drives."""
    clang = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "bin", "clang")
    res = subprocess.run([clang, "-print-resource-dir"], capture_output=True, text=True, check=True)
    return os.path.join(res.stdout.strip(), "lib", "linux", "libclang_rt.asan-x86_64.so")


def build(verbose: bool = False, out: str = LIB, host_sanitize: bool = False) -> str:
    """Compile every HIP source for gfx950 and link the shared library (the
    in-tree one unless `out` names another path; `host_sanitize` instruments
    the entry points' host code)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tag = "%d" % os.getpid()
    odir = CSRC if out == LIB else os.path.dirname(os.path.abspath(out))
    objs = [os.path.join(odir, os.path.splitext(s)[0] + ".o.tmp" + tag) for s in SOURCES]

    def compile_one(i):
        extra = HOST_SANITIZE if host_sanitize and SOURCES[i] == "s3cmtf.hip" else []
        cmd = [hipcc, *FLAGS, *extra, "-I", INCLUDE, "-I", CSRC, "-c", "-o", objs[i],
               os.path.join(CSRC, SOURCES[i])]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)

    jobs = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    try:
        with ThreadPoolExecutor(jobs) as ex:
            list(ex.map(compile_one, range(len(SOURCES))))
        tmp = out + ".tmp" + tag
        link = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-shared-libsan"] if host_sanitize else []
        cmd = [hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *link, "-o", tmp, *objs]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(tmp, out)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    return out


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
    sys.exit(0)
