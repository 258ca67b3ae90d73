"""Build the HIP library in-tree: ``libbytestore.so`` next to this file.

hipcc compiles the host encoder (C++17) and the gfx950 kernels into one shared
library with a plain C ABI (``include/bytestore.h``).  Packed FP32 instructions
are disabled for all device code.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbytestore.so")
SOURCES = [os.path.join(CSRC, f) for f in (
    "host_encode.cpp", "k_misc.hip", "k_scan_slices.hip", "k_scan_lt.hip", "k_scan_gt.hip", "k_scan_eq.hip",
    "k_scan_between.hip", "k_scan_packed_a.hip", "k_scan_packed_b.hip", "k_batch.hip", "k_batch_short.hip", "k_batch_packed.hip")]
HEADERS = [os.path.join(CSRC, "internal.h"), os.path.join(CSRC, "device_common.h"), os.path.join(CSRC, "scan_kernel.h"), os.path.join(CSRC, "slice_scan.h"),
           os.path.join(CSRC, "batch_kernel.h"),
           os.path.join(ROOT, "include", "bytestore.h")]
BUILD_DIR = os.path.join(ROOT, "_build")
ARCH = os.environ.get("BST_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), "hipcc"):
        if os.path.sep not in cand or os.path.exists(cand):
            return cand
    return "hipcc"


FLAGS = ["-O3", "-std=c++17", "--offload-arch=" + ARCH, "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def compile_command(src: str, obj: str) -> list:
    return [hipcc(), *FLAGS, "-c", src, "-o", obj]


def link_command(objs: list, out: str) -> list:
    return [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-o", out]


def _jobs() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def build(verbose: bool = False) -> str:
    """Compile every source (always: this is the 'does it build' step) and link."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    objs = [os.path.join(BUILD_DIR, os.path.basename(s) + ".o") for s in SOURCES]
    procs = []
    pending = list(zip(SOURCES, objs))
    failed = []
    while pending or procs:
        while pending and len(procs) < _jobs():
            src, obj = pending.pop(0)
            cmd = compile_command(src, obj)
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        src, p = procs.pop(0)
        out, _ = p.communicate()
        if p.returncode != 0:
            failed.append((src, out))
    if failed:
        for src, out in failed:
            sys.stderr.write("---- %s\n%s\n" % (src, out))
        raise RuntimeError("hipcc failed: " + ", ".join(os.path.basename(s) for s, _ in failed))
    tmp = LIB + ".tmp%d" % os.getpid()
    res = subprocess.run(link_command(objs, tmp), capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed linking %s" % LIB)
    os.replace(tmp, LIB)
    return LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in SOURCES + HEADERS)


if __name__ == "__main__":
    print(build(verbose=True))
