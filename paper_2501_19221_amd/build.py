"""Build libqpa.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2501_19221_amd.build            # incremental
    python -m paper_2501_19221_amd.build --force    # rebuild everything
    python -m paper_2501_19221_amd.build --sanitize # host code under AddressSanitizer and
                                                    # UndefinedBehaviorSanitizer, a separate
                                                    # copy in _build_san/libqpa_san.so
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libqpa.so")
OBJ_SAN = os.path.join(HERE, "_build_san")
LIB_SAN = os.path.join(OBJ_SAN, "libqpa_san.so")
# host side only (the device code is not instrumented): the sanitizer runtime is preloaded
# by whoever loads the copy
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]
HEADERS = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")) + \
    [os.path.join(os.path.dirname(HERE), "include", "qpa.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
CFLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-fPIC", "-std=c++17", "-ffp-contract=off",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _stale(obj, deps):
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(d) > t for d in deps)


def _compile(src, force, sanitize=False):
    obj = os.path.join(OBJ_SAN if sanitize else OBJ, os.path.basename(src)[:-4] + ".o")
    if force or _stale(obj, [src] + HEADERS):
        cmd = [HIPCC] + CFLAGS + (SAN_FLAGS if sanitize else []) + ["-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        err = "\n".join(ln for ln in (r.stdout + r.stderr).splitlines()
                        if "packed-fp32-ops' is not a recognized feature" not in ln)
        if r.returncode != 0:
            raise RuntimeError("hipcc failed for %s:\n%s" % (src, err))
        if err.strip():
            sys.stderr.write(err + "\n")
    return obj


def build(force: bool = False, jobs: int = 8, sanitize: bool = False) -> str:
    obj_dir, lib = (OBJ_SAN, LIB_SAN) if sanitize else (OBJ, LIB)
    os.makedirs(obj_dir, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(jobs, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, force, sanitize), srcs))
    if force or _stale(lib, objs):
        tmp = lib + ".tmp%d" % os.getpid()
        cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
        if sanitize:
            cmd[1:1] = ["-fsanitize=address", "-fsanitize=undefined", "-shared-libsan"]
        subprocess.check_call(cmd)
        os.replace(tmp, lib)
    return lib


def sanitizer_runtime() -> str:
    """Path of the compiler's AddressSanitizer runtime (to preload for a sanitized copy)."""
    out = subprocess.run([HIPCC, "--print-file-name=libclang_rt.asan-x86_64.so"],
                         capture_output=True, text=True).stdout.strip()
    return out


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--force", action="store_true")
    ap.add_argument("--sanitize", action="store_true")
    a = ap.parse_args()
    print(build(force=a.force, sanitize=a.sanitize))
