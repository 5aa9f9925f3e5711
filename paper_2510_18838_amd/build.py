"""Builds the HIP library libpcms_mls.so for gfx950 in-tree.

Every translation unit under csrc/ is compiled with hipcc in parallel and
linked into one shared library next to this file.  FP contraction is off
(the kernels write their fused multiply-adds explicitly) and packed FP32
instructions are disabled.
"""
from __future__ import annotations

import glob
import hashlib
import os
import re
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libpcms_mls.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
]


INCLUDE_DIRS = (os.path.join(HERE, "csrc"), os.path.join(ROOT, "include"))
CACHE = os.path.join(ROOT, "_build")


def _local_includes(path, seen):
    """Paths of the project headers `path` includes, recursively."""
    for name in re.findall(r'^\s*#\s*include\s+"([^"]+)"', open(path).read(), re.M):
        for d in (os.path.dirname(path),) + INCLUDE_DIRS:
            h = os.path.join(d, name)
            if os.path.exists(h):
                if h not in seen:
                    seen.add(h)
                    _local_includes(h, seen)
                break
    return seen


def _digest(src):
    h = hashlib.sha256(" ".join([HIPCC, *FLAGS]).encode())
    for f in [src] + sorted(_local_includes(src, set())):
        h.update(f.encode())
        h.update(open(f, "rb").read())
    return h.hexdigest()[:24]


def build(verbose: bool = False, jobs: int = 8, incremental: bool = False) -> str:
    """Compiles every translation unit and links the library.  With
    incremental=True, objects whose source and project headers are unchanged
    are reused from _build/ (a development convenience; the default compiles
    everything)."""
    srcs = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
    objdir = tempfile.mkdtemp(prefix="pcms_build_")
    objs, procs = [], []
    if incremental:
        os.makedirs(CACHE, exist_ok=True)
    for src in srcs:
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        objs.append(obj)
        if incremental:
            cached = os.path.join(CACHE, os.path.basename(src) + "." + _digest(src) + ".o")
            objs[-1] = obj = cached
            if os.path.exists(cached):
                continue
        cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        while sum(p.poll() is None for _, p in procs) >= jobs:
            procs[0][1].wait()
    failed = []
    for src, p in procs:
        out = p.communicate()[0].decode(errors="replace")
        if p.returncode != 0:
            failed.append((src, out))
        elif verbose and out.strip():
            print(out)
    if failed:
        msg = "\n".join(f"--- {s}\n{o}" for s, o in failed)
        raise RuntimeError(f"hipcc failed:\n{msg}")
    tmp = LIB + ".tmp"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    for o in objs:
        if not incremental:
            os.remove(o)
    os.rmdir(objdir)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="--incremental" in sys.argv))
