"""Builds and runs the CPU emulation of the HIP kernels (tests/emu/pcms_emu.cpp).

The emulation compiles the kernels' per-target code for the host with the
address and undefined-behaviour sanitisers, so indexing mistakes show up on
the CPU as sanitiser reports instead of GPU memory faults.
"""
from __future__ import annotations

import math
import os
import subprocess
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
EMU_DIR = os.path.join(HERE, "emu")
SRC = os.path.join(EMU_DIR, "pcms_emu.cpp")
EXE = os.path.join(EMU_DIR, "pcms_emu")
DEPS = [SRC, os.path.join(EMU_DIR, "emu_common.h"), os.path.join(EMU_DIR, "emu_dim.cpp")] + \
       [os.path.join(ROOT, "paper_2510_18838_amd", "csrc", f)
                for f in ("device_common.h", "search.h", "fit.h", "bvh.h")] + \
       [os.path.join(ROOT, "include", "pcms_mls.h")]


def build(force=False) -> str:
    """Compiles the emulator (the driver and one object per dimension, in
    parallel) unless it is newer than every source it depends on."""
    if (not force and os.path.exists(EXE)
            and os.path.getmtime(EXE) >= max(os.path.getmtime(d) for d in DEPS)):
        return EXE
    flags = ["g++", "-std=c++20", "-O1", "-pthread", "-g", "-fno-omit-frame-pointer",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
             "-DPCMS_HOST_EMULATION", "-I", os.path.join(ROOT, "include"),
             "-I", os.path.join(ROOT, "paper_2510_18838_amd", "csrc"), "-I", EMU_DIR]
    with tempfile.TemporaryDirectory() as d:
        jobs, objs = [], []
        for name, src, extra in [("main", SRC, [])] + [
                (f"d{k}", os.path.join(EMU_DIR, "emu_dim.cpp"), [f"-DPCMS_EMU_DIM={k}"])
                for k in range(1, 6)]:
            obj = os.path.join(d, name + ".o")
            objs.append(obj)
            jobs.append(subprocess.Popen(flags + extra + ["-c", src, "-o", obj]))
        if any(j.wait() != 0 for j in jobs):
            raise RuntimeError("emulator build failed")
        subprocess.check_call(flags + objs + ["-o", EXE + ".tmp"])
    os.replace(EXE + ".tmp", EXE)
    return EXE


def _cell_spec(prob):
    """Bucket sizing of a one-shot call (same rule as the library, including
    its PCMS_CELL_FACTOR override)."""
    env = os.environ.get("PCMS_CELL_FACTOR")
    cf = float(env) if env else (0.7 if prob.mode == 1 else 1.0)
    cf = cf if cf > 0 else 1.0
    if prob.mode == 1:
        d = prob.dim
        return 0.0, cf ** d * prob.k / (math.pi ** (d / 2) / math.gamma(d / 2 + 1))
    return cf * prob.radius, 0.0


def run(prob, op, precision=0, weight=0, lam=0.0, group=1, tgt=None, lbvh=False):
    """op 0: neighbour lists; op 1: transfer; op 2: transfer operator (shape
    functions, original target order); group: lanes per target (1, as
    in the kernels, or 4); lbvh: locate sources with the LBVH instead of the
    uniform grid (ops 0 and 1).  Returns a dict like the GPU helpers."""
    exe = build()
    t = prob.tgt if tgt is None else tgt
    n_src, dim = prob.src.shape
    n_tgt = t.shape[0]
    nf = prob.vals.shape[0]
    cw, ppc = _cell_spec(prob)
    g = np.ones(5)
    if prob.inv_scale is not None:
        g[:dim] = prob.inv_scale
    hdr = np.array([0x50434d53454d55, op | (0x10 if lbvh else 0), n_src, dim, n_tgt, nf, prob.degree, prob.mode, prob.k,
                    prob.n_min, prob.max_iter, prob.k_cap, weight, precision, group], np.int64)
    dbl = np.array([prob.radius, lam, cw, ppc, *g], np.float64)
    with tempfile.TemporaryDirectory() as d:
        fin, fout = os.path.join(d, "in.bin"), os.path.join(d, "out.bin")
        with open(fin, "wb") as fh:
            fh.write(hdr.tobytes())
            fh.write(dbl.tobytes())
            fh.write(np.ascontiguousarray(prob.src, np.float64).tobytes())
            fh.write(np.ascontiguousarray(prob.vals, np.float64).tobytes())
            fh.write(np.ascontiguousarray(t, np.float64).tobytes())
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        res = subprocess.run([exe, fin, fout], capture_output=True, text=True, env=env)
        if res.returncode != 0:
            raise RuntimeError(f"emulation failed ({res.returncode}):\n{res.stderr[-4000:]}")
        raw = open(fout, "rb").read()
        run.last_stderr = res.stderr
    off = 0

    def take(dtype, count):
        nonlocal off
        a = np.frombuffer(raw, dtype=dtype, count=count, offset=off)
        off += a.nbytes
        return a.copy()

    if op == 0:
        nbr = take(np.int32, n_tgt * prob.k_cap).reshape(n_tgt, prob.k_cap)
        n_kept = take(np.int32, n_tgt)
        n_found = take(np.int32, n_tgt)
        r2 = take(np.float64, n_tgt)
        st = take(np.uint8, n_tgt)
        return dict(nbr=nbr, n_kept=n_kept, n_found=n_found, r2=r2, status=st)
    if op == 2:
        n_kept = take(np.int32, n_tgt)
        cols = take(np.int32, n_tgt * prob.k_cap).reshape(n_tgt, prob.k_cap)
        w = take(np.float64, n_tgt * prob.k_cap).reshape(n_tgt, prob.k_cap)
        st = take(np.uint8, n_tgt)
        return dict(n_kept=n_kept, cols=cols, weights=w, status=st)
    out = take(np.float64, nf * n_tgt).reshape(nf, n_tgt)
    st = take(np.uint8, n_tgt)
    return dict(out=out, status=st)
