#!/usr/bin/env python3
"""Benchmark of the MLS point-cloud field transfer on one MI355X.

Metric: target points per second of the 3-D quadratic transfer (mixed
precision vs FP64) on the 4M x 4M Gaussian-mixture workload: 4*10^6 sources
(8-component mixture, 10x density contrast), 4*10^6 uniform targets,
quadratic basis (m = 10), radius = distance to the 40th nearest source,
neighbour cap 64, eight fields.  One step is one whole transfer: grid build,
target ordering, field gather, search, moment assembly, Cholesky solve and
evaluation, with inputs already resident in HBM.

Prints one JSON line with the contract's fields plus:
  roofline      the search-and-fit kernel (the dominant one): algorithmic
                flops per launch / its event-timed average duration, against
                the VALU peak (ALU-bound path)
  cpu_baseline  the FP64 CPU oracle timed on a bounded sample of the same
                workload on the host cores
  fp64          the same steps with the plain FP64 path, for the comparison
  accuracy      max relative error of the headline path vs FP64 (all
                targets) and vs the oracle (the sampled targets), and of the
                FP64 path vs the oracle
  statuses      per-target status counts of the headline run
  n_found_histogram  sources inside the radius, per target, over the first
                200k targets (a neighbour-list call outside the timed steps)
  cpu_baseline_1thread  the oracle on one host thread (smaller sample)
  operator, batched  the precomputed-operator and batched legs
  other_configs  the 2-D lattice, 5-D and small 2-D workloads, FP64 and
                MIXED_REFINE
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "target pts/sec, 3D quadratic MLS transfer: mixed vs FP64 at ≤1e-6 rel err"
# VALU peak: 256 CUs x 4 SIMD x 16 lanes x 2 flops (FMA) x 2.4 GHz.  FP32 and
# FP64 vector FMA issue at the same rate; packed FP32 is not used.
VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0
# Algorithmic cost per target of the search-and-fit kernel, per workload (the
# survey's cost model): flops = distinct-moment assembly + single-right-hand-
# side solve + exact FP64 distance tests of a one-radius bucket stencil; HBM
# bytes of a fused search-and-fit (no materialised lists) = 40 d + 12 +
# 24 n_f (sorted coordinates and FP32 records, targets, field records,
# outputs).
COST = {
    "c1": {"flops": 1200 + 27 + 400, "bytes": 40 * 2 + 12 + 24 * 1},
    "c2": {"flops": 4000 + 144 + 700, "bytes": 40 * 2 + 12 + 24 * 4},
    "c3": {"flops": 8100 + 530 + 2300, "bytes": 40 * 3 + 12 + 24 * 8},
    "c5": {"flops": 9700 + 144 + 44000, "bytes": 40 * 5 + 12 + 24 * 4},
}


def batch_alg_bytes(probs):
    """Fused-kernel bytes of the batched workload: the per-target figure
    40 d + 12 + 24 n_f split evenly between a problem's sources and targets
    (the two are equal in number in the other workloads)."""
    return sum((p.src.shape[0] + p.tgt.shape[0]) * (20 * p.dim + 6 + 12 * p.n_fields)
               for p in probs)


def roofline(name, n_tgt, kernel_ms, traffic=None, kernel="k_transfer"):
    """Both bounds of a search-and-fit launch: the VALU one (the binding one
    for these kernels) and the HBM one, from the algorithmic cost per target
    and the kernel's event-timed duration."""
    c = COST[name]
    tf = c["flops"] * n_tgt / (kernel_ms * 1e-3) / 1e12
    gbs = c["bytes"] * n_tgt / (kernel_ms * 1e-3) / 1e9
    r = {"bound": "alu", "kernel": kernel, "achieved": tf, "peak": VALU_PEAK_TFLOPS,
         "unit": "TFLOP/s", "frac": tf / VALU_PEAK_TFLOPS, "traffic": traffic,
         "alg_flops_per_target": c["flops"], "units_per_launch": int(n_tgt),
         "kernel_ms": kernel_ms,
         "hbm": {"achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": gbs / HBM_PEAK_GBS, "alg_bytes_per_target": c["bytes"]}}
    if traffic:
        r["hbm"]["counted_gbs"] = traffic / (kernel_ms * 1e-3) / 1e9
        r["hbm"]["counted_frac"] = r["hbm"]["counted_gbs"] / HBM_PEAK_GBS
    return r


def time_transfer(torch, pcms, p, src, vals, tgt, rad, precision, steps, warmup, out, st,
                  summary, lbvh=False):
    """K one-shot transfers enqueued back to back (PCMS_ASYNC, statuses into a
    device summary), bracketed by device synchronisations: ms per step from
    the host clock over the K steps and each step's duration from HIP events
    recorded on the launch stream (median, min).  Then the same K steps with
    PCMS_PROFILE for the phases' HIP-event times inside the library
    (averaged): a profiled call runs its phases one after the other, while
    the timed calls order the targets beside the grid build and field
    gather, so the phases of the profiled steps add up to a little more than
    the timed step.  lbvh: each step builds an LBVH instead of the grid."""
    extra = pcms.LBVH if lbvh else 0
    o = pcms.opts(precision=precision, flags=pcms.ASYNC | extra, summary=summary)
    op = pcms.opts(precision=precision, flags=pcms.PROFILE | pcms.ASYNC | extra, summary=summary)

    def call(opts):
        pcms.pcms_mls_transfer(src, vals, tgt, p.degree, rad, p.k_cap, inv_scale=p.inv_scale,
                               o=opts, out=out, status=st)
    for _ in range(warmup):
        call(o)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    t0 = time.perf_counter()
    for e0, e1 in ev:
        e0.record()
        call(o)
        e1.record()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    per = sorted(e0.elapsed_time(e1) for e0, e1 in ev)
    pcms.phase_ms_sum(reset=True)
    for _ in range(steps):
        call(op)
    torch.cuda.synchronize()
    calls, sums = pcms.phase_ms_sum(reset=True)
    phases = {k: v / max(calls, 1) for k, v in sums.items()}
    return {"ms_per_step": ms, "ms_median": float(np.median(per)), "ms_min": float(per[0]),
            "phases_ms": phases}


def lbvh_leg(torch, pcms, p, name, src, vals, tgt, rad, precision, label, steps, summary,
             grid_row, grid_out):
    """The same one-shot transfer on the LBVH search backend: timing, phases
    and roofline like the grid's, the speed ratio to the grid, and the
    agreement with the grid's outputs (statuses identical, values to
    rounding)."""
    m = tgt.shape[0]
    out = torch.empty((p.n_fields, m), dtype=torch.float64, device=tgt.device)
    st = torch.empty(m, dtype=torch.uint8, device=tgt.device)
    t = time_transfer(torch, pcms, p, src, vals, tgt, rad, precision, steps, 2, out, st, summary,
                      lbvh=True)
    t["value"] = m / (t["ms_per_step"] * 1e-3)
    t["roofline"] = roofline(name, m, t["phases_ms"]["search_fit"],
                             load_traffic(f"{name}_lbvh_{label}", source_digest()))
    t["speedup_vs_grid"] = grid_row["ms_per_step"] / t["ms_per_step"]
    g_out, g_st = grid_out
    b_out, b_st = out.cpu().numpy(), st.cpu().numpy()
    t["statuses_equal_grid"] = bool(np.array_equal(g_st, b_st))
    ok = ((g_st & 0xF) == 0) & (g_st == b_st)
    diff = 0.0
    for l in range(p.n_fields):
        ref = g_out[l][ok]
        if ref.size:
            diff = max(diff, float(np.abs(b_out[l][ok] - ref).max() / np.abs(ref).max()))
    t["max_rel_diff_vs_grid"] = diff
    log(f"{name} {label} on the LBVH: {t['ms_per_step']:.3f} ms/step "
        f"({t['speedup_vs_grid']:.2f}x the grid), phases {t['phases_ms']}")
    return t


def oracle_error(orc, p, out, st, n_sample, seed):
    """Max over fields of the inf-norm error against the oracle over the
    valid targets of a seeded sample (the accuracy gate's measure)."""
    rng = np.random.default_rng(seed)
    m = p.tgt.shape[0]
    idx = np.sort(rng.choice(m, size=min(n_sample, m), replace=False))
    ref = orc.transfer(p.src, p.vals, p.tgt[idx], p.degree, **orc.problem_kwargs(p))
    got = out[:, idx]
    ok = ((ref["status"] & 0xF) == 0) & (st[idx] == ref["status"])
    if not ok.any():
        return None, 0
    err = max(float(np.abs(got[l, ok] - ref["out"][l, ok]).max() /
                    np.abs(ref["out"][l, ok]).max()) for l in range(p.n_fields))
    return err, int(ok.sum())


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_digest():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2510_18838_amd", "csrc")
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def load_traffic(name, kernel_digest):
    """HBM bytes per launch of the workload's search-and-fit kernel from the
    committed counter summary (FETCH_SIZE + WRITE_SIZE, calibrated), if it
    was taken on the current kernel sources; else None."""
    p = os.path.join(ROOT, "profiles", f"traffic_{name}.json")
    if not os.path.exists(p):
        return None
    with open(p) as fh:
        t = json.load(fh)
    if t.get("source_digest") != kernel_digest:
        return None
    return t.get("bytes_per_launch")


def operator_leg(torch, pcms, p, src, tgt, vals, rad, steps, dev):
    """The precomputed transfer operator of the same workload: built once
    (MIXED_REFINE), then applied to the 8 fields per step -- the coupling
    pattern of fixed clouds exchanging new fields.  The apply kernel is HBM
    bound: its roofline counts the operator's 12 bytes per kept source, the
    per-target count and order (8 bytes), the field values read once and the
    outputs written once."""
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        t0 = time.perf_counter()
        op = pcms.Operator(src, tgt, p.degree, rad, p.k_cap, o=pcms.opts(precision=pcms.MIXED_REFINE),
                           stream=stream)
        stream.synchronize()
        build_ms = (time.perf_counter() - t0) * 1e3
        n_kept, _, _ = op.export(stream=stream)
        kept = int(n_kept.clamp_min(0).sum())
        out = torch.empty((p.n_fields, tgt.shape[0]), dtype=torch.float64, device=dev)
        op.apply(vals, out=out, stream=stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            op.apply(vals, out=out, stream=stream)
        e1.record(stream)
        e1.synchronize()
    ms = e0.elapsed_time(e1) / steps
    m, n_src, nf = tgt.shape[0], src.shape[0], p.n_fields
    alg_bytes = kept * 12 + m * 8 + n_src * nf * 8 + m * nf * 8
    achieved = alg_bytes / (ms * 1e-3) / 1e9
    log(f"operator: build {build_ms:.2f} ms, width {op.width}, apply {ms:.3f} ms "
        f"({achieved:.0f} GB/s algorithmic)")
    op.free()
    return {
        "build_ms": build_ms, "apply_ms": ms, "apply_value": m / (ms * 1e-3),
        "unit": "target pts/s (apply, 8 fields)", "width": op.width, "kept_total": kept,
        "roofline": {"bound": "hbm", "kernel": "k_op_apply", "achieved": achieved,
                     "peak": 8000.0, "unit": "GB/s", "frac": achieved / 8000.0,
                     "traffic": load_traffic("c3_op_apply", source_digest()),
                     "alg_bytes_per_launch": alg_bytes},
    }


ROUNDTRIP_LAMBDAS = (1e-8, 1e-6, 1e-4, 1e-2, 1.0)


def roundtrip(torch, pcms, synth, dev, iters=(1, 2, 5, 10, 20, 50, 100)):
    """The paper's round-trip accuracy protocol on point clouds: the field of
    Eq. 4 on ~307k jittered-lattice points (the vertex count of the paper's
    mesh) mapped to ~611k points (its element count) and back, repeatedly,
    with the C4 weight, linear and quadratic bases and three cut-off radii
    (in units of the source spacing h); the accuracy error of Eq. 2 (L2
    norm over the source points) after each iteration.  Both transfer
    operators are built once and applied per iteration.  A sweep of the
    Tikhonov parameter of Eq. 1 (lambda, in the radius-scaled basis) follows
    for the quadratic fits at 2.5h and 3.5h and the linear fit at 3.5h."""
    src, tgt, f = synth.roundtrip_clouds()
    h = 4.0 / 554
    s_d, t_d = torch.from_numpy(src).to(dev), torch.from_numpy(tgt).to(dev)
    fd = torch.from_numpy(f[None, :]).to(dev)
    rows = []
    cases = [(d, rr, 0.0) for d in (1, 2) for rr in (2.5, 3.5, 5.0)]
    cases += [(d, rr, lam) for d, rr in ((2, 2.5), (2, 3.5), (1, 3.5)) for lam in ROUNDTRIP_LAMBDAS]
    for degree, rr, lam in cases:
        rad = pcms.radius(pcms.RADIUS_FIXED, r=rr * h)
        o = pcms.opts(precision=pcms.FP64, weight=pcms.WEIGHT_C4, lam=lam)
        t0 = time.perf_counter()
        fwd = pcms.Operator(s_d, t_d, degree, rad, 128, o=o)
        back = pcms.Operator(t_d, s_d, degree, rad, 128, o=o)
        torch.cuda.synchronize()
        build = (time.perf_counter() - t0) * 1e3
        g = fd
        ok = torch.isfinite(back.apply(fwd.apply(g)))[0]
        err, t0 = {}, time.perf_counter()
        for it in range(1, max(iters) + 1):
            g = back.apply(fwd.apply(g))
            if it in iters:
                d = (g[0] - fd[0])[ok]
                err[it] = float(torch.linalg.norm(d) / torch.linalg.norm(fd[0][ok]))
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / max(iters)
        log(f"round trip degree {degree} r={rr}h lambda={lam:g}: " +
            " ".join(f"{k}:{v:.2e}" for k, v in err.items()))
        rows.append({"degree": degree, "radius_h": rr, "lambda": lam, "accuracy_error": err,
                     "build_ms": build, "ms_per_iteration": ms})
        fwd.free()
        back.free()
    return {"experiment": "round trip, Eq. 4 field, 2-D point clouds", "n_src": int(src.shape[0]),
            "n_tgt": int(tgt.shape[0]), "weight": "C4", "rows": rows}


def timed_graph(torch, plan, stream, steps, summary):
    """Replays of a captured plan: per-replay HIP-event durations on the
    launch stream (median, min) and the mean over the K replays."""
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    with torch.cuda.stream(stream):
        for _ in range(2):          # capture, then one replay
            plan.exec(stream=stream, summary=summary)
        stream.synchronize()
        for e0, e1 in ev:
            e0.record(stream)
            plan.exec(stream=stream, summary=summary)
            e1.record(stream)
        stream.synchronize()
    per = sorted(e0.elapsed_time(e1) for e0, e1 in ev)
    return float(np.mean(per)), float(np.median(per)), float(per[0])


def batched_leg(torch, pcms, synth, dev, steps, orc=None):
    """512 transfer problems of uneven size (1k-200k points, log-uniform),
    2-D/3-D, linear/quadratic, 1-16 fields, growing radius: the batched plan
    (MIXED_REFINE, every stage captured once into a HIP graph and replayed,
    one search-and-fit launch per class of problems, knobs from the
    autotuner) against the same problems through the one-problem FP64 path,
    one call after another."""
    import tempfile
    t0 = time.time()
    probs = synth.c4()
    n_tgt = sum(p.tgt.shape[0] for p in probs)
    log(f"batched workload generated in {time.time() - t0:.1f}s: {len(probs)} problems, "
        f"{n_tgt} targets")
    bps = [pcms.batch_problem_of(p, dev) for p in probs]
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    with tempfile.TemporaryDirectory() as d:
        cache = os.path.join(d, "tune.json")
        t0 = time.time()
        tune = pcms.pcms_autotune(bps[::8], pcms.batch_opts(precision=pcms.MIXED_REFINE),
                                  cache_path=cache, stream=stream)
        log(f"autotune ({len(bps[::8])} problems) {time.time() - t0:.1f}s: block {tune.block} "
            f"cell factor {tune.cell_factor}")
        plan = pcms.BatchPlan(bps, pcms.batch_opts(precision=pcms.MIXED_REFINE, tune_cache=cache))
    summary = torch.zeros(4, dtype=torch.int32, device=dev)
    ms_b, med_b, min_b = timed_graph(torch, plan, stream, steps, summary)
    log(f"batched MIXED_REFINE: {ms_b:.3f} ms per batch (median {med_b:.3f}, min {min_b:.3f})")
    outs_b = [bp.out.clone() for bp in bps]
    st_b = [bp.status.clone() for bp in bps]
    # the same batch in FP64 (same knobs), for the precision comparison
    plan64 = pcms.BatchPlan(bps, pcms.batch_opts(precision=pcms.FP64, block=int(tune.block),
                                                 cell_factor=float(tune.cell_factor)))
    ms_b64, med_b64, min_b64 = timed_graph(torch, plan64, stream, steps, summary)
    plan64.free()
    log(f"batched FP64: {ms_b64:.3f} ms per batch")
    # the same problems through the one-problem FP64 path
    o64 = pcms.opts(precision=pcms.FP64)

    def unbatched():
        for bp in bps:
            pcms.pcms_mls_transfer(bp.src, bp.src_vals, bp.tgt, bp.basis_degree, bp.rad, bp.k_cap,
                                   inv_scale=bp.inv_scale, o=o64, out=bp.out, status=bp.status)
    unbatched()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    unbatched()
    torch.cuda.synchronize()
    ms_u = (time.perf_counter() - t0) * 1e3
    log(f"one-problem FP64, {len(bps)} calls: {ms_u:.3f} ms")
    err = 0.0
    for q, bp in enumerate(bps):
        ok = ((bp.status & 0xF) == 0) & (st_b[q] == bp.status)
        if int(ok.sum()) == 0:
            continue
        ref = bp.out[:, ok]
        err = max(err, float(((outs_b[q][:, ok] - ref).abs().amax(dim=1) /
                              ref.abs().amax(dim=1).clamp_min(1e-300)).max()))
    plan.free()
    oerr = None
    if orc is not None:
        # MIXED_REFINE against the oracle on 300 targets of each of 16 problems
        rng = np.random.default_rng(44)
        oerr = 0.0
        for q in sorted(rng.choice(len(probs), size=16, replace=False)):
            e, _ = oracle_error(orc, probs[q], outs_b[q].cpu().numpy(), st_b[q].cpu().numpy(),
                                n_sample=300, seed=int(q))
            if e is not None:
                oerr = max(oerr, e)
    alg = batch_alg_bytes(probs)
    gbs = alg / (med_b * 1e-3) / 1e9
    traffic = load_traffic("c4_batch_mixed_refine", source_digest())
    return {
        "workload": "512 problems: n_src, n_tgt log-uniform in [1e3, 2e5], d in {2, 3}, degree "
                    "in {1, 2}, 1-16 fields, growing radius, k_cap 32-64",
        "n_problems": len(bps), "n_tgt": int(n_tgt),
        "mixed_refine_batched": {"ms": ms_b, "ms_median": med_b, "ms_min": min_b,
                                 "value": n_tgt / (ms_b / 1e3), "unit": "target pts/s",
                                 "launch": "HIP graph replay, one kernel per class",
                                 "max_rel_err_vs_oracle_sample": oerr},
        "roofline": {"bound": "hbm", "kernel": "one graph replay (grid builds, target order, "
                     "field records, one k_batch_transfer launch per class)", "achieved": gbs,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                     "traffic": traffic, "traffic_scope": "the class kernels of one replay",
                     "alg_bytes_per_launch": alg, "launch_ms_median": med_b},
        "fp64_batched": {"ms": ms_b64, "ms_median": med_b64, "ms_min": min_b64,
                         "value": n_tgt / (ms_b64 / 1e3), "unit": "target pts/s",
                         "launch": "the same plan in FP64"},
        "fp64_unbatched": {"ms": ms_u, "value": n_tgt / (ms_u / 1e3), "unit": "target pts/s",
                           "launch": "one one-shot call per problem"},
        "speedup": ms_u / ms_b,
        "max_rel_err_vs_fp64": err,
        "tune": {"block": int(tune.block), "cell_factor": float(tune.cell_factor),
                 "sample_ms": float(tune.ms)},
    }


def configs_leg(torch, pcms, synth, dev, steps, orc=None, lbvh=True):
    """The other single-GPU workloads: the 2-D lattice transfer (1M -> 1M,
    quadratic, fixed radius 3.5 cells, 4 fields), the 5-D transfer (2M -> 2M,
    linear, growing radius in a standardising metric, 4 fields) and the small
    2-D correctness case (2k -> 1.5k, linear, fixed radius): one-shot steps in
    FP64 and MIXED_REFINE timed like the headline, each precision's roofline
    from its search-and-fit kernel's event time, the mixed path's error
    against FP64 (all targets) and both against the oracle on a sample.  The
    5-D transfer is also timed on the LBVH search backend."""
    rows = {}
    digest = source_digest()
    summary = torch.zeros(4, dtype=torch.int32, device=dev)
    for name, make in (("c1", synth.c1), ("c2", synth.c2), ("c5", synth.c5)):
        p = make()
        src, vals, tgt = (torch.from_numpy(x).to(dev) for x in (p.src, p.vals, p.tgt))
        m = tgt.shape[0]
        rad = pcms.radius_of(p)
        row = {"n_src": int(p.src.shape[0]), "n_tgt": int(m), "dim": p.dim,
               "basis_degree": p.degree, "n_fields": p.n_fields}
        outs = {}
        for label, prec in (("fp64", pcms.FP64), ("mixed_refine", pcms.MIXED_REFINE)):
            out = torch.empty((p.n_fields, m), dtype=torch.float64, device=dev)
            st = torch.empty(m, dtype=torch.uint8, device=dev)
            t = time_transfer(torch, pcms, p, src, vals, tgt, rad, prec, steps, 2, out, st,
                              summary)
            t["value"] = m / (t["ms_per_step"] * 1e-3)
            kname = f"{name}_{label}"
            t["roofline"] = roofline(name, m, t["phases_ms"]["search_fit"],
                                     load_traffic(kname, digest))
            row[label] = t
            outs[label] = (out.cpu().numpy(), st.cpu().numpy())
        ok = (outs["fp64"][1] & 0xF) == 0
        ok &= outs["fp64"][1] == outs["mixed_refine"][1]
        err = 0.0
        for l in range(p.n_fields):
            ref = outs["fp64"][0][l][ok]
            err = max(err, float(np.abs(outs["mixed_refine"][0][l][ok] - ref).max() /
                                 np.abs(ref).max()))
        row["mixed_refine_max_rel_err_vs_fp64"] = err
        row["mixed_speedup"] = row["fp64"]["ms_per_step"] / row["mixed_refine"]["ms_per_step"]
        row["valid_targets"] = int(ok.sum())
        if name == "c5" and lbvh:
            row["lbvh"] = {label: lbvh_leg(torch, pcms, p, name, src, vals, tgt, rad, prec, label,
                                           steps, summary, row[label], outs[label])
                           for label, prec in (("fp64", pcms.FP64),
                                               ("mixed_refine", pcms.MIXED_REFINE))}
        if orc is not None:
            for label in ("fp64", "mixed_refine"):
                e, n_ok = oracle_error(orc, p, *outs[label], n_sample=2000, seed=7)
                row[label]["max_rel_err_vs_oracle_sample"] = e
                row[label]["oracle_sample_valid"] = n_ok
        log(f"{name}: fp64 {row['fp64']['ms_per_step']:.3f} ms, mixed_refine "
            f"{row['mixed_refine']['ms_per_step']:.3f} ms, err vs fp64 {err:.2e}")
        rows[name] = row
        del src, vals, tgt, outs
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", choices=["mixed", "mixed_refine", "fp64"], default="mixed_refine")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison leg")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--scale", type=float, default=1.0, help="shrink the workload (profiling aid)")
    ap.add_argument("--no-operator", action="store_true",
                    help="skip the precomputed-operator leg")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched leg (512 uneven problems, one graph replay)")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other single-GPU workloads (2-D lattice, 5-D, small 2-D)")
    ap.add_argument("--no-lbvh", action="store_true",
                    help="skip the LBVH search-backend legs")
    ap.add_argument("--roundtrip", action="store_true",
                    help="only run the round-trip accuracy experiment (source -> target -> "
                         "source iterations of the Eq. 4 field) and print its table as JSON")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a plain device-to-device copy of this many bytes three times "
                         "(calibrates the HBM byte counters against a known traffic)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(see the design notes for how the transfer would shard)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2510_18838_amd import pcms, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_bytes:
        n = args.copy_bytes // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copied {8 * n} bytes three times")
        return
    pcms.lib()
    dev = torch.device("cuda:0")
    if args.roundtrip:
        print(json.dumps(roundtrip(torch, pcms, synth, dev)), flush=True)
        return
    n = int(4_000_000 * args.scale)
    t0 = time.time()
    p = synth.c3(n_src=n)
    log(f"workload generated in {time.time() - t0:.1f}s: n_src={p.src.shape[0]} "
        f"n_tgt={p.tgt.shape[0]} fields={p.n_fields}")
    src = torch.from_numpy(p.src).to(dev)
    vals = torch.from_numpy(p.vals).to(dev)
    tgt = torch.from_numpy(p.tgt).to(dev)
    M = tgt.shape[0]
    out = torch.empty((p.n_fields, M), dtype=torch.float64, device=dev)
    st = torch.empty(M, dtype=torch.uint8, device=dev)
    rad = pcms.radius_of(p)
    prec = {"mixed": pcms.MIXED, "mixed_refine": pcms.MIXED_REFINE, "fp64": pcms.FP64}[args.precision]

    summary = torch.zeros(4, dtype=torch.int32, device=dev)
    log(f"timing {args.steps} steps ({args.warmup} warm-up), precision {args.precision}")
    head = time_transfer(torch, pcms, p, src, vals, tgt, rad, prec, args.steps, args.warmup, out,
                         st, summary)
    ms, phases = head["ms_per_step"], head["phases_ms"]
    log(f"{ms:.3f} ms/step (event median {head['ms_median']:.3f}, min {head['ms_min']:.3f}), "
        f"phases {phases}")
    value = M / (ms / 1e3)
    head_out = out.clone()
    status = st.cpu().numpy()
    out64 = None

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "target pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == pcms.FP64 else "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": "3-D quadratic MLS transfer, 4M Gaussian-mixture sources (10x density "
                        "contrast) -> 4M uniform targets, kNN-40 radius, k_cap 64, 8 fields",
            "n_src": int(p.src.shape[0]), "n_tgt": int(M), "basis_degree": p.degree,
            "n_fields": p.n_fields, "precision": args.precision,
        },
        "step_ms_event": {"median": head["ms_median"], "min": head["ms_min"]},
        "phases_ms": phases,
        "statuses": {"ok": int(((status & 0xF) == 0).sum()),
                     "underdetermined": int(((status & 0xF) == 1).sum()),
                     "singular": int(((status & 0xF) == 2).sum()),
                     "radius_exhausted": int(((status & 0xF) == 3).sum()),
                     "capped": int(((status & 0x10) != 0).sum())},
    }
    result["roofline"] = roofline("c3", M, phases["search_fit"],
                                  load_traffic(f"c3_{args.precision}", source_digest()))

    if not args.no_fp64 and prec != pcms.FP64:
        out64 = torch.empty_like(out)
        t64 = time_transfer(torch, pcms, p, src, vals, tgt, rad, pcms.FP64, args.steps, 1, out64,
                            st, summary)
        ms64, ph64 = t64["ms_per_step"], t64["phases_ms"]
        ok = torch.from_numpy((status & 0xF) == 0).to(dev)
        err = 0.0
        for l in range(p.n_fields):
            ref = out64[l][ok]
            err = max(err, float((head_out[l][ok] - ref).abs().max() / ref.abs().max()))
        result["fp64"] = {"value": M / (ms64 / 1e3), "ms_per_step": ms64, "phases_ms": ph64,
                          "step_ms_event": {"median": t64["ms_median"], "min": t64["ms_min"]},
                          "mixed_speedup": ms64 / ms,
                          "roofline": roofline("c3", M, ph64["search_fit"],
                                               load_traffic("c3_fp64", source_digest()))}
        result["accuracy"] = {"max_rel_err_vs_fp64_all_targets": err}
        log(f"fp64 {ms64:.3f} ms/step; headline vs fp64 max rel err {err:.3e}")

    if not args.no_lbvh:
        result["lbvh"] = lbvh_leg(torch, pcms, p, "c3", src, vals, tgt, rad, prec, args.precision,
                                  args.steps, summary, head, (head_out.cpu().numpy(), status))

    # kept-source counts of a 200k-target subset (outside the timed region)
    sub = tgt[:min(M, 200000)].contiguous()
    grid = pcms.pcms_grid_build(src, pts_per_cell=0.7 ** 3 * p.k / (4.0 * np.pi / 3.0))
    nb = pcms.pcms_neighbors(grid, sub, rad, p.k_cap)
    torch.cuda.synchronize()
    counts = np.bincount(nb["n_found"].cpu().numpy().clip(0, 4 * p.k_cap))
    result["n_found_histogram"] = {"targets": int(sub.shape[0]),
                                   "counts": {str(i): int(c) for i, c in enumerate(counts) if c}}
    grid.free()
    del nb

    if not args.no_cpu:
        import oracle
        threads = oracle.max_threads()
        # size the sample from a short probe so the timed CPU leg takes ~cpu_seconds
        probe = min(20000, M)
        t0 = time.time()
        oracle.transfer(p.src, p.vals, p.tgt[:probe], p.degree, **oracle.problem_kwargs(p))
        rate = probe / max(time.time() - t0, 1e-3)
        sample = int(min(M, max(probe, rate * args.cpu_seconds)))
        t0 = time.time()
        ref = oracle.transfer(p.src, p.vals, p.tgt[:sample], p.degree, **oracle.problem_kwargs(p))
        dt = time.time() - t0
        result["cpu_baseline"] = {
            "value": sample / dt, "unit": "target pts/s", "cores": threads, "kind": "oracle",
            "sample": f"all {p.src.shape[0]} sources (its own grid build included), "
                      f"the first {sample} of {M} targets, FP64, {dt:.1f}s",
        }
        got = head_out[:, :sample].cpu().numpy()
        ok = ((ref["status"] & 0xF) == 0) & (status[:sample] == ref["status"])
        err = max(float(np.abs(got[l, ok] - ref["out"][l, ok]).max() / np.abs(ref["out"][l, ok]).max())
                  for l in range(p.n_fields))
        result.setdefault("accuracy", {})["max_rel_err_vs_oracle_sample"] = err
        if out64 is not None:
            g64 = out64[:, :sample].cpu().numpy()
            result["accuracy"]["fp64_max_rel_err_vs_oracle_sample"] = max(
                float(np.abs(g64[l, ok] - ref["out"][l, ok]).max() / np.abs(ref["out"][l, ok]).max())
                for l in range(p.n_fields))
        # the oracle on one thread, on a twentieth of the sample
        s1 = max(1000, sample // 20)
        t0 = time.time()
        oracle.transfer(p.src, p.vals, p.tgt[:s1], p.degree, nthreads=1, **oracle.problem_kwargs(p))
        dt1 = time.time() - t0
        result["cpu_baseline_1thread"] = {"value": s1 / dt1, "unit": "target pts/s", "cores": 1,
                                          "sample": f"the first {s1} targets, {dt1:.1f}s"}
        log(f"cpu oracle: {sample} targets in {dt:.1f}s on {threads} threads; "
            f"headline vs oracle max rel err {err:.3e}")

    if not args.no_operator:
        result["operator"] = operator_leg(torch, pcms, p, src, tgt, vals, rad, args.steps, dev)

    if not args.no_batch:
        del head_out, out
        orc_b = None
        if not args.no_cpu:
            import oracle as orc_b
        result["batched"] = batched_leg(torch, pcms, synth, dev, args.steps, orc_b)

    if not args.no_configs:
        orc = None
        if not args.no_cpu:
            import oracle as orc
        result["other_configs"] = configs_leg(torch, pcms, synth, dev, args.steps, orc,
                                              lbvh=not args.no_lbvh)

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
