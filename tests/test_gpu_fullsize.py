"""Parity at the workloads' full sizes, in the launch configuration bench.py
times (one-shot transfer, library block and cell choices; the batched plan
with autotuned knobs): every target runs on the GPU, and a seeded sample of
targets is checked against the FP64 oracle (which computes those targets one
by one over all sources) to the same bars as the small cases -- neighbour
lists, counts, radii and statuses bit-exact, values within the precision's
tolerance plus the conditioning term.  Properties that hold at any size are
checked on every target."""
import numpy as np
import pytest
import torch

import parity_cases as C
from gpu_helpers import DEV, dev, gpu_neighbors, say
from paper_2510_18838_amd import pcms, synth

pytestmark = pytest.mark.gpu


class Sampled:
    """Backend returning precomputed full-size GPU results at sampled rows."""

    def __init__(self, results, idx):
        self.results, self.idx = results, idx

    def transfer(self, prob, precision, weight=0, lam=0.0):
        out, st = self.results[precision]
        return dict(out=out[:, self.idx], status=st[self.idx])


def full_transfer(prob, precision, lbvh=False):
    src, vals, tgt = dev(prob.src), dev(prob.vals), dev(prob.tgt)
    out, st, _ = pcms.pcms_mls_transfer(src, vals, tgt, prob.degree, pcms.radius_of(prob),
                                        prob.k_cap, inv_scale=prob.inv_scale,
                                        o=pcms.opts(precision=precision,
                                                    flags=pcms.LBVH if lbvh else 0))
    torch.cuda.synchronize()
    return out.cpu().numpy(), st.cpu().numpy()


def check_everywhere(out, st, where):
    """Any-size properties: known status codes, finite values exactly where
    the status is OK (with or without the cap bit), NaN elsewhere."""
    assert np.isin(st & 0xF, (0, 1, 2, 3)).all() and not (st & 0xE0).any(), where
    ok = (st & 0xF) == 0
    assert np.isfinite(out[:, ok]).all(), f"{where}: non-finite values at valid targets"
    assert np.isnan(out[:, ~ok]).all(), f"{where}: failed targets not NaN"


def run_full(prob, precisions, n_sample, n_lists, seed, lbvh=False):
    say(f"{prob.name}{' on the LBVH' if lbvh else ''}: n_src={prob.src.shape[0]} "
        f"n_tgt={prob.tgt.shape[0]} d={prob.dim} p={prob.degree} nf={prob.n_fields}")
    results = {}
    for prec in precisions:
        out, st = full_transfer(prob, prec, lbvh)
        check_everywhere(out, st, f"{prob.name} precision {prec}")
        results[prec] = (out, st)
        say(f"  precision {prec}: {int(((st & 0xF) == 0).sum())} valid targets, "
            f"{int(((st & 0x10) != 0).sum())} capped")
    rng = np.random.default_rng(seed)
    m = prob.tgt.shape[0]
    idx = np.sort(rng.choice(m, size=min(n_sample, m), replace=False))
    sub = C.custom(prob.src, prob.vals, prob.tgt[idx], prob.degree, prob.mode, radius=prob.radius,
                   k=prob.k, n_min=prob.n_min, max_iter=prob.max_iter, k_cap=prob.k_cap,
                   inv_scale=prob.inv_scale)
    C.check_transfer(Sampled(results, idx), sub, f"{prob.name} full, {len(idx)} sampled",
                     precisions=precisions)
    rows = idx[:n_lists]
    sub_l = C.custom(prob.src, prob.vals, prob.tgt[rows], prob.degree, prob.mode,
                     radius=prob.radius, k=prob.k, n_min=prob.n_min, max_iter=prob.max_iter,
                     k_cap=prob.k_cap, inv_scale=prob.inv_scale)

    class Lists:
        def neighbors(self, _):
            return gpu_neighbors(prob, rows=rows, lbvh=lbvh)

    C.check_lists(Lists(), sub_l, f"{prob.name} full lists, {len(rows)} sampled")


def test_full_c3_mixed_vs_fp64():
    run_full(synth.c3(), (pcms.MIXED_REFINE, pcms.FP64), n_sample=3000, n_lists=1500, seed=31)


def test_full_c2():
    run_full(synth.c2(), (pcms.FP64, pcms.MIXED_REFINE, pcms.MIXED), n_sample=3000, n_lists=1500,
             seed=32)


def test_full_c5():
    run_full(synth.c5(), (pcms.FP64, pcms.MIXED_REFINE), n_sample=1500, n_lists=800, seed=35)


def test_full_c5_lbvh():
    """The 5-D workload on the LBVH, in the configuration bench.py times for
    that backend."""
    run_full(synth.c5(), (pcms.FP64, pcms.MIXED_REFINE), n_sample=1500, n_lists=800, seed=36,
             lbvh=True)


def test_full_c3_lbvh():
    run_full(synth.c3(), (pcms.MIXED_REFINE,), n_sample=2000, n_lists=1000, seed=37, lbvh=True)


def test_full_batch_c4():
    """The whole 512-problem batch through one plan; sampled targets of
    sampled problems against the oracle."""
    probs = synth.c4()
    bps = [pcms.batch_problem_of(p, DEV) for p in probs]
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    tune = pcms.pcms_autotune(bps[::8], pcms.batch_opts(precision=pcms.MIXED_REFINE), stream=stream)
    plan = pcms.BatchPlan(bps, pcms.batch_opts(precision=pcms.MIXED_REFINE, block=tune.block,
                                               cell_factor=tune.cell_factor))
    with torch.cuda.stream(stream):
        plan.exec(stream=stream)
        plan.exec(stream=stream)      # a graph replay
    torch.cuda.synchronize()
    rng = np.random.default_rng(34)
    for q in sorted(rng.choice(len(probs), size=24, replace=False)):
        p, bp = probs[q], bps[q]
        out, st = bp.out.cpu().numpy(), bp.status.cpu().numpy()
        check_everywhere(out, st, f"c4[{q}]")
        m = p.tgt.shape[0]
        idx = np.sort(rng.choice(m, size=min(300, m), replace=False))
        sub = C.custom(p.src, p.vals, p.tgt[idx], p.degree, p.mode, radius=p.radius, k=p.k,
                       n_min=p.n_min, max_iter=p.max_iter, k_cap=p.k_cap, inv_scale=p.inv_scale)
        C.check_transfer(Sampled({pcms.MIXED_REFINE: (out, st)}, idx), sub,
                         f"c4[{q}] d={p.dim} p={p.degree} nf={p.n_fields} n_tgt={m}",
                         precisions=(pcms.MIXED_REFINE,))
    plan.free()
