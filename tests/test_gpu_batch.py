"""Batched transfer on the GPU: one plan over problems of uneven size,
dimension, degree, field count and radius mode, checked against the
one-problem path (bit-identical: the batch builds each problem's grid with
the same layout and runs the same per-target code) and against the oracle,
through graph capture and replays."""
import numpy as np
import pytest
import torch

import parity_cases as C
from gpu_helpers import DEV, gpu_transfer, say
from paper_2510_18838_amd import pcms, synth

pytestmark = pytest.mark.gpu


def batch_problems():
    probs = [synth.c4_problem(b, size_scale=0.04) for b in range(16)]
    # other dimensions and modes: 1-D kNN, 4-D and 5-D (one-problem kernel
    # inside the batch), an anisotropic metric, a fixed radius, no targets
    probs.append(synth.uniform_problem(41, 3000, 700, 1, 2, synth.KNN, n_fields=2, k=8, k_cap=16))
    probs.append(synth.uniform_problem(42, 4000, 600, 4, 1, synth.GROW, n_fields=3, radius=0.15,
                                       n_min=10, k_cap=24))
    probs.append(synth.uniform_problem(43, 9000, 400, 5, 1, synth.KNN, n_fields=2, k=15,
                                       k_cap=24))
    probs.append(synth.uniform_problem(44, 5000, 800, 3, 2, synth.KNN, n_fields=5, k=25,
                                       k_cap=32, inv_scale=[2.0, 1.0, 0.5]))
    probs.append(synth.uniform_problem(45, 5000, 900, 2, 1, synth.FIXED, n_fields=1,
                                       radius=0.04, k_cap=40))
    probs.append(synth.uniform_problem(46, 2000, 0, 3, 1, synth.KNN, n_fields=1, k=10, k_cap=16))
    return probs


class FromBatch:
    """Results of one problem of an executed batch, as a parity backend."""

    def __init__(self, bp):
        self.bp = bp

    def transfer(self, prob, precision, weight=0, lam=0.0):
        return dict(out=self.bp.out.cpu().numpy(), status=self.bp.status.cpu().numpy())


def run_batch(probs, precision, **kw):
    bps = [pcms.batch_problem_of(p, DEV) for p in probs]
    plan = pcms.BatchPlan(bps, pcms.batch_opts(precision=precision, **kw))
    return plan, bps


@pytest.mark.parametrize("precision", [pcms.FP64, pcms.MIXED_REFINE])
def test_batch_matches_one_problem_path(precision):
    probs = batch_problems()
    say(f"batch of {len(probs)} problems, precision {precision}")
    plan, bps = run_batch(probs, precision)
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan.exec(stream=stream)
    torch.cuda.synchronize()
    for q, (p, bp) in enumerate(zip(probs, bps)):
        if p.tgt.shape[0] == 0:
            continue
        out, st, _ = gpu_transfer(p, precision)
        got, gst = bp.out.cpu().numpy(), bp.status.cpu().numpy()
        assert (gst == st).all(), f"problem {q}: statuses differ"
        both = np.isnan(out) & np.isnan(got)
        assert ((got == out) | both).all(), f"problem {q}: values differ from the one-problem path"
    plan.free()


def test_batch_against_oracle():
    probs = batch_problems()
    plan, bps = run_batch(probs, pcms.MIXED_REFINE)
    plan.exec(stream=torch.cuda.current_stream())
    torch.cuda.synchronize()

    for q in (0, 3, 7, 16, 17, 18, 19, 20):
        p = probs[q]
        say(f"problem {q}: d={p.dim} p={p.degree} nf={p.n_fields} n_src={p.src.shape[0]} "
            f"n_tgt={p.tgt.shape[0]}")
        C.check_transfer(FromBatch(bps[q]), p, f"batch[{q}]", precisions=(pcms.MIXED_REFINE,))
    plan.free()


def test_batch_graph_replays_and_new_values():
    """Replays of the captured graph give the same values; new source values
    written into the same buffers are picked up (the fit is linear in them,
    and doubling is exact)."""
    probs = [synth.c4_problem(b, size_scale=0.03) for b in range(6)]
    plan, bps = run_batch(probs, pcms.FP64)
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan.exec(stream=stream)
        first = [bp.out.clone() for bp in bps]
        for rep in range(3):
            torch.cuda.synchronize()
            plan.exec(stream=stream)
            torch.cuda.synchronize()
            for q, bp in enumerate(bps):
                assert torch.equal(bp.out.nan_to_num(7.0), first[q].nan_to_num(7.0)), \
                    f"replay {rep}: problem {q} changed"
        for bp in bps:
            bp.src_vals.mul_(2.0)
        torch.cuda.synchronize()
        plan.exec(stream=stream)
    torch.cuda.synchronize()
    for q, bp in enumerate(bps):
        assert torch.equal(bp.out.nan_to_num(7.0), (2.0 * first[q]).nan_to_num(7.0)), \
            f"problem {q}: new values not picked up"
    plan.free()


def test_batch_async_summary_counts_statuses():
    probs = batch_problems()
    plan, bps = run_batch(probs, pcms.MIXED_REFINE)
    summary = torch.full((4,), -1, dtype=torch.int32, device=DEV)
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        code = plan.exec(stream=stream, summary=summary)
    torch.cuda.synchronize()
    assert code == pcms.PCMS_OK
    st = np.concatenate([bp.status.cpu().numpy() for bp in bps])
    want = [int(((st & 0xF) == 1).sum()), int(((st & 0xF) == 2).sum()),
            int(((st & 0xF) == 3).sum()), int(((st & 0x10) != 0).sum())]
    assert summary.cpu().tolist() == want
    plan.free()


def test_autotune_picks_a_setting_and_caches_it(tmp_path):
    probs = [synth.c4_problem(b, size_scale=0.02) for b in range(4)]
    bps = [pcms.batch_problem_of(p, DEV) for p in probs]
    path = str(tmp_path / "tune.json")
    res = pcms.pcms_autotune(bps, pcms.batch_opts(precision=pcms.MIXED_REFINE), cache_path=path)
    say(f"autotune: block {res.block} cell factor {res.cell_factor} {res.ms:.3f} ms")
    assert res.block in (64, 128, 256) and res.cell_factor in (0.6, 0.7, 0.85, 1.0)
    assert res.ms > 0
    text = open(path).read()
    assert f'"block": {res.block}' in text
    plan = pcms.BatchPlan(bps, pcms.batch_opts(precision=pcms.MIXED_REFINE, tune_cache=path))
    plan.exec(stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    # another cell size changes only the order of the sums: same bar against the oracle
    for q, (p, bp) in enumerate(zip(probs, bps)):
        C.check_transfer(FromBatch(bp), p, f"tuned[{q}]", precisions=(pcms.MIXED_REFINE,))
    plan.free()
