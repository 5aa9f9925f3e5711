"""The precomputed transfer operator on the GPU: its kept sources and shape
functions against the oracle's, its application against the one-shot
transfer (bit-identical in FP64: same shape functions summed in the same
order) and against exact polynomial reproduction, at small and full size."""
import numpy as np
import pytest
import torch

import parity_cases as C
from gpu_helpers import DEV, dev, gpu_neighbors, gpu_transfer, say
from paper_2510_18838_amd import pcms, synth

pytestmark = pytest.mark.gpu


def build(prob, precision):
    return pcms.Operator(dev(prob.src), dev(prob.tgt), prob.degree, pcms.radius_of(prob),
                         prob.k_cap, inv_scale=prob.inv_scale, o=pcms.opts(precision=precision))


class OpBackend:
    def operator(self, prob, precision):
        op = build(prob, precision)
        n_kept, cols, w = op.export()
        torch.cuda.synchronize()
        r = dict(n_kept=n_kept.cpu().numpy(), cols=cols.cpu().numpy(), weights=w.cpu().numpy(),
                 status=op.status.cpu().numpy())
        assert op.width <= prob.k_cap
        op.free()
        # every row is written in full: kept entries, then -1 and 0
        slot = np.arange(prob.k_cap)[None, :]
        pad = slot >= np.maximum(r["n_kept"], 0)[:, None]
        assert (r["cols"][pad] == -1).all() and (r["weights"][pad] == 0.0).all(), \
            "operator export: row padding not written"
        return r


def test_operator_against_oracle():
    C.case_operator(OpBackend())


class SearchBackend(OpBackend):
    def neighbors(self, prob):
        return gpu_neighbors(prob)

    def transfer(self, prob, precision, weight=0, lam=0.0, block=0):
        out, st, _ = gpu_transfer(prob, precision, weight=weight, lam=lam, block=block)
        return dict(out=out, status=st)


def test_fp32_filtered_search_keeps_the_fp64_lists():
    C.case_fp32_filter(SearchBackend())


def test_random_capped_lists_with_ties():
    C.case_random_caps(SearchBackend())


def test_full_c3_filtered_search_keeps_the_fp64_lists():
    """Every target of the full 3-D workload: the mixed-precision search
    (FP32 records) keeps the same sources, in the same order, as FP64."""
    prob = synth.c3()
    be = OpBackend()
    a, b = be.operator(prob, pcms.FP64), be.operator(prob, pcms.MIXED_REFINE)
    both = (a["n_kept"] >= 0) & (b["n_kept"] >= 0)
    say(f"full c3: {int(both.sum())} targets valid in both, "
        f"{int((a['n_kept'] >= 0).sum())} in FP64")
    assert (a["n_kept"][both] == b["n_kept"][both]).all()
    w = a["cols"].shape[1]
    mask = np.arange(w)[None, :] < a["n_kept"][:, None]
    mask &= both[:, None]
    assert (a["cols"][mask] == b["cols"][mask]).all()


@pytest.mark.parametrize("name", ["c2", "c3", "c5"])
def test_apply_matches_transfer(name):
    prob = C.scaled(name, small=True)
    for prec in (pcms.FP64, pcms.MIXED_REFINE):
        op = build(prob, prec)
        got = op.apply(dev(prob.vals))
        torch.cuda.synchronize()
        got = got.cpu().numpy()
        ref, st, _ = gpu_transfer(prob, prec)
        assert (op.status.cpu().numpy() == st).all()
        ok = (st & 0xF) == 0
        assert np.isnan(got[:, ~ok]).all()
        if prec == pcms.FP64:
            assert np.array_equal(got[:, ok], ref[:, ok]), f"{name}: FP64 apply != transfer"
        else:
            # the one-shot mixed transfer centres the field values
            scale = np.abs(ref[:, ok]).max(axis=1, keepdims=True)
            e = (np.abs(got[:, ok] - ref[:, ok]) / scale).max()
            say(f"{name} MIXED_REFINE apply vs transfer: {e:.3e}")
            assert e <= 1e-9
        op.free()


def test_apply_reproduces_polynomials():
    """Fields that are polynomials of the basis degree are reproduced exactly
    by the shape functions (at lambda = 0), whatever the weights."""
    prob = synth.uniform_problem(53, 20000, 3000, 3, 2, synth.KNN, n_fields=1, k=30, k_cap=40)
    op = build(prob, pcms.FP64)
    rng = np.random.default_rng(5)
    x = prob.src
    c = rng.standard_normal((4, 10))
    feats = np.stack([np.ones(len(x)), x[:, 0], x[:, 1], x[:, 2], x[:, 0] ** 2, x[:, 0] * x[:, 1],
                      x[:, 0] * x[:, 2], x[:, 1] ** 2, x[:, 1] * x[:, 2], x[:, 2] ** 2])
    vals = c @ feats
    t = prob.tgt
    tf = np.stack([np.ones(len(t)), t[:, 0], t[:, 1], t[:, 2], t[:, 0] ** 2, t[:, 0] * t[:, 1],
                   t[:, 0] * t[:, 2], t[:, 1] ** 2, t[:, 1] * t[:, 2], t[:, 2] ** 2])
    want = c @ tf
    got = op.apply(dev(vals)).cpu().numpy()
    ok = (op.status.cpu().numpy() & 0xF) == 0
    e = np.abs(got[:, ok] - want[:, ok]).max() / np.abs(want[:, ok]).max()
    say(f"operator polynomial reproduction: {e:.3e}")
    assert e <= 1e-11
    op.free()


def test_full_c3_operator():
    prob = synth.c3()
    op = build(prob, pcms.MIXED_REFINE)
    vals = dev(prob.vals)
    got = op.apply(vals)
    torch.cuda.synchronize()
    ref, st, _ = gpu_transfer(prob, pcms.MIXED_REFINE)
    got = got.cpu().numpy()
    ok = (st & 0xF) == 0
    assert (op.status.cpu().numpy() == st).all()
    scale = np.abs(ref[:, ok]).max(axis=1, keepdims=True)
    e = (np.abs(got[:, ok] - ref[:, ok]) / scale).max()
    say(f"full c3 operator apply vs transfer: {e:.3e}, width {op.width}")
    # the mixed transfer sums fields centred on the first kept value, the
    # operator sums them as they are: the two differ by the partition-of-unity
    # defect of the refined coefficients (refinement stops near 1e-9 |y|)
    assert e <= 1e-7
    op.free()


def test_round_trip_iterations_match_oracle():
    """Source -> target -> source iterations through two operators (the
    paper's round-trip accuracy protocol) against the same iterations done
    with the FP64 oracle, on a small instance."""
    import oracle
    src, tgt, f = synth.roundtrip_clouds(40, 57)
    h = 4.0 / 40
    kw = dict(mode=synth.FIXED, r=3.5 * h, k_cap=96)
    ops = [pcms.Operator(dev(a), dev(b), 2, pcms.radius(pcms.RADIUS_FIXED, r=3.5 * h), 96,
                         o=pcms.opts(precision=pcms.FP64, weight=pcms.WEIGHT_C4))
           for a, b in ((src, tgt), (tgt, src))]
    g = dev(f[None, :])
    ref = f[None, :]
    for it in range(3):
        g = ops[1].apply(ops[0].apply(g))
        ref_t = oracle.transfer(src, ref, tgt, 2, weight_kind=1, **kw)["out"]
        ref = oracle.transfer(tgt, ref_t, src, 2, weight_kind=1, **kw)["out"]
        got = g.cpu().numpy()
        ok = np.isfinite(ref[0])
        e = np.abs(got[0, ok] - ref[0, ok]).max() / np.abs(ref[0, ok]).max()
        acc = np.linalg.norm(got[0, ok] - f[ok]) / np.linalg.norm(f[ok])
        say(f"round trip {it + 1}: vs oracle {e:.3e}, accuracy error {acc:.3e}")
        assert e <= 1e-10
