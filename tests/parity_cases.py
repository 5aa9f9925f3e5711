"""Parity cases shared by the GPU tests and the CPU emulation tests.

A backend provides neighbors(prob) and transfer(prob, precision, weight, lam,
block) returning the same dicts as the oracle wrapper; every case compares
it with the FP64 CPU oracle on seeded inputs.

Bars: neighbour lists, counts, squared radii and statuses bit-exact; values
within TOL (max over fields of the inf-norm error over valid targets,
relative to the field's inf-norm: Eq. 2's accuracy error read with the
inf-norm), plus a per-target conditioning term COND * kappa.  MIXED_REFINE is
the mixed-precision mode held to 1e-6: it refines to the FP64 solution, so it
takes the FP64 conditioning term, and its error over the whole case must also
meet the flat 1e-6 gate of the accuracy metric.  MIXED without refinement is
held to 1e-4 + 100 u32 kappa (its error grows with the conditioning of the
FP32 moment matrix).
"""
from __future__ import annotations

import math

import numpy as np

import oracle
from paper_2510_18838_amd import synth

FP64, MIXED, MIXED_REFINE = 0, 1, 2
TOL = {FP64: 1e-10, MIXED_REFINE: 1e-6, MIXED: 1e-4}
# rounding grows with the conditioning kappa of the moment matrix: 1000 u64
# for FP64 normal equations, and for refined mixed, whose residual is formed
# from FP64 per-neighbour data so that it converges to the FP64 solution;
# 100 u32 for unrefined FP32 assembly
COND = {FP64: 1e3 * 1.1e-16, MIXED_REFINE: 1e3 * 1.1e-16, MIXED: 100 * 6e-8}
# the accuracy metric's gate (Eq. 2 with the inf-norm), over all valid targets
GATE = {MIXED_REFINE: 1e-6}
CAPPED = 0x10


def say(msg):
    print(msg, flush=True)


def compare_lists(got, ref, where=""):
    for key in ("n_kept", "n_found", "status"):
        bad = np.nonzero(got[key] != ref[key])[0]
        assert bad.size == 0, (f"{where}: {key} differs at {bad[:5]}: "
                               f"got {got[key][bad[:5]]} ref {ref[key][bad[:5]]}")
    bad = np.nonzero(got["r2"] != ref["r2"])[0]
    assert bad.size == 0, f"{where}: r2 differs at {bad[:5]}"
    for i in range(len(ref["n_kept"])):
        n = ref["n_kept"][i]
        if not np.array_equal(got["nbr"][i, :n], ref["nbr"][i, :n]):
            raise AssertionError(f"{where}: list of target {i} differs")


def rel_err(got, ref, mask):
    """max over fields of ||got - ref||_inf / ||ref||_inf over the targets in mask."""
    if not mask.any():
        return 0.0
    worst = 0.0
    for l in range(ref.shape[0]):
        den = np.abs(ref[l, mask]).max()
        num = np.abs(got[l, mask] - ref[l, mask]).max()
        worst = max(worst, num / den)
    return worst


def check_lists(be, prob, where, brute=False):
    ref = oracle.neighbors(prob.src, prob.tgt, brute=brute, **oracle.problem_kwargs(prob))
    compare_lists(be.neighbors(prob), ref, where)
    return ref


# Table 1's No_Op (identity) weight is phi = 1; on the selected sources, the
# only ones that enter the fit, it is the Const weight
NO_OP, CONST = 5, 3


def check_transfer(be, prob, where, precisions=(FP64, MIXED_REFINE, MIXED), weight=0, lam=0.0):
    ref = oracle.transfer(prob.src, prob.vals, prob.tgt, prob.degree,
                          weight_kind=CONST if weight == NO_OP else weight, lam=lam,
                          **oracle.problem_kwargs(prob))
    ok = (ref["status"] & 0xF) == 0
    errs = {}
    for prec in precisions:
        r = be.transfer(prob, prec, weight=weight, lam=lam)
        got, st = r["out"], r["status"]
        bad = np.nonzero(st != ref["status"])[0]
        # statuses may differ only where the oracle's smallest Cholesky pivot
        # is near the singularity threshold (FP64) or beyond FP32 reach (mixed)
        limit = 1e-11 if prec == FP64 else 1e-5
        assert all(ref["pivot_ratio"][i] < limit for i in bad), \
            f"{where}: status differs at {bad[:5]}: {st[bad[:5]]} vs {ref['status'][bad[:5]]}"
        mask = ok & (st == ref["status"])
        assert np.isfinite(got[:, mask]).all(), f"{where}: non-finite values"
        assert np.isnan(got[:, (st & 0xF) != 0]).all(), f"{where}: failed targets not NaN"
        e = rel_err(got, ref["out"], mask)
        errs[prec] = e
        # per target: TOL plus a conditioning term, kappa ~ 1 / (smallest
        # Cholesky pivot / largest diagonal entry) of the oracle's moment matrix
        kappa = 1.0 / np.maximum(ref["pivot_ratio"][mask], 1e-300)
        scale = np.abs(ref["out"][:, mask]).max(axis=1, keepdims=True)
        dev = (np.abs(got[:, mask] - ref["out"][:, mask]) / scale).max(axis=0)
        bound = TOL[prec] + COND[prec] * kappa
        well = kappa < 1e6
        e_well = float(dev[well].max()) if well.any() else 0.0
        say(f"{where} precision={prec}: max rel err {e:.3e} over {int(mask.sum())} targets, "
            f"{e_well:.3e} over the {int(well.sum())} with kappa < 1e6")
        worst = np.argmax(dev - bound) if dev.size else 0
        assert (dev <= bound).all(), (f"{where}: precision {prec} error {dev[worst]:.3e} above "
                                      f"{bound[worst]:.3e} (kappa {kappa[worst]:.2e})")
        if prec in GATE:
            assert e <= GATE[prec], f"{where}: precision {prec} error {e:.3e} above the gate {GATE[prec]:.0e}"
    return errs


def custom(src, vals, tgt, degree, mode, **kw):
    vals = np.atleast_2d(vals)
    return synth.Problem("custom", np.ascontiguousarray(src, dtype=np.float64),
                         np.ascontiguousarray(vals, dtype=np.float64),
                         np.ascontiguousarray(tgt, dtype=np.float64), degree=degree, mode=mode,
                         **kw)


# ---------------------------------------------------------------------------
# cases
# ---------------------------------------------------------------------------

def case_c1(be):
    p = synth.c1()
    ref = check_lists(be, p, "c1", brute=True)
    assert (ref["status"] & CAPPED).sum() > 10         # the cap path is exercised
    check_transfer(be, p, "c1")


def scaled(name, small=False):
    if name == "c2":
        return synth.c2(n_side=60 if small else 150, n_tgt=2011 if small else 20011)
    if name == "c3":
        return synth.c3(n_src=15000 if small else 60000, n_tgt=2013 if small else 20013,
                        n_fields=3 if small else 8)
    if name == "c5":
        return synth.c5(n=12000 if small else 40000, n_tgt=2007 if small else 15007)
    raise KeyError(name)


def case_scaled(be, name, small=False):
    p = scaled(name, small)
    say(f"{name}: n_src={p.src.shape[0]} n_tgt={p.tgt.shape[0]} dim={p.dim}")
    check_lists(be, p, name)
    check_transfer(be, p, name)


def case_c4(be, n=8, size_scale=0.05):
    for b in range(n):
        p = synth.c4_problem(b, size_scale=size_scale)
        say(f"c4 problem {b}: n_src={p.src.shape[0]} n_tgt={p.tgt.shape[0]} d={p.dim} "
            f"p={p.degree} nf={p.n_fields}")
        check_lists(be, p, f"c4[{b}]")
        check_transfer(be, p, f"c4[{b}]")


DIM_CASES = [(1, 2, synth.KNN), (1, 1, synth.FIXED), (4, 1, synth.KNN), (4, 2, synth.GROW),
             (2, 0, synth.FIXED), (3, 0, synth.KNN), (5, 2, synth.KNN)]


def case_dims(be, dim, degree, mode, scale=1.0):
    m = math.comb(dim + degree, degree)
    n_src = int((6000 if dim < 5 else 20000) * scale)
    kw = dict(radius=(0.02 if dim == 1 else 0.15), k=2 * m + 3, n_min=2 * m, k_cap=max(3 * m, 8))
    p = synth.uniform_problem(7 + dim * 3 + degree, n_src, int(3001 * scale), dim, degree, mode,
                              n_fields=3, **kw)
    check_lists(be, p, f"d{dim}p{degree}")
    check_transfer(be, p, f"d{dim}p{degree}m{mode}")


def case_weight(be, weight):
    p = synth.uniform_problem(31, 5000, 2000, 2, 2, synth.KNN, n_fields=2, k=20, k_cap=32)
    check_transfer(be, p, f"weight {weight}", precisions=(FP64, MIXED_REFINE), weight=weight)


def case_tikhonov(be, lam):
    p = synth.uniform_problem(32, 5000, 2000, 3, 2, synth.KNN, n_fields=2, k=25, k_cap=32)
    check_transfer(be, p, f"lambda {lam}", precisions=(FP64, MIXED_REFINE), lam=lam)


def case_far_targets(be):
    rng = np.random.default_rng(3)
    src = rng.uniform(0, 1, (500, 2))
    vals = rng.standard_normal(500)
    tgt = np.array([[0.5, 0.5], [7.0, -3.0], [1.02, 0.5]])
    for t in (tgt[:1], tgt):
        p = custom(src, vals, t, 1, synth.FIXED, radius=0.1, k_cap=64)
        check_transfer(be, p, f"far fixed {len(t)}")
        r = be.transfer(p, FP64)
        if len(t) > 1:
            assert r["status"][1] == 1
    p = custom(src, vals, tgt, 2, synth.KNN, k=12, k_cap=16)
    check_lists(be, p, "far knn")
    check_transfer(be, p, "far knn")


def case_singular_exhausted(be):
    x = np.linspace(0, 1, 64)
    line = np.stack([x, np.full_like(x, 0.5)], 1)
    # collinear sources and a quadratic basis: G is singular in exact
    # arithmetic for targets on the line and off it (where the y monomials are
    # constant multiples of 1); FP32 accumulation leaves pivots of rounding
    # size, which the unrefined mixed mode must still call singular
    p = custom(line, x, np.array([[0.5, 0.5], [0.25, 0.5], [0.5, 0.6], [0.3, 0.41]]), 2,
               synth.FIXED, radius=0.3, k_cap=64)
    for prec in (FP64, MIXED_REFINE, MIXED):
        r = be.transfer(p, prec)
        assert (r["status"] == 2).all() and np.isnan(r["out"]).all(), (prec, r["status"])
    rng = np.random.default_rng(5)
    src = rng.uniform(0, 1, (300, 2))
    p = custom(src, src[:, 0], np.array([[0.5, 0.5], [0.2, 0.7]]), 1, synth.GROW, radius=1e-4,
               n_min=10, max_iter=0, k_cap=32)
    r = be.transfer(p, FP64)
    assert (r["status"] == 3).all()
    p.max_iter = 40
    check_lists(be, p, "grow")
    check_transfer(be, p, "grow")


def case_ties(be):
    g1 = np.arange(9) * 0.125
    lat = np.stack(np.meshgrid(g1, g1, indexing="ij"), -1).reshape(-1, 2)
    src = np.concatenate([lat, lat[::3]])                  # exact ties and duplicates
    tgt = np.concatenate([lat[::5], lat[::7] + 0.0625])
    for mode, kw in [(synth.FIXED, dict(radius=0.25, k_cap=6)), (synth.KNN, dict(k=9, k_cap=5)),
                     (synth.KNN, dict(k=13, k_cap=40)),
                     (synth.GROW, dict(radius=0.1, n_min=11, k_cap=7))]:
        p = custom(src, src[:, 0] + 2 * src[:, 1], tgt, 1, mode, **kw)
        check_lists(be, p, f"ties {mode} {kw}", brute=True)
    same = np.full((50, 3), 0.25)                          # one bucket, all distances tie
    p = custom(same, np.ones(50), np.array([[0.25, 0.25, 0.25], [0.3, 0.2, 0.1]]), 0,
               synth.KNN, k=10, k_cap=16)
    check_lists(be, p, "coincident", brute=True)


def case_box_boundary(be):
    """kNN targets where the bounding-box correction of the radius estimate
    acts: corners, edge and face centres, targets just inside and outside
    the faces, in 2-D and 3-D, on the grid and (for backends that have it)
    the LBVH; then a flat 3-D cloud (one coordinate constant) and a thin
    slab, where the correction is bounded.  Lists and radii bit-exact,
    values to the usual bars."""
    rng = np.random.default_rng(29)
    for d in (2, 3):
        src = rng.uniform(0, 1, (6000 if d == 3 else 3000, d))
        corners = np.array(np.meshgrid(*[[0.0, 1.0]] * d, indexing="ij")).reshape(d, -1).T
        faces = np.concatenate([np.eye(d) * v + 0.5 * (1 - np.eye(d)) for v in (0.0, 1.0)])
        mids = (corners[:, None, :] + corners[None, :, :]).reshape(-1, d) / 2
        near = rng.uniform(0, 1, (300, d))
        axis = rng.integers(0, d, 300)
        side = rng.integers(0, 2, 300).astype(float)
        near[np.arange(300), axis] = side + rng.uniform(-0.03, 0.03, 300)
        tgt = np.concatenate([corners, faces, mids, near, corners * 1.1 - 0.05])
        vals = np.stack([np.sin(3 * src.sum(1)), src[:, 0] ** 2])
        for k, deg in ((10, 1), (40, 2)):
            p = custom(src, vals, tgt, deg, synth.KNN, k=k, k_cap=64)
            check_lists(be, p, f"box boundary d={d} k={k}")
            check_transfer(be, p, f"box boundary d={d} k={k}")
    flat = rng.uniform(0, 1, (2000, 3))
    flat[:, 2] = 0.5
    slab = rng.uniform(0, 1, (2000, 3))
    slab[:, 2] = 0.5 + 1e-3 * slab[:, 2]
    tgt = np.concatenate([rng.uniform(0, 1, (200, 3)), [[0.5, 0.5, 0.5], [0.0, 0.0, 0.5]]])
    for name, src in (("flat", flat), ("slab", slab)):
        p = custom(src, np.sin(4 * src[:, 0]), tgt, 1, synth.KNN, k=12, k_cap=32)
        check_lists(be, p, f"{name} cloud", brute=True)


def case_tight_caps(be):
    p = synth.uniform_problem(41, 3000, 1500, 2, 2, synth.FIXED, n_fields=1, radius=0.08, k_cap=6)
    check_lists(be, p, "k_cap = m")
    check_transfer(be, p, "k_cap = m")
    p.k_cap, p.degree = 1, 0
    check_lists(be, p, "k_cap = 1")
    check_transfer(be, p, "k_cap = 1")


def check_operator(be, prob, where, precisions=(FP64, MIXED_REFINE)):
    """The transfer operator (kept sources and shape functions per target)
    against the oracle's lists and shape functions N_e = w_e p_e^T G^{-1} e_0:
    the same sources (bit-exact sets), the weights to the precision's bar
    relative to the target's largest |N|."""
    ref = oracle.transfer(prob.src, prob.vals, prob.tgt, prob.degree, want_shape=True,
                          **oracle.problem_kwargs(prob))
    ok_ref = (ref["status"] & 0xF) == 0
    for prec in precisions:
        r = be.operator(prob, prec)
        st = r["status"]
        bad = np.nonzero(st != ref["status"])[0]
        limit = 1e-11 if prec == FP64 else 1e-5
        assert all(ref["pivot_ratio"][i] < limit for i in bad), \
            f"{where}: status differs at {bad[:5]}"
        valid = ok_ref & (st == ref["status"])
        assert (r["n_kept"][(st & 0xF) != 0] == -1).all(), f"{where}: failed targets not marked"
        worst = 0.0
        for i in np.nonzero(valid)[0]:
            n = ref["n_kept"][i]
            assert r["n_kept"][i] == n, f"{where}: target {i} keeps {r['n_kept'][i]} vs {n}"
            order = np.argsort(r["cols"][i, :n], kind="stable")
            cols, w = r["cols"][i, :n][order], r["weights"][i, :n][order]
            assert np.array_equal(cols, ref["nbr"][i, :n]), f"{where}: target {i} sources differ"
            wr = ref["shape"][i, :n]
            kappa = 1.0 / max(ref["pivot_ratio"][i], 1e-300)
            dev = np.abs(w - wr).max() / np.abs(wr).max()
            bound = TOL[prec] + COND[prec] * kappa
            assert dev <= bound, f"{where}: target {i} shape functions off by {dev:.3e} > {bound:.3e}"
            worst = max(worst, dev)
        say(f"{where} precision={prec}: operator max rel dev {worst:.3e} over {int(valid.sum())} targets")


def case_operator(be):
    check_operator(be, synth.c1(), "operator c1")
    check_operator(be, synth.uniform_problem(51, 4000, 700, 3, 2, synth.KNN, n_fields=1, k=30,
                                             k_cap=40), "operator 3-D kNN")
    check_operator(be, synth.uniform_problem(52, 3000, 500, 2, 2, synth.GROW, n_fields=1,
                                             radius=0.02, n_min=12, k_cap=24,
                                             inv_scale=[1.0, 3.0]), "operator 2-D grow, metric")


def check_same_search(be, prob, where):
    """The mixed-precision searches read FP32 records and recheck candidates
    near a threshold with their FP64 records: the kept sources, their order
    and the counts must equal those of the FP64 search exactly."""
    a, b = be.operator(prob, FP64), be.operator(prob, MIXED_REFINE)
    both = (a["n_kept"] >= 0) & (b["n_kept"] >= 0)
    # only the solve may fail differently (singularity seen through FP32)
    assert ((a["status"] & 0x10) == (b["status"] & 0x10)).all(), f"{where}: capped flags differ"
    assert (a["n_kept"][both] == b["n_kept"][both]).all(), f"{where}: kept counts differ"
    for i in np.nonzero(both)[0]:
        n = a["n_kept"][i]
        assert np.array_equal(a["cols"][i, :n], b["cols"][i, :n]), f"{where}: target {i} differs"
    say(f"{where}: {int(both.sum())} targets, same kept sources in the same order")


def case_fp32_filter(be):
    """Inputs that put many candidates within FP32 rounding of a threshold
    (shells of sources at the support radius, kNN shells where every distance
    ties to 1e-7), coordinates far from the origin (FP32 records too coarse to
    classify anything), tiny coordinates (FP32 underflow), a strongly
    anisotropic metric and exact ties: the FP32-filtered search keeps what
    the FP64 search keeps."""
    rng = np.random.default_rng(61)
    centres = rng.uniform(0.2, 0.8, (12, 3))
    r = 0.05
    shell = []
    for c in centres:
        d = rng.standard_normal((150, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        shell.append(c + d * (r * (1.0 + rng.uniform(-1e-7, 1e-7, (150, 1)))))
    src = np.concatenate(shell + [rng.uniform(0, 1, (3000, 3))])
    vals = src[:, 0] - src[:, 2]
    # degree 0: the fit stays defined however small the shell's weights are
    p = custom(src, vals, centres, 0, synth.FIXED, radius=r, k_cap=256)
    check_lists(be, p, "shell fixed", brute=True)
    check_same_search(be, p, "shell fixed")
    # some targets keep only shell sources, whose weights are ~1e-28
    check_transfer(be, p, "shell fixed")
    p = custom(src, vals, centres, 0, synth.KNN, k=60, k_cap=64)
    check_lists(be, p, "shell knn", brute=True)
    check_same_search(be, p, "shell knn")
    for name, off, scale in (("offset 1e6", 1e6, 1.0), ("tiny 1e-25", 0.0, 1e-25)):
        s2 = off + scale * rng.uniform(0, 1, (4000, 2))
        t2 = off + scale * rng.uniform(0, 1, (300, 2))
        for mode, kw in ((synth.KNN, dict(k=12, k_cap=16)),
                         (synth.FIXED, dict(radius=0.02 * scale, k_cap=64))):
            p = custom(s2, s2[:, 0] * 0 + 1.0, t2, 1, mode, **kw)
            check_lists(be, p, f"{name} {mode}")
            check_same_search(be, p, f"{name} {mode}")
    p = synth.uniform_problem(62, 6000, 500, 3, 1, synth.KNN, n_fields=1, k=20, k_cap=32,
                              inv_scale=[1e3, 1.0, 1e-3])
    check_lists(be, p, "anisotropic")
    check_same_search(be, p, "anisotropic")
    g1 = np.arange(9) * 0.125
    lat = np.stack(np.meshgrid(g1, g1, indexing="ij"), -1).reshape(-1, 2)
    src = np.concatenate([lat, lat[::3]])
    tgt = np.concatenate([lat[::5], lat[::7] + 0.0625])
    for mode, kw in ((synth.FIXED, dict(radius=0.25, k_cap=40)), (synth.KNN, dict(k=13, k_cap=40))):
        p = custom(src, src[:, 0] + 2 * src[:, 1], tgt, 1, mode, **kw)
        check_same_search(be, p, f"lattice ties {mode}")


def case_random_caps(be, trials=40, seed=7):
    """Seeded random small problems (uniform, lattice with duplicates,
    clustered; 1-3 dimensions; fixed, kNN beyond the cap, growing radii;
    caps from m to 23) whose lists are mostly capped and full of exact ties:
    the lists against brute force, and the mixed-precision search's kept
    sources against the FP64 search's."""
    rng = np.random.default_rng(seed)
    for trial in range(trials):
        d = int(rng.integers(1, 4))
        kind = int(rng.integers(0, 3))
        n = int(rng.integers(50, 600))
        if kind == 0:
            src = rng.uniform(0, 1, (n, d))
        elif kind == 1:
            g1 = np.arange(int(round(n ** (1 / d))) + 1) / 8.0
            src = np.stack(np.meshgrid(*([g1] * d), indexing="ij"), -1).reshape(-1, d)
            src = np.concatenate([src, src[::3]])
        else:
            src = rng.normal(0.5, 0.05, (n, d))
        tgt = np.concatenate([src[rng.integers(0, len(src), 20)], rng.uniform(0, 1, (20, d))])
        mode = int(rng.integers(0, 3))
        k_cap = int(rng.integers(max(2, d + 1), 24))
        if mode == 0:
            kw, m = dict(radius=float(rng.uniform(0.1, 0.4)), k_cap=k_cap), synth.FIXED
        elif mode == 1:
            kw, m = dict(k=int(rng.integers(k_cap + 2, k_cap + 20)), k_cap=k_cap), synth.KNN
        else:
            kw, m = dict(radius=float(rng.uniform(0.02, 0.1)), n_min=int(rng.integers(3, 12)),
                         k_cap=k_cap), synth.GROW
        p = custom(src, src[:, 0], tgt, 0, m, **kw)
        where = f"random caps {trial} (d={d}, kind={kind}, mode={m}, {kw})"
        check_lists(be, p, where, brute=True)
        check_same_search(be, p, where)
