"""Host-side checks of the C interface: the library loads, exports every
declared entry point, and rejects bad arguments before touching the GPU."""
import ctypes
import os
import re

import pytest

from paper_2510_18838_amd import pcms

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pcms_mls.h")

needs_lib = pytest.mark.skipif(not os.path.exists(pcms.LIB_PATH),
                               reason="libpcms_mls.so not built (run __graft_entry__.build())")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pcms_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("pcms_grid_build", "pcms_neighbors", "pcms_mls_transfer"):
        assert n in names


@needs_lib
def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(pcms.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert set(pcms.EXPORTED) <= set(declared_functions())


@needs_lib
def test_version_and_defaults():
    L = pcms.lib()
    assert L.pcms_version() >= 100
    o = pcms.MlsOpts()
    o.precision = 7
    L.pcms_mls_opts_default(ctypes.byref(o))
    assert o.weight == 0 and o.precision == 0 and o.lam == 0.0 and o.flags == 0


FAKE = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first


def _transfer(**kw):
    a = dict(src=FAKE, n_src=100, dim=2, vals=FAKE, nf=1, tgt=FAKE, n_tgt=10, degree=1,
             rad=pcms.radius(pcms.RADIUS_FIXED, r=0.1), k_cap=32, g=None, o=None, out=FAKE)
    a.update(kw)
    o = a["o"]
    return pcms.lib().pcms_mls_transfer(a["src"], a["n_src"], a["dim"], a["vals"], a["nf"],
                                        a["tgt"], a["n_tgt"], a["degree"], ctypes.byref(a["rad"]),
                                        a["k_cap"], a["g"], None if o is None else ctypes.byref(o),
                                        None, a["out"], None)


@needs_lib
@pytest.mark.parametrize("kw,msg", [
    (dict(dim=0), "dim"), (dict(dim=6), "dim"), (dict(degree=3), "basis_degree"),
    (dict(degree=-1), "basis_degree"), (dict(nf=0), "n_fields"), (dict(n_src=0), "n_src"),
    (dict(n_tgt=-1), "n_tgt"), (dict(k_cap=2), "k_cap"), (dict(k_cap=257), "k_cap"),
    (dict(src=None), "src"), (dict(vals=None), "required"), (dict(out=None), "required"),
    (dict(rad=pcms.radius(pcms.RADIUS_FIXED, r=0.0)), "radius"),
    (dict(rad=pcms.radius(pcms.RADIUS_FIXED, r=float("inf"))), "radius"),
    (dict(rad=pcms.radius(pcms.RADIUS_KNN, k=0)), "k must"),
    (dict(rad=pcms.radius(pcms.RADIUS_KNN, k=101)), "k must"),
    (dict(rad=pcms.radius(pcms.RADIUS_GROW, r=0.1, n_min=0)), "n_min"),
    (dict(rad=pcms.radius(pcms.RADIUS_GROW, r=0.1, n_min=3, max_iter=-1)), "max_iter"),
    (dict(rad=pcms.radius(7, r=0.1)), "mode"),
])
def test_transfer_rejects_bad_arguments(kw, msg):
    assert _transfer(**kw) == pcms.PCMS_ERR_ARG
    assert msg in pcms.last_error()


@needs_lib
def test_transfer_rejects_bad_options():
    o = pcms.opts(lam=-1.0)
    assert _transfer(o=o) == pcms.PCMS_ERR_ARG and "lambda" in pcms.last_error()
    o = pcms.opts(precision=3)
    assert _transfer(o=o) == pcms.PCMS_ERR_ARG
    o = pcms.opts(weight=9)
    assert _transfer(o=o) == pcms.PCMS_ERR_ARG
    o = pcms.opts(block=96)
    assert _transfer(o=o) == pcms.PCMS_ERR_ARG
    o = pcms.opts(flags=pcms.ASYNC)
    assert _transfer(o=o) == pcms.PCMS_ERR_ARG and "summary" in pcms.last_error()
    g = (ctypes.c_double * 2)(1.0, -2.0)
    assert _transfer(g=ctypes.cast(g, ctypes.c_void_p)) == pcms.PCMS_ERR_ARG
    o = pcms.opts(flags=0x80)
    assert _transfer(o=o) == pcms.PCMS_ERR_ARG and "flag" in pcms.last_error()


@needs_lib
def test_empty_target_set_is_a_no_op():
    assert _transfer(n_tgt=0, tgt=None, out=None, vals=None) == pcms.PCMS_OK


@needs_lib
def test_grid_and_neighbor_argument_checks():
    L = pcms.lib()
    h = ctypes.c_void_p()
    assert L.pcms_grid_build(FAKE, 10, 9, None, 0.0, 0.0, None, ctypes.byref(h)) == pcms.PCMS_ERR_ARG
    assert L.pcms_grid_build(None, 10, 2, None, 0.0, 0.0, None, ctypes.byref(h)) == pcms.PCMS_ERR_ARG
    assert L.pcms_grid_build(FAKE, 10, 2, None, -1.0, 0.0, None, ctypes.byref(h)) == pcms.PCMS_ERR_ARG
    r = pcms.radius(pcms.RADIUS_FIXED, r=0.1)
    assert L.pcms_neighbors(None, FAKE, 5, ctypes.byref(r), 8, None, FAKE, FAKE, None, None,
                            None) == pcms.PCMS_ERR_ARG
    assert L.pcms_mls_transfer_grid(None, FAKE, 1, FAKE, 5, 1, ctypes.byref(r), 8, None, None,
                                    FAKE, None) == pcms.PCMS_ERR_ARG
    assert L.pcms_grid_free(None) == pcms.PCMS_OK
    assert L.pcms_lbvh_build(FAKE, 10, 6, None, 0, None, ctypes.byref(h)) == pcms.PCMS_ERR_ARG
    assert L.pcms_lbvh_build(None, 10, 2, None, 0, None, ctypes.byref(h)) == pcms.PCMS_ERR_ARG
    assert L.pcms_lbvh_build(FAKE, 0, 2, None, 0, None, ctypes.byref(h)) == pcms.PCMS_ERR_ARG
    bad = (ctypes.c_double * 2)(1.0, 0.0)
    assert L.pcms_lbvh_build(FAKE, 10, 2, ctypes.cast(bad, ctypes.c_void_p), 0, None,
                             ctypes.byref(h)) == pcms.PCMS_ERR_ARG
    assert L.pcms_lbvh_build(FAKE, 10, 2, None, 0, None, None) == pcms.PCMS_ERR_ARG
    assert L.pcms_lbvh_build(FAKE, 10, 2, None, 65, None, ctypes.byref(h)) == pcms.PCMS_ERR_ARG
    assert L.pcms_lbvh_build(FAKE, 10, 2, None, -1, None, ctypes.byref(h)) == pcms.PCMS_ERR_ARG
    assert L.pcms_grid_is_lbvh(None) == 0


def _problem(**kw):
    a = dict(src=0x1000, n_src=100, dim=2, basis_degree=1, src_vals=0x1000, n_fields=1, k_cap=32,
             tgt=0x1000, n_tgt=10, radius=pcms.radius(pcms.RADIUS_FIXED, r=0.1), inv_scale=None,
             tgt_vals=0x1000, status=None)
    a.update(kw)
    return pcms.Problem(**a)


def _plan(probs, o=None):
    arr = (pcms.Problem * max(len(probs), 1))(*probs)
    h = ctypes.c_void_p()
    return pcms.lib().pcms_batch_plan_create(arr if probs else None, len(probs),
                                             None if o is None else ctypes.byref(o),
                                             ctypes.byref(h))


@needs_lib
def test_batch_defaults():
    o = pcms.BatchOpts()
    pcms.lib().pcms_batch_opts_default(ctypes.byref(o))
    assert o.weight == 0 and o.precision == pcms.MIXED_REFINE and o.block == 0
    assert o.cell_factor == 0.0 and o.tune_cache is None


@needs_lib
@pytest.mark.parametrize("kw,msg", [
    (dict(dim=6), "problem 1: dim"), (dict(n_src=0), "problem 1: n_src"),
    (dict(k_cap=2), "problem 1: k_cap"), (dict(src=None), "problem 1: src"),
    (dict(tgt_vals=None), "problem 1: src_vals, tgt and tgt_vals"),
    (dict(radius=pcms.radius(pcms.RADIUS_KNN, k=500)), "problem 1: KNN k"),
])
def test_batch_plan_rejects_bad_problems(kw, msg):
    assert _plan([_problem(), _problem(**kw)]) == pcms.PCMS_ERR_ARG
    assert msg in pcms.last_error()


@needs_lib
def test_batch_plan_rejects_bad_options():
    assert _plan([]) == pcms.PCMS_ERR_ARG
    assert _plan([_problem()], pcms.batch_opts(block=96)) == pcms.PCMS_ERR_ARG
    assert _plan([_problem()], pcms.batch_opts(cell_factor=5.0)) == pcms.PCMS_ERR_ARG
    assert _plan([_problem()], pcms.batch_opts(precision=4)) == pcms.PCMS_ERR_ARG
    assert _plan([_problem()], pcms.batch_opts(lam=-1.0)) == pcms.PCMS_ERR_ARG
    L = pcms.lib()
    assert L.pcms_batch_plan_exec(None, None, None) == pcms.PCMS_ERR_ARG
    assert L.pcms_batch_plan_free(None) == pcms.PCMS_OK


@needs_lib
def test_operator_argument_checks():
    L = pcms.lib()
    h = ctypes.c_void_p()
    r = pcms.radius(pcms.RADIUS_FIXED, r=0.1)
    o = pcms.opts()
    build = lambda **kw: L.pcms_operator_build(
        kw.get("src", FAKE), kw.get("n_src", 100), kw.get("dim", 2), kw.get("tgt", FAKE),
        kw.get("n_tgt", 10), kw.get("degree", 1), ctypes.byref(kw.get("rad", r)),
        kw.get("k_cap", 32), None, ctypes.byref(o), None, None, ctypes.byref(h))
    assert build(dim=6) == pcms.PCMS_ERR_ARG and "dim" in pcms.last_error()
    assert build(src=None) == pcms.PCMS_ERR_ARG
    assert build(tgt=None) == pcms.PCMS_ERR_ARG
    assert build(k_cap=2) == pcms.PCMS_ERR_ARG
    assert build(rad=pcms.radius(pcms.RADIUS_KNN, k=0)) == pcms.PCMS_ERR_ARG
    assert L.pcms_operator_apply(None, FAKE, 1, None, FAKE) == pcms.PCMS_ERR_ARG
    assert L.pcms_operator_export(None, 8, None, FAKE, None, None) == pcms.PCMS_ERR_ARG
    assert L.pcms_operator_width(None) == 0
    assert L.pcms_operator_free(None) == pcms.PCMS_OK


# --- the Python binding's shape checks (no GPU: a ValueError is raised before
# any library call; the GPU-device test is relaxed so CPU tensors reach them)

@pytest.fixture
def cpu_as_gpu(monkeypatch):
    import torch
    monkeypatch.setattr(pcms, "_is_gpu", lambda t: True)
    return torch


def _f64(torch, *shape):
    return torch.zeros(*shape, dtype=torch.float64)


@needs_lib
@pytest.mark.parametrize("case,msg", [
    ("src_1d", "src must have shape"),
    ("src_6cols", "1 to 5 columns"),
    ("tgt_dim", "tgt must have shape"),
    ("vals_len", "src_vals must have shape"),
    ("vals_2d_len", "src_vals must have shape"),
    ("vals_dtype", "src_vals must be torch.float64"),
    ("out_shape", "out must have shape"),
    ("out_dtype", "out must be torch.float64"),
    ("status_len", "status must have shape"),
    ("status_dtype", "status must be torch.uint8"),
    ("tgt_strided", "tgt must be contiguous"),
])
def test_binding_rejects_bad_shapes(cpu_as_gpu, case, msg):
    torch = cpu_as_gpu
    src, vals, tgt = _f64(torch, 100, 2), _f64(torch, 3, 100), _f64(torch, 10, 2)
    out, status = None, None
    if case == "src_1d":
        src = _f64(torch, 100)
    elif case == "src_6cols":
        src, tgt = _f64(torch, 100, 6), _f64(torch, 10, 6)
    elif case == "tgt_dim":
        tgt = _f64(torch, 10, 3)
    elif case == "vals_len":
        vals = _f64(torch, 99)
    elif case == "vals_2d_len":
        vals = _f64(torch, 3, 101)
    elif case == "vals_dtype":
        vals = torch.zeros(3, 100, dtype=torch.float32)
    elif case == "out_shape":
        out = _f64(torch, 3, 9)
    elif case == "out_dtype":
        out = torch.zeros(3, 10, dtype=torch.float32)
    elif case == "status_len":
        status = torch.zeros(11, dtype=torch.uint8)
    elif case == "status_dtype":
        status = torch.zeros(10, dtype=torch.int32)
    elif case == "tgt_strided":
        tgt = _f64(torch, 2, 10).t()
    with pytest.raises(ValueError, match=msg):
        pcms.pcms_mls_transfer(src, vals, tgt, 1, pcms.radius(pcms.RADIUS_FIXED, r=0.1), 32,
                               out=out, status=status)


@needs_lib
def test_binding_rejects_bad_shapes_on_grid_operator_and_batch(cpu_as_gpu):
    torch = cpu_as_gpu
    g = pcms.Grid(None, 100, 2)           # a handle-less stand-in: checks run first
    rad = pcms.radius(pcms.RADIUS_FIXED, r=0.1)
    with pytest.raises(ValueError, match="tgt must have shape"):
        pcms.pcms_neighbors(g, _f64(torch, 10, 3), rad, 16)
    with pytest.raises(ValueError, match="src_vals must have shape"):
        pcms.pcms_mls_transfer_grid(g, _f64(torch, 2, 50), _f64(torch, 10, 2), 1, rad, 16)
    with pytest.raises(ValueError, match="out must have shape"):
        pcms.pcms_mls_transfer_grid(g, _f64(torch, 2, 100), _f64(torch, 10, 2), 1, rad, 16,
                                    out=_f64(torch, 1, 10))
    with pytest.raises(ValueError, match="src_vals must have shape"):
        pcms.BatchProblem(_f64(torch, 100, 3), _f64(torch, 2, 90), _f64(torch, 7, 3), 1, rad, 16)
    with pytest.raises(ValueError, match="tgt must have shape"):
        pcms.BatchProblem(_f64(torch, 100, 3), _f64(torch, 2, 100), _f64(torch, 7, 2), 1, rad, 16)
    op = pcms.Operator.__new__(pcms.Operator)   # the apply-side checks of a built operator
    op.n_src, op.n_tgt, op.device, op.handle = 100, 10, torch.device("cpu"), None
    with pytest.raises(ValueError, match="src_vals must have shape"):
        op.apply(_f64(torch, 4, 99))
    with pytest.raises(ValueError, match="out must have shape"):
        op.apply(_f64(torch, 4, 100), out=_f64(torch, 4, 11))
    with pytest.raises(ValueError, match="status must have shape"):
        pcms.Operator(_f64(torch, 100, 2), _f64(torch, 10, 2), 1, rad, 16,
                      status=torch.zeros(9, dtype=torch.uint8))


@needs_lib
def test_workspace_query():
    """Host-only sizes: the grid holds at least its FP64 and FP32 records and
    both permutations; the transfer on a grid at least the bucket-ordered
    field records and the target order; the one-shot call both."""
    n_src, dim, nf, n_tgt = 1_000_000, 3, 8, 500_000
    w = pcms.pcms_workspace_query(n_src, dim, nf, n_tgt)
    assert w["grid_bytes"] >= n_src * (4 * 8 + 3 * 4 + 2 * 4)
    assert w["transfer_grid_bytes"] >= n_src * nf * 8 + n_tgt * 4
    assert w["transfer_bytes"] >= w["grid_bytes"] + w["transfer_grid_bytes"]
    assert w["operator_apply_bytes"] == n_src * nf * 8
    assert w["noalloc_limit"] == pcms.lib().pcms_noalloc_scratch_bytes() == 128 << 20
    # the LBVH: one bucket instead of the grid's, plus (n_src / 8 - 1) nodes of
    # 16 floats in 3-D
    nodes = (n_src // 8 - 1) * 16 * 4
    assert w["lbvh_bytes"] >= n_src * (4 * 8 + 3 * 4 + 2 * 4) + nodes
    assert w["lbvh_build_bytes"] >= n_src * 12
    assert w["transfer_bytes"] >= w["lbvh_bytes"] + w["transfer_grid_bytes"]
    w2 = pcms.pcms_workspace_query(n_src, dim, nf + 1, n_tgt)   # odd counts pad to even
    assert w2["operator_apply_bytes"] == n_src * (nf + 2) * 8
    for bad in ((0, 3, 1, 1), (10, 0, 1, 1), (10, 6, 1, 1), (10, 3, 0, 1), (10, 3, 1, -1)):
        with pytest.raises(pcms.PcmsError):
            pcms.pcms_workspace_query(*bad)
