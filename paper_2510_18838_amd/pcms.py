"""Python binding of the C interface in include/pcms_mls.h.

Argument marshalling only: every step of the transfer runs in the HIP
library (libpcms_mls.so).  Tensors are passed as device pointers together
with torch's current HIP stream.  When the library is missing this module
raises; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpcms_mls.so")

PCMS_OK = 0
PCMS_ERR_ARG = 1
PCMS_ERR_HIP = 2
PCMS_ERR_NOMEM = 3
PCMS_ERR_UNDERDETERMINED = 4
PCMS_ERR_SINGULAR = 5
PCMS_ERR_RADIUS_EXHAUSTED = 6

TGT_OK, TGT_UNDERDETERMINED, TGT_SINGULAR, TGT_RADIUS_EXHAUSTED, TGT_CAPPED = 0, 1, 2, 3, 0x10
RADIUS_FIXED, RADIUS_KNN, RADIUS_GROW = 0, 1, 2
WEIGHT_WENDLAND_C2, WEIGHT_C4, WEIGHT_GAUSSIAN, WEIGHT_CONST, WEIGHT_IMQ, WEIGHT_NO_OP = range(6)
FP64, MIXED, MIXED_REFINE = 0, 1, 2
ASYNC = 0x1
PROFILE = 0x2
LBVH = 0x4

EXPORTED = ("pcms_mls_opts_default", "pcms_grid_build", "pcms_grid_free", "pcms_neighbors",
            "pcms_mls_transfer", "pcms_mls_transfer_grid", "pcms_last_phase_ms", "pcms_version",
            "pcms_last_error", "pcms_batch_opts_default", "pcms_batch_plan_create",
            "pcms_batch_plan_exec", "pcms_batch_plan_free", "pcms_autotune",
            "pcms_operator_build", "pcms_operator_apply", "pcms_operator_export",
            "pcms_operator_width", "pcms_operator_free", "pcms_mls_transfer_grid_noalloc",
            "pcms_noalloc_scratch_bytes", "pcms_workspace_query", "pcms_phase_ms_sum",
            "pcms_lbvh_build", "pcms_grid_is_lbvh")


class PcmsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pcms error {code}: {msg}")
        self.code = code


class Radius(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("k", ctypes.c_int32), ("n_min", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("r", ctypes.c_double)]


class MlsOpts(ctypes.Structure):
    _fields_ = [("weight", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("lam", ctypes.c_double), ("flags", ctypes.c_uint32), ("block", ctypes.c_int32),
                ("summary", ctypes.c_void_p)]


class Problem(ctypes.Structure):
    _fields_ = [("src", ctypes.c_void_p), ("n_src", ctypes.c_int64), ("dim", ctypes.c_int32),
                ("basis_degree", ctypes.c_int32), ("src_vals", ctypes.c_void_p),
                ("n_fields", ctypes.c_int32), ("k_cap", ctypes.c_int32), ("tgt", ctypes.c_void_p),
                ("n_tgt", ctypes.c_int64), ("radius", Radius), ("inv_scale", ctypes.c_void_p),
                ("tgt_vals", ctypes.c_void_p), ("status", ctypes.c_void_p)]


class BatchOpts(ctypes.Structure):
    _fields_ = [("weight", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("lam", ctypes.c_double), ("block", ctypes.c_int32),
                ("cell_factor", ctypes.c_double), ("tune_cache", ctypes.c_char_p)]


class Workspace(ctypes.Structure):
    _fields_ = [("grid_bytes", ctypes.c_size_t), ("grid_build_bytes", ctypes.c_size_t),
                ("transfer_bytes", ctypes.c_size_t), ("transfer_grid_bytes", ctypes.c_size_t),
                ("operator_apply_bytes", ctypes.c_size_t), ("noalloc_limit", ctypes.c_size_t),
                ("lbvh_bytes", ctypes.c_size_t), ("lbvh_build_bytes", ctypes.c_size_t)]


class TuneResult(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("cell_factor", ctypes.c_double),
                ("ms", ctypes.c_float)]


_lib = None


def lib() -> ctypes.CDLL:
    """Loads libpcms_mls.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2510_18838_amd/build.py "
                          "(or __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i64, i32, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    L.pcms_mls_opts_default.argtypes = [ctypes.POINTER(MlsOpts)]
    L.pcms_mls_opts_default.restype = None
    L.pcms_grid_build.argtypes = [P, i64, i32, P, dbl, dbl, P, ctypes.POINTER(P)]
    L.pcms_grid_build.restype = i32
    L.pcms_lbvh_build.argtypes = [P, i64, i32, P, i32, P, ctypes.POINTER(P)]
    L.pcms_lbvh_build.restype = i32
    L.pcms_grid_is_lbvh.argtypes = [P]
    L.pcms_grid_is_lbvh.restype = i32
    L.pcms_grid_free.argtypes = [P]
    L.pcms_grid_free.restype = i32
    L.pcms_neighbors.argtypes = [P, P, i64, ctypes.POINTER(Radius), i32, P, P, P, P, P, P]
    L.pcms_neighbors.restype = i32
    L.pcms_mls_transfer.argtypes = [P, i64, i32, P, i32, P, i64, i32, ctypes.POINTER(Radius), i32,
                                    P, ctypes.POINTER(MlsOpts), P, P, P]
    L.pcms_mls_transfer.restype = i32
    L.pcms_mls_transfer_grid.argtypes = [P, P, i32, P, i64, i32, ctypes.POINTER(Radius), i32,
                                         ctypes.POINTER(MlsOpts), P, P, P]
    L.pcms_mls_transfer_grid.restype = i32
    L.pcms_mls_transfer_grid_noalloc.argtypes = L.pcms_mls_transfer_grid.argtypes
    L.pcms_mls_transfer_grid_noalloc.restype = i32
    L.pcms_workspace_query.argtypes = [i64, i32, i32, i64, ctypes.POINTER(Workspace)]
    L.pcms_workspace_query.restype = i32
    L.pcms_noalloc_scratch_bytes.argtypes = []
    L.pcms_noalloc_scratch_bytes.restype = ctypes.c_size_t
    L.pcms_last_phase_ms.argtypes = [P, i32]
    L.pcms_last_phase_ms.restype = i32
    L.pcms_phase_ms_sum.argtypes = [P, i32, i32]
    L.pcms_phase_ms_sum.restype = i32
    L.pcms_version.argtypes = []
    L.pcms_version.restype = i32
    L.pcms_last_error.argtypes = []
    L.pcms_last_error.restype = ctypes.c_char_p
    L.pcms_batch_opts_default.argtypes = [ctypes.POINTER(BatchOpts)]
    L.pcms_batch_opts_default.restype = None
    L.pcms_batch_plan_create.argtypes = [ctypes.POINTER(Problem), i32, ctypes.POINTER(BatchOpts),
                                         ctypes.POINTER(P)]
    L.pcms_batch_plan_create.restype = i32
    L.pcms_batch_plan_exec.argtypes = [P, P, P]
    L.pcms_batch_plan_exec.restype = i32
    L.pcms_batch_plan_free.argtypes = [P]
    L.pcms_batch_plan_free.restype = i32
    L.pcms_autotune.argtypes = [ctypes.POINTER(Problem), i32, ctypes.POINTER(BatchOpts),
                                ctypes.c_char_p, P, ctypes.POINTER(TuneResult)]
    L.pcms_autotune.restype = i32
    L.pcms_operator_build.argtypes = [P, i64, i32, P, i64, i32, ctypes.POINTER(Radius), i32, P,
                                      ctypes.POINTER(MlsOpts), P, P, ctypes.POINTER(P)]
    L.pcms_operator_build.restype = i32
    L.pcms_operator_apply.argtypes = [P, P, i32, P, P]
    L.pcms_operator_apply.restype = i32
    L.pcms_operator_export.argtypes = [P, i32, P, P, P, P]
    L.pcms_operator_export.restype = i32
    L.pcms_operator_width.argtypes = [P]
    L.pcms_operator_width.restype = i32
    L.pcms_operator_free.argtypes = [P]
    L.pcms_operator_free.restype = i32
    _lib = L
    return L


def last_error() -> str:
    return lib().pcms_last_error().decode()


PHASES = ("grid_build", "target_order", "field_gather", "search_fit", "output_transpose")


def last_phase_ms() -> dict:
    """Phase times (ms) of this thread's last call made with the PROFILE flag."""
    buf = (ctypes.c_float * len(PHASES))()
    n = lib().pcms_last_phase_ms(ctypes.cast(buf, ctypes.c_void_p), len(PHASES))
    return {PHASES[i]: float(buf[i]) for i in range(n)}


def phase_ms_sum(reset: bool = True):
    """(calls, {phase: summed ms}) over this thread's profiled calls since the
    last reset."""
    buf = (ctypes.c_double * len(PHASES))()
    n = lib().pcms_phase_ms_sum(ctypes.cast(buf, ctypes.c_void_p), len(PHASES), int(reset))
    if n < 0:
        raise PcmsError(PCMS_ERR_HIP, last_error())
    return n, {PHASES[i]: float(buf[i]) for i in range(len(PHASES))}


def _check(code: int, allow=()):
    if code != PCMS_OK and code not in allow:
        raise PcmsError(code, last_error())
    return code


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _is_gpu(t: torch.Tensor) -> bool:
    return t.is_cuda


def _dev(t: torch.Tensor, dtype, name, shape=None, device=None):
    """Checks that t is a contiguous tensor of `dtype` on a GPU device (on
    `device` if given) with the given shape (None entries are free).  The C
    interface receives bare pointers, so a wrong shape here would become an
    out-of-bounds device access; it raises ValueError instead."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if shape is not None and (t.dim() != len(shape) or
                              any(w is not None and int(v) != int(w)
                                  for v, w in zip(t.shape, shape))):
        want = "(" + ", ".join("*" if w is None else str(int(w)) for w in shape) + ")"
        raise ValueError(f"{name} must have shape {want}, got {tuple(t.shape)}")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if not _is_gpu(t):
        raise ValueError(f"{name} must be a CUDA/HIP tensor, got one on {t.device}")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, the other arguments on {device}")
    return t


def _points(t: torch.Tensor, name, dim=None, device=None):
    """[n][dim] float64 points, 1 <= dim <= 5."""
    _dev(t, torch.float64, name, shape=(None, dim), device=device)
    if not 1 <= t.shape[1] <= 5:
        raise ValueError(f"{name} must have 1 to 5 columns, got {t.shape[1]}")
    return t


def _fields(t: torch.Tensor, n: int, name, device=None):
    """Field values [n_fields][n] (or [n] for one field), float64."""
    if isinstance(t, torch.Tensor) and t.dim() == 1:
        _dev(t, torch.float64, name, shape=(n,), device=device)
        return t.view(1, -1)
    _dev(t, torch.float64, name, shape=(None, n), device=device)
    if t.shape[0] < 1:
        raise ValueError(f"{name} must hold at least one field")
    return t


def _outputs(out, status, nf: int, n_tgt: int, device):
    """Caller-supplied or new output buffers [nf][n_tgt] float64 and [n_tgt] uint8."""
    if out is None:
        out = torch.empty((nf, n_tgt), dtype=torch.float64, device=device)
    else:
        _dev(out, torch.float64, "out", shape=(nf, n_tgt), device=device)
    if status is None:
        status = torch.empty(n_tgt, dtype=torch.uint8, device=device)
    else:
        _dev(status, torch.uint8, "status", shape=(n_tgt,), device=device)
    return out, status


def radius(mode=RADIUS_FIXED, r=0.0, k=0, n_min=0, max_iter=40) -> Radius:
    return Radius(int(mode), int(k), int(n_min), int(max_iter), float(r))


def opts(weight=WEIGHT_WENDLAND_C2, precision=FP64, lam=0.0, flags=0, block=0,
         summary: Optional[torch.Tensor] = None) -> MlsOpts:
    o = MlsOpts()
    lib().pcms_mls_opts_default(ctypes.byref(o))
    o.weight, o.precision, o.lam, o.flags, o.block = weight, precision, lam, flags, block
    o.summary = None if summary is None else summary.data_ptr()
    return o


def num_monomials(dim: int, degree: int) -> int:
    return math.comb(dim + degree, degree)


class Grid:
    """Owning wrapper of a pcms_grid handle (a uniform grid or an LBVH)."""

    def __init__(self, handle: ctypes.c_void_p, n_src: int, dim: int):
        self.handle, self.n_src, self.dim = handle, n_src, dim

    @property
    def is_lbvh(self) -> bool:
        return bool(lib().pcms_grid_is_lbvh(self.handle))

    def free(self):
        if self.handle:
            lib().pcms_grid_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _host_scale(inv_scale, dim):
    if inv_scale is None:
        return None, None
    arr = (ctypes.c_double * dim)(*[float(x) for x in inv_scale])
    return arr, ctypes.cast(arr, ctypes.c_void_p)


def pcms_grid_build(src: torch.Tensor, inv_scale=None, cell_width=0.0, pts_per_cell=0.0,
                    stream=None) -> Grid:
    _points(src, "src")
    n, dim = src.shape
    keep, g = _host_scale(inv_scale, dim)
    h = ctypes.c_void_p()
    _check(lib().pcms_grid_build(_ptr(src), n, dim, g, float(cell_width), float(pts_per_cell),
                                 _stream(stream), ctypes.byref(h)))
    return Grid(h, n, dim)


def pcms_lbvh_build(src: torch.Tensor, inv_scale=None, max_leaf=0, stream=None) -> Grid:
    """LBVH over the sources (leaves of at most max_leaf sources, 0 = the
    library default), usable wherever a grid is."""
    _points(src, "src")
    n, dim = src.shape
    keep, g = _host_scale(inv_scale, dim)
    h = ctypes.c_void_p()
    _check(lib().pcms_lbvh_build(_ptr(src), n, dim, g, int(max_leaf), _stream(stream),
                                 ctypes.byref(h)))
    return Grid(h, n, dim)


def pcms_neighbors(grid: Grid, tgt: torch.Tensor, rad: Radius, k_cap: int, stream=None,
                   allow_status_errors=True):
    """Returns dict(nbr [n_tgt, k_cap] int32, n_kept, n_found, r2, status, code)."""
    _points(tgt, "tgt", dim=grid.dim)
    n = tgt.shape[0]
    dev = tgt.device
    nbr = torch.full((n, k_cap), -1, dtype=torch.int32, device=dev)
    n_kept = torch.zeros(n, dtype=torch.int32, device=dev)
    n_found = torch.zeros(n, dtype=torch.int32, device=dev)
    r2 = torch.zeros(n, dtype=torch.float64, device=dev)
    st = torch.zeros(n, dtype=torch.uint8, device=dev)
    allow = (PCMS_ERR_RADIUS_EXHAUSTED,) if allow_status_errors else ()
    code = _check(lib().pcms_neighbors(grid.handle, _ptr(tgt), n, ctypes.byref(rad), int(k_cap),
                                       _stream(stream), _ptr(nbr), _ptr(n_kept), _ptr(n_found),
                                       _ptr(r2), _ptr(st)), allow)
    return dict(nbr=nbr, n_kept=n_kept, n_found=n_found, r2=r2, status=st, code=code)


_STATUS_CODES = (PCMS_ERR_UNDERDETERMINED, PCMS_ERR_SINGULAR, PCMS_ERR_RADIUS_EXHAUSTED)


def pcms_mls_transfer(src: torch.Tensor, src_vals: torch.Tensor, tgt: torch.Tensor,
                      basis_degree: int, rad: Radius, k_cap: int, inv_scale=None,
                      o: Optional[MlsOpts] = None, stream=None, out: Optional[torch.Tensor] = None,
                      status: Optional[torch.Tensor] = None, allow_status_errors=True):
    """One-shot transfer.  Returns (tgt_vals [n_fields, n_tgt], status [n_tgt], code)."""
    _points(src, "src")
    n_src, dim = src.shape
    _points(tgt, "tgt", dim=dim, device=src.device)
    vals2 = _fields(src_vals, n_src, "src_vals", device=src.device)
    nf = vals2.shape[0]
    n_tgt = tgt.shape[0]
    out, status = _outputs(out, status, nf, n_tgt, src.device)
    keep, g = _host_scale(inv_scale, dim)
    o = opts() if o is None else o
    allow = _STATUS_CODES if allow_status_errors else ()
    code = _check(lib().pcms_mls_transfer(_ptr(src), n_src, dim, _ptr(vals2), nf, _ptr(tgt), n_tgt,
                                          int(basis_degree), ctypes.byref(rad), int(k_cap), g,
                                          ctypes.byref(o), _stream(stream), _ptr(out),
                                          _ptr(status)), allow)
    return out, status, code


def pcms_mls_transfer_grid(grid: Grid, src_vals: torch.Tensor, tgt: torch.Tensor,
                           basis_degree: int, rad: Radius, k_cap: int,
                           o: Optional[MlsOpts] = None, stream=None,
                           out: Optional[torch.Tensor] = None,
                           status: Optional[torch.Tensor] = None, allow_status_errors=True):
    _points(tgt, "tgt", dim=grid.dim)
    vals2 = _fields(src_vals, grid.n_src, "src_vals", device=tgt.device)
    nf = vals2.shape[0]
    n_tgt = tgt.shape[0]
    out, status = _outputs(out, status, nf, n_tgt, tgt.device)
    o = opts() if o is None else o
    allow = _STATUS_CODES if allow_status_errors else ()
    code = _check(lib().pcms_mls_transfer_grid(grid.handle, _ptr(vals2), nf, _ptr(tgt), n_tgt,
                                               int(basis_degree), ctypes.byref(rad), int(k_cap),
                                               ctypes.byref(o), _stream(stream), _ptr(out),
                                               _ptr(status)), allow)
    return out, status, code


def pcms_mls_transfer_grid_noalloc(grid: Grid, src_vals: torch.Tensor, tgt: torch.Tensor,
                                   basis_degree: int, rad: Radius, k_cap: int,
                                   out: torch.Tensor, status: torch.Tensor,
                                   o: Optional[MlsOpts] = None, stream=None,
                                   allow_status_errors=True):
    """The allocation-free transfer on a prebuilt grid: the caller passes the
    output buffers, and the library's work space is its fixed device array.
    Returns (tgt_vals, status, code)."""
    _points(tgt, "tgt", dim=grid.dim)
    vals2 = _fields(src_vals, grid.n_src, "src_vals", device=tgt.device)
    nf = vals2.shape[0]
    n_tgt = tgt.shape[0]
    _dev(out, torch.float64, "out", shape=(nf, n_tgt), device=tgt.device)
    _dev(status, torch.uint8, "status", shape=(n_tgt,), device=tgt.device)
    o = opts() if o is None else o
    allow = _STATUS_CODES if allow_status_errors else ()
    code = _check(lib().pcms_mls_transfer_grid_noalloc(grid.handle, _ptr(vals2), nf, _ptr(tgt),
                                                       n_tgt, int(basis_degree), ctypes.byref(rad),
                                                       int(k_cap), ctypes.byref(o),
                                                       _stream(stream), _ptr(out), _ptr(status)),
                  allow)
    return out, status, code


def pcms_workspace_query(n_src: int, dim: int, n_fields: int, n_tgt: int) -> dict:
    """Device bytes the calls take for a problem of these sizes (host-only)."""
    w = Workspace()
    _check(lib().pcms_workspace_query(int(n_src), int(dim), int(n_fields), int(n_tgt),
                                      ctypes.byref(w)))
    return {name: int(getattr(w, name)) for name, _ in Workspace._fields_}


def noalloc_scratch_bytes() -> int:
    return int(lib().pcms_noalloc_scratch_bytes())


def radius_of(prob) -> Radius:
    """Radius spec of a synth.Problem."""
    return radius(prob.mode, prob.radius, prob.k, prob.n_min, prob.max_iter)


# --- batched transfer ------------------------------------------------------

def batch_opts(weight=WEIGHT_WENDLAND_C2, precision=MIXED_REFINE, lam=0.0, block=0,
               cell_factor=0.0, tune_cache: Optional[str] = None) -> BatchOpts:
    o = BatchOpts()
    lib().pcms_batch_opts_default(ctypes.byref(o))
    o.weight, o.precision, o.lam, o.block, o.cell_factor = weight, precision, lam, block, cell_factor
    o.tune_cache = None if tune_cache is None else tune_cache.encode()
    return o


class BatchProblem:
    """Device tensors of one problem of a batch (kept alive by the plan)."""

    def __init__(self, src, src_vals, tgt, basis_degree, rad: Radius, k_cap, inv_scale=None,
                 out=None, status=None):
        _points(src, "src")
        _points(tgt, "tgt", dim=src.shape[1], device=src.device)
        self.src, self.tgt = src, tgt
        self.src_vals = _fields(src_vals, src.shape[0], "src_vals", device=src.device)
        nf, n_tgt = self.src_vals.shape[0], tgt.shape[0]
        self.out, self.status = _outputs(out, status, nf, n_tgt, src.device)
        self.basis_degree, self.rad, self.k_cap = int(basis_degree), rad, int(k_cap)
        self.inv_scale = inv_scale

    def c_struct(self):
        n_src, dim = self.src.shape
        keep, g = _host_scale(self.inv_scale, dim)
        p = Problem(self.src.data_ptr(), n_src, dim, self.basis_degree, self.src_vals.data_ptr(),
                    self.src_vals.shape[0], self.k_cap, self.tgt.data_ptr(), self.tgt.shape[0],
                    self.rad, None if g is None else g.value, self.out.data_ptr(),
                    self.status.data_ptr())
        return p, keep


def _problem_array(problems):
    arr = (Problem * len(problems))()
    keep = []
    for i, bp in enumerate(problems):
        arr[i], k = bp.c_struct()
        keep.append(k)
    return arr, keep


class BatchPlan:
    """Owning wrapper of a pcms_batch_plan; holds the problems' tensors."""

    def __init__(self, problems, o: Optional[BatchOpts] = None):
        self.problems = list(problems)
        arr, self._keep = _problem_array(self.problems)
        self._opts = batch_opts() if o is None else o
        h = ctypes.c_void_p()
        _check(lib().pcms_batch_plan_create(arr, len(self.problems), ctypes.byref(self._opts),
                                            ctypes.byref(h)))
        self.handle = h

    def exec(self, stream=None, summary: Optional[torch.Tensor] = None,
             allow_status_errors=True) -> int:
        allow = _STATUS_CODES if allow_status_errors else ()
        return _check(lib().pcms_batch_plan_exec(self.handle, _stream(stream), _ptr(summary)),
                      allow)

    def free(self):
        if getattr(self, "handle", None):
            lib().pcms_batch_plan_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def pcms_autotune(problems, o: Optional[BatchOpts] = None, cache_path: Optional[str] = None,
                  stream=None) -> TuneResult:
    arr, keep = _problem_array(list(problems))
    o = batch_opts() if o is None else o
    res = TuneResult()
    _check(lib().pcms_autotune(arr, len(problems), ctypes.byref(o),
                               None if cache_path is None else cache_path.encode(),
                               _stream(stream), ctypes.byref(res)))
    return res


def batch_problem_of(prob, dev, out=None) -> BatchProblem:
    """BatchProblem of a synth.Problem, with its arrays copied to `dev`."""
    src = torch.from_numpy(prob.src).to(dev)
    vals = torch.from_numpy(prob.vals).to(dev)
    tgt = torch.from_numpy(prob.tgt).to(dev)
    return BatchProblem(src, vals, tgt, prob.degree, radius_of(prob), prob.k_cap,
                        inv_scale=prob.inv_scale, out=out)


# --- precomputed transfer operator ----------------------------------------

class Operator:
    """Owning wrapper of a pcms_operator (shape functions of fixed clouds)."""

    def __init__(self, src: torch.Tensor, tgt: torch.Tensor, basis_degree: int, rad: Radius,
                 k_cap: int, inv_scale=None, o: Optional[MlsOpts] = None, stream=None,
                 status: Optional[torch.Tensor] = None, allow_status_errors=True):
        _points(src, "src")
        n_src, dim = src.shape
        _points(tgt, "tgt", dim=dim, device=src.device)
        self.n_src, self.n_tgt, self.k_cap = n_src, tgt.shape[0], int(k_cap)
        self.device = src.device
        if status is None:
            status = torch.empty(self.n_tgt, dtype=torch.uint8, device=src.device)
        else:
            _dev(status, torch.uint8, "status", shape=(self.n_tgt,), device=src.device)
        self.status = status
        keep, g = _host_scale(inv_scale, dim)
        o = opts() if o is None else o
        h = ctypes.c_void_p()
        allow = _STATUS_CODES if allow_status_errors else ()
        self.code = _check(lib().pcms_operator_build(_ptr(src), n_src, dim, _ptr(tgt), self.n_tgt,
                                                     int(basis_degree), ctypes.byref(rad),
                                                     int(k_cap), g, ctypes.byref(o),
                                                     _stream(stream), _ptr(self.status),
                                                     ctypes.byref(h)), allow)
        self.handle = h
        self.width = lib().pcms_operator_width(h)

    def apply(self, src_vals: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None):
        vals2 = _fields(src_vals, self.n_src, "src_vals", device=self.device)
        nf = vals2.shape[0]
        if out is None:
            out = torch.empty((nf, self.n_tgt), dtype=torch.float64, device=self.device)
        else:
            _dev(out, torch.float64, "out", shape=(nf, self.n_tgt), device=self.device)
        _check(lib().pcms_operator_apply(self.handle, _ptr(vals2), nf, _stream(stream), _ptr(out)))
        return out

    def export(self, stream=None):
        """(n_kept [n_tgt], cols [n_tgt, k_cap], weights [n_tgt, k_cap]) device tensors."""
        dev = self.status.device
        n_kept = torch.empty(self.n_tgt, dtype=torch.int32, device=dev)
        cols = torch.empty((self.n_tgt, self.k_cap), dtype=torch.int32, device=dev)
        w = torch.empty((self.n_tgt, self.k_cap), dtype=torch.float64, device=dev)
        _check(lib().pcms_operator_export(self.handle, self.k_cap, _stream(stream), _ptr(n_kept),
                                          _ptr(cols), _ptr(w)))
        return n_kept, cols, w

    def free(self):
        if getattr(self, "handle", None):
            lib().pcms_operator_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
