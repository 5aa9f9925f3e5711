"""Seeded synthetic inputs for the point-cloud field-transfer workloads.

This module only draws random numbers and evaluates the analytic test fields
that stand in for the paper's simulation data (the WEST, LTX, XGCm and GNET
meshes and fields of Sections 3.2.1 and 5 are not available).  It holds none
of the transfer method's arithmetic: no neighbour search, no weights, no
least-squares fitting.  Both the HIP library's tests and the CPU oracle take
their inputs from here.

Workloads (sizes as named in the benchmark configuration list):

* ``c1``  2-D, 2,000 uniform sources, 1,500 uniform targets, linear basis,
  fixed support radius 0.06, neighbour cap 32, one field
  sin(2 pi x) cos(2 pi y).
* ``c2``  2-D, 10^6 sources on a jittered 1000x1000 lattice (jitter +-0.3
  cell), 10^6 uniform targets, quadratic basis, radius 3.5 cells, cap 48,
  four random trigonometric fields (field 0 is the paper's Eq. 4 field).
* ``c3``  3-D, 4*10^6 sources from an 8-component Gaussian mixture with a
  10x density contrast, 4*10^6 uniform targets, quadratic basis, radius =
  distance to the 40th nearest source, cap 64, eight fields.
* ``c4``  512 independent problems of uneven size (log-uniform 1k..200k
  points), 2-D/3-D, linear/quadratic, 1..16 fields, growing radius.
* ``c5``  5-D, 2*10^6 sources and targets: 3 uniform dimensions and 2
  truncated-normal dimensions, per-dimension standardising metric, growing
  radius aiming at ~64 neighbours, cap 96, four Maxwellian-like fields.

Every draw uses ``numpy.random.SeedSequence([2510, 18838, cfg_id])`` spawned
into (sources, targets, fields, misc) streams, so a workload is a pure
function of its id and size parameters.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# radius modes, same numbering as the C interface
FIXED, KNN, GROW = 0, 1, 2


@dataclass
class Problem:
    """One transfer instance: source cloud, fields, target cloud, options."""
    name: str
    src: np.ndarray            # [n_src, dim] float64, C order
    vals: np.ndarray           # [n_fields, n_src] float64, C order
    tgt: np.ndarray            # [n_tgt, dim] float64, C order
    degree: int
    mode: int
    radius: float = 0.0        # FIXED radius, or GROW initial radius
    k: int = 0                 # KNN order
    n_min: int = 0             # GROW minimum neighbour count
    max_iter: int = 40         # GROW doubling limit
    k_cap: int = 32
    inv_scale: Optional[np.ndarray] = None   # [dim] metric scaling (None = 1)

    @property
    def dim(self) -> int:
        return self.src.shape[1]

    @property
    def n_fields(self) -> int:
        return self.vals.shape[0]

    @property
    def m(self) -> int:
        return math.comb(self.dim + self.degree, self.degree)


def _streams(cfg_id, *extra):
    ss = np.random.SeedSequence([2510, 18838, cfg_id, *extra])
    return [np.random.default_rng(s) for s in ss.spawn(4)]


# ---------------------------------------------------------------------------
# analytic fields
# ---------------------------------------------------------------------------

def eq4_field(x: np.ndarray) -> np.ndarray:
    """The paper's smooth test field f = sin(x) cos(y) + 2 (Section 3.2.1, Eq. 4)."""
    return np.sin(x[:, 0]) * np.cos(x[:, 1]) + 2.0


def _wave_vectors(d: int, deg: int) -> np.ndarray:
    """Integer wave vectors k with 1 <= |k|_1 <= deg whose first non-zero entry is positive."""
    out = []
    rng = range(-deg, deg + 1)
    for k in np.array(np.meshgrid(*([list(rng)] * d), indexing="ij")).reshape(d, -1).T:
        s = int(np.abs(k).sum())
        if s < 1 or s > deg:
            continue
        nz = k[np.nonzero(k)[0][0]]
        if nz > 0:
            out.append(k)
    return np.array(out, dtype=np.float64)


def trig_field(rng: np.random.Generator, x: np.ndarray, deg: int) -> np.ndarray:
    """Random trigonometric polynomial a0 + sum a_k cos(2 pi k.x) + b_k sin(2 pi k.x).

    Coefficients a_k, b_k ~ N(0, 1) / (1 + |k|^2); a0 ~ 2 + N(0, 1).
    """
    import torch   # multi-threaded host evaluation of the large fields

    d = x.shape[1]
    K = _wave_vectors(d, deg)
    amp = 1.0 / (1.0 + (K * K).sum(1))
    a = rng.standard_normal(len(K)) * amp
    b = rng.standard_normal(len(K)) * amp
    a0 = 2.0 + rng.standard_normal()
    out = np.full(x.shape[0], a0)
    Kt = torch.from_numpy(2.0 * np.pi * K.T.copy())
    at, bt = torch.from_numpy(a), torch.from_numpy(b)
    chunk = 1 << 18
    for s in range(0, x.shape[0], chunk):
        ph = torch.from_numpy(np.ascontiguousarray(x[s:s + chunk])) @ Kt
        out[s:s + chunk] += (torch.cos(ph) @ at + torch.sin(ph) @ bt).numpy()
    return out


def _fields(rng, x, n_fields, deg, eq4_first=True):
    vals = np.empty((n_fields, x.shape[0]))
    for l in range(n_fields):
        if l == 0 and eq4_first:
            vals[l] = eq4_field(x)
        else:
            vals[l] = trig_field(rng, x, deg)
    return vals


# ---------------------------------------------------------------------------
# configurations
# ---------------------------------------------------------------------------

def c1() -> Problem:
    rs, rt, rf, _ = _streams(1)
    src = rs.uniform(0.0, 1.0, (2000, 2))
    tgt = rt.uniform(0.0, 1.0, (1500, 2))
    vals = (np.sin(2 * np.pi * src[:, 0]) * np.cos(2 * np.pi * src[:, 1]))[None, :].copy()
    return Problem("c1", src, vals, tgt, degree=1, mode=FIXED, radius=0.06, k_cap=32)


def c2(n_side: int = 1000, n_tgt: Optional[int] = None) -> Problem:
    """Jittered lattice; ``n_side`` scales it down for tests (radius stays 3.5 cells)."""
    rs, rt, rf, _ = _streams(2)
    n_tgt = n_side * n_side if n_tgt is None else n_tgt
    i, j = np.meshgrid(np.arange(n_side), np.arange(n_side), indexing="ij")
    base = np.stack([i.ravel(), j.ravel()], 1).astype(np.float64)
    src = (base + 0.5 + rs.uniform(-0.3, 0.3, base.shape)) / n_side
    tgt = rt.uniform(0.0, 1.0, (n_tgt, 2))
    vals = _fields(rf, src, 4, 4)
    return Problem("c2", np.ascontiguousarray(src), vals, tgt, degree=2, mode=FIXED,
                   radius=3.5 / n_side, k_cap=48)


def _mixture_params(rm: np.random.Generator, contrast: float = 10.0):
    mu = rm.uniform(0.2, 0.8, (8, 3))
    sig = rm.uniform(0.06, 0.12, 8)
    g = (np.arange(16) + 0.5) / 16.0
    cc = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)

    def gauss_sum(x):
        acc = np.zeros(x.shape[0])
        for c in range(8):
            r2 = ((x - mu[c]) ** 2).sum(1)
            acc += np.exp(-0.5 * r2 / sig[c] ** 2) / ((2 * np.pi) ** 1.5 * sig[c] ** 3) / 8.0
        return acc

    gs = gauss_sum(cc)
    lo, hi = 0.0, 1.0
    for _ in range(200):                    # bisection on the mixture weight
        w = 0.5 * (lo + hi)
        rho = (1.0 - w) + w * gs
        if rho.max() / rho.min() > contrast:
            hi = w
        else:
            lo = w
    return mu, sig, 0.5 * (lo + hi)


def mixture_points(rng: np.random.Generator, n: int, mu, sig, w) -> np.ndarray:
    """Rejection sampling of (1-w) U[0,1]^3 + w * mean_c N(mu_c, sig_c^2 I) restricted to the cube."""
    out = np.empty((0, 3))
    while out.shape[0] < n:
        need = n - out.shape[0]
        b = int(need * 1.3) + 1024
        comp = rng.integers(0, 8, b)
        is_g = rng.uniform(0.0, 1.0, b) < w
        x = rng.uniform(0.0, 1.0, (b, 3))
        gz = rng.standard_normal((b, 3)) * sig[comp][:, None] + mu[comp]
        x[is_g] = gz[is_g]
        ok = np.all((x >= 0.0) & (x <= 1.0), axis=1)
        out = np.concatenate([out, x[ok]])
    return np.ascontiguousarray(out[:n])


def c3(n_src: int = 4_000_000, n_tgt: Optional[int] = None, n_fields: int = 8) -> Problem:
    rs, rt, rf, rm = _streams(3)
    n_tgt = n_src if n_tgt is None else n_tgt
    mu, sig, w = _mixture_params(rm)
    src = mixture_points(rs, n_src, mu, sig, w)
    tgt = rt.uniform(0.0, 1.0, (n_tgt, 3))
    vals = _fields(rf, src, n_fields, 2)
    return Problem("c3", src, vals, tgt, degree=2, mode=KNN, k=40, k_cap=64)


_KBAR = {(2, 1): (20, 32), (2, 2): (38, 48), (3, 1): (24, 32), (3, 2): (40, 64)}


def unit_ball_volume(d: int) -> float:
    return math.pi ** (d / 2) / math.gamma(d / 2 + 1)


def c4_problem(b: int, size_scale: float = 1.0) -> Problem:
    """Problem ``b`` of the 512-problem batch (``size_scale`` < 1 shrinks it for tests)."""
    rs, rt, rf, rm = _streams(4, b)
    lo, hi = math.log(1e3), math.log(2e5)
    n_src = max(16, int(round(math.exp(rm.uniform(lo, hi)) * size_scale)))
    n_tgt = max(1, int(round(math.exp(rm.uniform(lo, hi)) * size_scale)))
    d = int(rm.integers(2, 4))
    p = int(rm.integers(1, 3))
    nf = int(rm.integers(1, 17))
    kbar, kcap = _KBAR[(d, p)]
    m = math.comb(d + p, p)
    r0 = (kbar / (n_src * unit_ball_volume(d))) ** (1.0 / d)
    src = rs.uniform(0.0, 1.0, (n_src, d))
    tgt = rt.uniform(0.0, 1.0, (n_tgt, d))
    vals = np.stack([trig_field(rf, src, 2) for _ in range(nf)])
    return Problem(f"c4_{b}", src, vals, tgt, degree=p, mode=GROW, radius=r0,
                   n_min=2 * m, k_cap=kcap)


def c4(n_problems: int = 512, size_scale: float = 1.0) -> List[Problem]:
    return [c4_problem(b, size_scale) for b in range(n_problems)]


def _c5_points(rng, n):
    u = rng.uniform(0.0, 1.0, (n, 3))
    v = rng.standard_normal((n, 2))
    bad = np.abs(v) > 4.0
    while bad.any():
        v[bad] = rng.standard_normal(int(bad.sum()))
        bad = np.abs(v) > 4.0
    return np.ascontiguousarray(np.concatenate([u, v], 1))


def c5(n: int = 2_000_000, n_tgt: Optional[int] = None) -> Problem:
    rs, rt, rf, rm = _streams(5)
    n_tgt = n if n_tgt is None else n_tgt
    src = _c5_points(rs, n)
    tgt = _c5_points(rt, n_tgt)
    g = np.array([math.sqrt(12.0)] * 3 + [1.0, 1.0])
    e_rho = 12.0 ** -1.5 / (4.0 * math.pi)
    r0 = (64.0 / (n * e_rho * unit_ball_volume(5))) ** 0.2
    vals = np.empty((4, n))
    for l in range(4):
        vl = rf.standard_normal(2) * 0.5
        base = 2.0 + trig_field(rf, src[:, :3], 2)
        vals[l] = np.exp(-0.5 * ((src[:, 3:] - vl) ** 2).sum(1)) * base
    return Problem("c5", src, vals, tgt, degree=1, mode=GROW, radius=r0, n_min=12,
                   k_cap=96, inv_scale=g)


def by_name(name: str, **kw):
    return {"c1": c1, "c2": c2, "c3": c3, "c4": c4, "c5": c5}[name](**kw)


def uniform_problem(seed: int, n_src: int, n_tgt: int, dim: int, degree: int, mode: int,
                    n_fields: int = 1, radius: float = 0.0, k: int = 0, n_min: int = 0,
                    k_cap: int = 32, max_iter: int = 40, inv_scale=None) -> Problem:
    """Small uniform problem for tests: U[0,1]^dim clouds, trigonometric fields."""
    rs, rt, rf, _ = _streams(100, seed)
    src = rs.uniform(0.0, 1.0, (n_src, dim))
    tgt = rt.uniform(0.0, 1.0, (n_tgt, dim))
    vals = np.stack([trig_field(rf, src, 2) for _ in range(n_fields)]) if n_src else \
        np.zeros((n_fields, 0))
    g = None if inv_scale is None else np.asarray(inv_scale, dtype=np.float64)
    return Problem(f"u{seed}", src, vals, tgt, degree=degree, mode=mode, radius=radius, k=k,
                   n_min=n_min, max_iter=max_iter, k_cap=k_cap, inv_scale=g)


def roundtrip_clouds(n_src_side: int = 554, n_tgt_side: int = 782, extent: float = 4.0):
    """Two 2-D jittered lattices over [0, extent]^2 standing in for a
    triangle mesh's vertices (n_src_side^2 points) and its element centroids
    (n_tgt_side^2, about twice as many), with the field of Eq. 4 sampled on
    the first: f = sin(x) cos(y) + 2."""
    rs, rt, _, _ = _streams(6)

    def lattice(rng, n):
        i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        base = np.stack([i.ravel(), j.ravel()], 1).astype(np.float64)
        return np.ascontiguousarray((base + 0.5 + rng.uniform(-0.3, 0.3, base.shape)) * (extent / n))

    src = lattice(rs, n_src_side)
    tgt = lattice(rt, n_tgt_side)
    f = np.sin(src[:, 0]) * np.cos(src[:, 1]) + 2.0
    return src, tgt, f
