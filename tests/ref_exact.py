"""Independent tiny-input references used to pin the oracle.

Nothing here imports the oracle or the HIP library.  Distances are the same
reading of the selection predicate as the oracle's (a fused multiply-add
chain over dimensions in FP64), but evaluated exactly with rational
arithmetic and rounded once per fused step, so the neighbour sets are exact.
The fits use NumPy's QR/SVD least-squares and dense solves on the explicit
(weighted) Vandermonde matrix, not normal equations.
"""
from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np


def fma(a: float, b: float, c: float) -> float:
    """Correctly rounded a*b + c (float() of a Fraction rounds to nearest even)."""
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def d2_exact(t, s, g=None) -> float:
    dim = len(t)
    g = [1.0] * dim if g is None else [float(x) for x in g]
    u = (float(t[0]) - float(s[0])) * g[0]
    acc = u * u
    for k in range(1, dim):
        u = (float(t[k]) - float(s[k])) * g[k]
        acc = fma(u, u, acc)
    return acc


def d2_matrix(tgt, src, g=None) -> np.ndarray:
    return np.array([[d2_exact(t, s, g) for s in src] for t in tgt])


def brute_lists(tgt, src, mode, r=0.0, k=0, n_min=0, max_iter=40, k_cap=32, g=None):
    """Exact neighbour lists by testing every pair.  Returns the same dict keys as the oracle."""
    D = d2_matrix(tgt, src, g)
    n_tgt = len(tgt)
    nbr = np.full((n_tgt, k_cap), -1, np.int32)
    n_kept = np.zeros(n_tgt, np.int32)
    n_found = np.zeros(n_tgt, np.int32)
    r2 = np.zeros(n_tgt)
    st = np.zeros(n_tgt, np.uint8)
    for i in range(n_tgt):
        row = D[i]
        status = 0
        if mode == 0:
            rr = r * r
        elif mode == 2:
            rr = r * r
            it = 0
            while (row < rr).sum() < n_min and it < max_iter:
                rr = 2.0 * rr
                it += 1
            if (row < rr).sum() < n_min:
                status = 3
        else:
            rr = float(np.sort(row)[k - 1])
        sel = [j for j in range(len(src)) if row[j] < rr]
        n_found[i] = len(sel)
        if len(sel) > k_cap:
            sel = sorted(sel, key=lambda j: (row[j], j))[:k_cap]
            status |= 0x10
        sel = sorted(sel)
        nbr[i, :len(sel)] = sel
        n_kept[i] = len(sel)
        r2[i] = rr
        st[i] = status
    return dict(nbr=nbr, n_kept=n_kept, n_found=n_found, r2=r2, status=st)


def exponents(dim: int, degree: int):
    """Exponent tuples of all monomials of total degree <= degree (any order)."""
    out = []
    for deg in range(degree + 1):
        for combo in itertools.combinations_with_replacement(range(dim), deg):
            e = [0] * dim
            for a in combo:
                e[a] += 1
            out.append(tuple(e))
    return out


def vandermonde(xi: np.ndarray, degree: int) -> np.ndarray:
    ex = exponents(xi.shape[1], degree)
    return np.stack([np.prod(xi ** np.array(e), axis=1) for e in ex], axis=1)


def wendland_c2(q):
    q = np.asarray(q, dtype=np.float64)
    return np.where(q < 1.0, (1.0 - q) ** 4 * (4.0 * q + 1.0), 0.0)


def wls_value(src_sel, f_sel, t, h, w, degree, lam=0.0, g=None):
    """Value at t of the weighted (ridge) least-squares polynomial, via lstsq on
    the row-scaled Vandermonde matrix stacked on sqrt(lambda) I."""
    dim = src_sel.shape[1]
    g = np.ones(dim) if g is None else np.asarray(g)
    xi = (src_sel - t) * g / h
    V = vandermonde(xi, degree)
    sw = np.sqrt(w)
    A = V * sw[:, None]
    b = f_sel * sw
    if lam > 0.0:
        m = V.shape[1]
        A = np.vstack([A, np.sqrt(lam) * np.eye(m)])
        b = np.concatenate([b, np.zeros(m)])
    c, *_ = np.linalg.lstsq(A, b, rcond=None)
    # the constant monomial is the first exponent tuple
    return c[0], np.linalg.cond(A)
