"""Shared helpers of the GPU parity tests (no method arithmetic here)."""
from __future__ import annotations

import numpy as np
import torch

from paper_2510_18838_amd import pcms

DEV = torch.device("cuda:0")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def say(msg):
    print(msg, flush=True)


def gpu_transfer(prob, precision=pcms.FP64, tgt=None, weight=pcms.WEIGHT_WENDLAND_C2, lam=0.0,
                 block=0, stream=None, lbvh=False):
    t = prob.tgt if tgt is None else tgt
    out, st, code = pcms.pcms_mls_transfer(
        dev(prob.src), dev(prob.vals), dev(t), prob.degree, pcms.radius_of(prob), prob.k_cap,
        inv_scale=prob.inv_scale, o=pcms.opts(weight=weight, precision=precision, lam=lam,
                                               block=block, flags=pcms.LBVH if lbvh else 0),
        stream=stream)
    torch.cuda.synchronize()
    return out.cpu().numpy(), st.cpu().numpy(), code


def gpu_neighbors(prob, tgt=None, rows=None, cell_width=None, lbvh=False):
    """Neighbour lists on the GPU (on a uniform grid, or an LBVH); `rows`
    keeps only those target rows on the host."""
    t = prob.tgt if tgt is None else tgt
    cw = prob.radius if cell_width is None and prob.mode != 1 else (cell_width or 0.0)
    ppc = 0.0
    if prob.mode == 1:
        import math
        d = prob.dim
        ppc = prob.k / (math.pi ** (d / 2) / math.gamma(d / 2 + 1))
    if lbvh:
        g = pcms.pcms_lbvh_build(dev(prob.src), inv_scale=prob.inv_scale)
        assert g.is_lbvh
    else:
        g = pcms.pcms_grid_build(dev(prob.src), inv_scale=prob.inv_scale, cell_width=cw,
                                 pts_per_cell=ppc)
    r = pcms.pcms_neighbors(g, dev(t), pcms.radius_of(prob), prob.k_cap)
    torch.cuda.synchronize()
    out = {}
    for key in ("nbr", "n_kept", "n_found", "r2", "status"):
        v = r[key]
        if rows is not None:
            v = v[torch.as_tensor(rows, device=v.device)]
        out[key] = v.cpu().numpy()
    g.free()
    return out




def gpu_operator(prob, precision, lbvh=False):
    """The operator's export (original target order, k_cap slots) and the
    build's statuses, as numpy arrays."""
    op = pcms.Operator(dev(prob.src), dev(prob.tgt), prob.degree, pcms.radius_of(prob),
                       prob.k_cap, inv_scale=prob.inv_scale,
                       o=pcms.opts(precision=precision, flags=pcms.LBVH if lbvh else 0))
    n_kept, cols, w = op.export()
    torch.cuda.synchronize()
    r = dict(n_kept=n_kept.cpu().numpy(), cols=cols.cpu().numpy(), weights=w.cpu().numpy(),
             status=op.status.cpu().numpy())
    op.free()
    return r
