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
                 block=0, stream=None):
    t = prob.tgt if tgt is None else tgt
    out, st, code = pcms.pcms_mls_transfer(
        dev(prob.src), dev(prob.vals), dev(t), prob.degree, pcms.radius_of(prob), prob.k_cap,
        inv_scale=prob.inv_scale, o=pcms.opts(weight=weight, precision=precision, lam=lam,
                                               block=block), stream=stream)
    torch.cuda.synchronize()
    return out.cpu().numpy(), st.cpu().numpy(), code


def gpu_neighbors(prob, tgt=None, rows=None, cell_width=None):
    """Neighbour lists on the GPU; `rows` keeps only those target rows on the host."""
    t = prob.tgt if tgt is None else tgt
    cw = prob.radius if cell_width is None and prob.mode != 1 else (cell_width or 0.0)
    ppc = 0.0
    if prob.mode == 1:
        import math
        d = prob.dim
        ppc = prob.k / (math.pi ** (d / 2) / math.gamma(d / 2 + 1))
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


