"""GPU parity of the LBVH search backend (pcms_lbvh_build, PCMS_LBVH): the
same cases and bars as the uniform grid against the FP64 oracle, and the
grid's own lists, counts, radii and statuses bit for bit."""
import numpy as np
import pytest
import torch

import parity_cases as C
from gpu_helpers import dev, gpu_neighbors, gpu_operator, gpu_transfer
from paper_2510_18838_amd import pcms, synth

pytestmark = pytest.mark.gpu


class LbvhBackend:
    def neighbors(self, prob):
        return gpu_neighbors(prob, lbvh=True)

    def transfer(self, prob, precision, weight=0, lam=0.0, block=0):
        out, st, _ = gpu_transfer(prob, precision, weight=weight, lam=lam, block=block, lbvh=True)
        return dict(out=out, status=st)

    def operator(self, prob, precision):
        return gpu_operator(prob, precision, lbvh=True)


BV = LbvhBackend()


def test_lbvh_c1():
    C.case_c1(BV)


@pytest.mark.parametrize("name", ["c2", "c3", "c5"])
def test_lbvh_scaled(name):
    C.case_scaled(BV, name)


@pytest.mark.parametrize("dim,degree,mode", C.DIM_CASES)
def test_lbvh_dimensions_and_degrees(dim, degree, mode):
    C.case_dims(BV, dim, degree, mode)


def test_lbvh_box_boundary():
    C.case_box_boundary(BV)


def test_lbvh_edge_cases():
    C.case_far_targets(BV)
    C.case_singular_exhausted(BV)
    C.case_ties(BV)
    C.case_tight_caps(BV)
    C.case_fp32_filter(BV)
    C.case_random_caps(BV)


def test_lbvh_tiny_clouds():
    """Clouds of one leaf or less (no internal node) and of a few leaves."""
    for n_src in (1, 5, 8, 9, 17, 64):
        p = synth.uniform_problem(40 + n_src, n_src, 300, 2, 0, synth.KNN, k=min(3, n_src),
                                  k_cap=8)
        C.check_lists(BV, p, f"lbvh knn n_src={n_src}")
        # a radius covering the unit square: every target keeps every source
        p = synth.uniform_problem(50 + n_src, n_src, 300, 2, 0, synth.FIXED, radius=1.5,
                                  k_cap=64)
        C.check_lists(BV, p, f"lbvh fixed n_src={n_src}")
        C.check_transfer(BV, p, f"lbvh fixed n_src={n_src}", precisions=(pcms.FP64,))


@pytest.mark.parametrize("name", ["c3", "c5"])
def test_lbvh_lists_match_grid(name):
    p = C.scaled(name)
    a, b = gpu_neighbors(p), gpu_neighbors(p, lbvh=True)
    for key in ("n_kept", "n_found", "r2", "status"):
        assert np.array_equal(a[key], b[key]), key
    for i in range(p.tgt.shape[0]):
        n = a["n_kept"][i]
        assert np.array_equal(a["nbr"][i, :n], b["nbr"][i, :n]), i


def test_lbvh_handle_paths_agree():
    """One-shot PCMS_LBVH, a prebuilt LBVH handle and the allocation-free
    call on it give bit-identical results (same tree, same sums)."""
    p = C.scaled("c5")
    a, sa, _ = gpu_transfer(p, pcms.MIXED_REFINE, lbvh=True)
    g = pcms.pcms_lbvh_build(dev(p.src), inv_scale=p.inv_scale)
    assert g.is_lbvh
    o = pcms.opts(precision=pcms.MIXED_REFINE)
    out, st, _ = pcms.pcms_mls_transfer_grid(g, dev(p.vals), dev(p.tgt), p.degree,
                                             pcms.radius_of(p), p.k_cap, o=o)
    torch.cuda.synchronize()
    assert np.array_equal(st.cpu().numpy(), sa)
    assert np.array_equal(out.cpu().numpy(), a, equal_nan=True)
    out2 = torch.empty_like(out)
    st2 = torch.empty_like(st)
    pcms.pcms_mls_transfer_grid_noalloc(g, dev(p.vals), dev(p.tgt), p.degree, pcms.radius_of(p),
                                        p.k_cap, out2, st2, o=o)
    torch.cuda.synchronize()
    assert torch.equal(st2, st)
    assert np.array_equal(out2.cpu().numpy(), a, equal_nan=True)
    g.free()


def test_lbvh_operator():
    C.case_operator(BV)
