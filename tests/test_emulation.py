"""The kernels' per-target code and grid-build pieces, compiled for the CPU
with the address and undefined-behaviour sanitisers, against the oracle.

Same cases and bars as the GPU parity tests (tests/parity_cases.py), at
smaller sizes.  This checks indexing and logic without a GPU.
"""
import numpy as np
import pytest

import emu_driver
import parity_cases as C
from paper_2510_18838_amd import synth


class EmuBackend:
    def __init__(self, group=1, lbvh=False):
        self.group, self.lbvh = group, lbvh

    def neighbors(self, prob):
        return emu_driver.run(prob, 0, group=self.group, lbvh=self.lbvh)

    def transfer(self, prob, precision, weight=0, lam=0.0, block=64):
        return emu_driver.run(prob, 1, precision=precision, weight=weight, lam=lam,
                              group=self.group, lbvh=self.lbvh)

    def operator(self, prob, precision):
        return emu_driver.run(prob, 2, precision=precision, group=self.group)


BE = EmuBackend(1)    # one lane per target, as the kernels run
BE4 = EmuBackend(4)   # four cooperating lanes: the group collectives
BV = EmuBackend(1, lbvh=True)   # the LBVH in place of the uniform grid


@pytest.fixture(scope="module", autouse=True)
def _built():
    emu_driver.build()


def test_emu_c1():
    C.case_c1(BE)


@pytest.mark.parametrize("name", ["c2", "c3", "c5"])
def test_emu_scaled(name):
    C.case_scaled(BE, name, small=True)


@pytest.mark.parametrize("sub", [1, 2, 8, 16])
def test_emu_row_slices(sub, monkeypatch):
    """Grids with dimension 0 cut into 1-16 slices per bucket width (the
    library's default is 4): the same lists and values, in 2-D and 3-D."""
    monkeypatch.setenv("PCMS_ROW_SLICES", str(sub))
    C.case_scaled(BE, "c3", small=True)
    C.case_scaled(BE, "c2", small=True)


def test_emu_box_boundary():
    C.case_box_boundary(BE)
    C.case_box_boundary(BV)


def test_emu_c4():
    C.case_c4(BE, n=6, size_scale=0.02)


@pytest.mark.parametrize("dim,degree,mode", C.DIM_CASES)
def test_emu_dims(dim, degree, mode):
    C.case_dims(BE, dim, degree, mode, scale=0.3)


@pytest.mark.parametrize("weight", [1, 2, 3, 4, 5])
def test_emu_weights(weight):
    C.case_weight(BE, weight)


def test_emu_tikhonov():
    C.case_tikhonov(BE, 0.5)


def test_emu_edge_cases():
    C.case_far_targets(BE)
    C.case_singular_exhausted(BE)
    C.case_ties(BE)
    C.case_tight_caps(BE)


def test_emu_lane_groups():
    """Four cooperating lanes per target give the same lists and statuses,
    and values within rounding, as one lane."""
    C.case_c1(BE4)
    C.case_ties(BE4)
    C.case_tight_caps(BE4)
    C.case_scaled(BE4, "c3", small=True)
    p = synth.c1()
    a, b = BE.neighbors(p), BE4.neighbors(p)
    for key in ("n_kept", "n_found", "r2", "status"):
        assert (a[key] == b[key]).all(), key
    for i in range(p.tgt.shape[0]):
        n = a["n_kept"][i]
        assert (a["nbr"][i, :n] == b["nbr"][i, :n]).all()


def test_emu_operator():
    C.case_operator(BE)


def test_emu_fp32_filter():
    C.case_fp32_filter(BE)


def test_emu_random_caps():
    C.case_random_caps(BE)


def _same_lists(a, b):
    for key in ("n_kept", "n_found", "r2", "status"):
        assert (a[key] == b[key]).all(), key
    for i in range(a["n_kept"].shape[0]):
        n = a["n_kept"][i]
        assert (a["nbr"][i, :n] == b["nbr"][i, :n]).all(), i


def test_emu_lbvh_cases():
    """The LBVH search against the oracle on the parity cases."""
    C.case_c1(BV)
    C.case_scaled(BV, "c3", small=True)
    C.case_far_targets(BV)
    C.case_singular_exhausted(BV)
    C.case_ties(BV)
    C.case_tight_caps(BV)
    C.case_fp32_filter(BV)
    C.case_random_caps(BV)


@pytest.mark.parametrize("dim,degree,mode", C.DIM_CASES)
def test_emu_lbvh_dims(dim, degree, mode):
    C.case_dims(BV, dim, degree, mode)


@pytest.mark.parametrize("name", ["c1", "c2", "c3", "c5"])
def test_emu_lbvh_matches_grid(name):
    """Lists and statuses on the LBVH are bitwise those of the grid (the same
    candidates reach the same selection); values agree to rounding, since the
    moment sums run over the kept sources in the structure's own source order
    (bucket order or Morton order)."""
    p = synth.c1() if name == "c1" else C.scaled(name, small=True)
    _same_lists(BE.neighbors(p), BV.neighbors(p))
    # |grid - lbvh| / (1 + |grid|): reordered FP64 sums stay near 1e-13 on these
    # cases; MIXED_REFINE inherits its FP32 stages' reordering, refined away
    for prec, bar in ((C.FP64, 1e-10), (C.MIXED_REFINE, 1e-7)):
        a, b = BE.transfer(p, prec), BV.transfer(p, prec)
        assert (a["status"] == b["status"]).all()
        ok = np.isfinite(a["out"])
        assert (np.isfinite(b["out"]) == ok).all()
        d = np.abs(a["out"] - b["out"])[ok] / (1.0 + np.abs(a["out"][ok]))
        assert d.max(initial=0.0) <= bar, (prec, d.max())
