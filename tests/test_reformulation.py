"""CPU checks of the second FP64 evaluation used for the FP64 parity bar
(tests/reformulation.py): it is the oracle's operator (agreement to rounding where the
problem is well conditioned), a planted mistake in it is visible, and the spread it
measures on a jump-coefficient case is what the GPU tests then allow."""
import numpy as np
import pytest

from oracle.hierarchy import build_hierarchy
from oracle.solve import Multilevel
from paper_2107_05613_amd import workloads as W
from reformulation import Reformulated, fp64_bar, spreads


def _case(kind, n, L, coef):
    w = W.Workload("t", kind, n, L, coef)
    a, b = W.coefficients(w)
    H = build_hierarchy(kind, n, L, a, b, check_targets=False)
    return H, W.rhs(H.A[0].shape[0], 0)[:, 0]


@pytest.mark.parametrize("spec", [("curl", 8, 3, "unit"), ("div", 8, 3, "unit")])
def test_reformulation_is_the_same_operator(spec):
    H, b = _case(*spec)
    s = spreads(H, b, 15)
    print(spec, s)
    assert max(s.values()) <= 1e-12
    assert fp64_bar(max(s.values())) == 1e-10


def test_planted_mistake_in_reformulation_is_visible():
    H, b = _case("curl", 8, 3, "unit")
    ml = Multilevel.from_hierarchy(H)
    rf = Reformulated(H.A, H.D, H.P)
    for lv in rf.levels[:-1]:
        lv.PtA = 0.5 * lv.PtA          # a dropped half of the restricted residual's A-term
    z0, z1 = ml.vcycle(b), rf.vcycle(b)
    assert np.max(np.abs(z1 - z0)) / np.max(np.abs(z0)) > 1e-3


def test_jump_coefficients_raise_the_spread():
    H, b = _case("div", 8, 3, "blocks")
    s = spreads(H, b, 20)
    print(s)
    assert 1e-13 < max(s.values()) < 1e-9
