"""The seeded input generators: shapes, determinism, ranges."""
import numpy as np

from paper_2107_05613_amd import workloads as W


def test_levels_rule():
    assert [W.default_levels(n) for n in (8, 16, 24, 32, 48, 64)] == [2, 3, 4, 4, 5, 5]
    for w in W.WORKLOADS.values():
        assert W.default_levels(w.n) == w.levels


def test_block_coefficients():
    c = W.block_coefficients(32, 0)
    assert c.shape == (512,)
    assert c.min() >= 1e-3 and c.max() <= 1e3
    assert np.array_equal(c, W.block_coefficients(32, 0))
    hx = W.hex_coefficients(32, c)
    # hex (i, j, k) belongs to block (i//4, j//4, k//4)
    i, j, k = 9, 30, 17
    assert hx[i + 32 * (j + 32 * k)] == c[(i // 4) + 8 * ((j // 4) + 8 * (k // 4))]


def test_rhs_shape_and_columns():
    b = W.rhs(100, 0, 3)
    assert b.shape == (100, 3) and b.flags.c_contiguous
    assert np.all(np.abs(b) <= 1)
    b1 = W.rhs(100, 0, 1)
    assert np.array_equal(b1[:, 0], b[:, 0])


def test_serving_requests():
    reqs = W.serving_requests(256, 0)
    assert len(reqs) == 256
    assert {r["kind"] for r in reqs} == {"curl", "div"}
    assert {r["n"] for r in reqs} <= {16, 24, 32, 48, 64}
    t = [r["t_arrive"] for r in reqs]
    assert t[0] == 0 and np.all(np.diff(t) >= 0)
