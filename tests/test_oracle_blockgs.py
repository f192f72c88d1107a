"""Pins of the oracle's l1-scaled symmetric block Gauss-Seidel sweep (section 4.1, last
paragraph, and section 5.1: the smoother of the cited smoother paper; row blocks stand
in for its processors).

The sweep is written as row relaxations in colour order with the couplings across
blocks frozen at the start of the sweep.  It is pinned against facts derived
independently of that form:
* blocks of one row: the closed form x + (2 d - a_ii) / d^2 (b - A x), d_i = sum_j |a_ij|
  (a forward and a backward l1-Jacobi step that both read x0 across blocks);
* one block holding every row: textbook symmetric Gauss-Seidel in colour order;
* any blocks: the matrix form x + Mb^{-1} (D + 2 D_l1) Mf^{-1} (b - A x), with Mf the
  lower triangle of the block-diagonal part of A in (block, colour, row) order plus
  the off-block l1 sums on the diagonal and Mb = Mf^T, built with dense algebra;
* a plain row-by-row loop in that order;
* the l1 convergence bound: the A-norm of I - M A is below 1.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle.hierarchy import build_hierarchy
from oracle.solve import (BlockGS, Multilevel, block_coloring, contiguous_blocks, greedy_coloring,
                          gs_sweep, l1_diag, pcg)
from paper_2107_05613_amd import workloads as W


def _hier(kind, n, L, coef="blocks", seed=0):
    w = W.Workload("t", kind, n, L, coef, coef_seed=seed)
    a, b = W.coefficients(w)
    return build_hierarchy(kind, n, L, a, b)


@pytest.fixture(scope="module")
def curl4():
    return _hier("curl", 4, 3)


@pytest.fixture(scope="module")
def div4():
    return _hier("div", 4, 3)


def _vecs(n, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)


def test_block_coloring_is_proper_inside_blocks(curl4):
    """Rows coupled inside a block differ in colour, each colour is the first fit over
    earlier rows of the same block; couplings across blocks do not constrain colours."""
    A = curl4.A[0].tocsr()
    blk = contiguous_blocks(A.shape[0], 16)
    color = block_coloring(A, blk)
    Ad = A.toarray()
    for i in range(A.shape[0]):
        nb = np.nonzero(Ad[i])[0]
        nb = nb[(nb != i) & (blk[nb] == blk[i])]
        assert np.all(color[nb] != color[i])
        earlier = set(color[nb[nb < i]].tolist())
        assert color[i] == min(set(range(len(earlier) + 1)) - earlier)
    assert np.array_equal(block_coloring(A, np.zeros(A.shape[0], dtype=int)), greedy_coloring(A))


@pytest.mark.parametrize("which", ["curl4", "div4"])
def test_point_blocks_closed_form(which, request):
    H = request.getfixturevalue(which)
    A = H.A[0].tocsr()
    n = A.shape[0]
    b, x = _vecs(n, 1)
    got = BlockGS(A, np.arange(n)).sweep(b, x)
    d, a = l1_diag(A), A.diagonal()
    ref = x + (2 * d - a) / d ** 2 * (b - A @ x)
    assert abs(got - ref).max() <= 1e-12 * abs(ref).max()


@pytest.mark.parametrize("which", ["curl4", "div4"])
def test_one_block_is_symmetric_gauss_seidel(which, request):
    H = request.getfixturevalue(which)
    A = H.A[0].tocsr()
    n = A.shape[0]
    b, x = _vecs(n, 2)
    got = BlockGS(A, np.zeros(n, dtype=int)).sweep(b, x)
    color = greedy_coloring(A)
    classes = [np.nonzero(color == c)[0] for c in range(color.max() + 1)]
    ref = gs_sweep(A, A.diagonal(), classes, b, x)
    assert abs(got - ref).max() <= 1e-12 * abs(ref).max()


def _matrix_form(A, blk, color):
    n = A.shape[0]
    order = np.lexsort((np.arange(n), color, blk))
    Ad = A.toarray()[np.ix_(order, order)]
    bo = blk[order]
    same = bo[:, None] == bo[None, :]
    Din = np.diag(np.diag(Ad))
    Dl1 = np.diag(np.where(same, 0.0, abs(Ad)).sum(axis=1))
    Mf = np.tril(np.where(same, Ad, 0.0), -1) + Din + Dl1
    S = np.linalg.solve(Mf.T, (Din + 2 * Dl1) @ np.linalg.inv(Mf))
    P = np.eye(n)[:, order]          # P y maps the ordered vector back
    return P @ S @ P.T


@pytest.mark.parametrize("which,block", [("curl4", 8), ("curl4", 37), ("div4", 16), ("div4", 64)])
def test_block_sweep_matrix_form_and_symmetry(which, block, request):
    H = request.getfixturevalue(which)
    A = H.A[0].tocsr()
    n = A.shape[0]
    blk = contiguous_blocks(n, block)
    g = BlockGS(A, blk)
    S = _matrix_form(A, blk, block_coloring(A, blk))
    assert abs(S - S.T).max() <= 1e-12 * abs(S).max()
    b, x = _vecs(n, 3)
    got = g.sweep(b, x)
    ref = x + S @ (b - A @ x)
    assert abs(got - ref).max() <= 1e-11 * abs(ref).max()
    # l1 bound: the error propagation I - S A contracts in the A-norm
    ev = sla.eigh(A.toarray(), np.linalg.inv(S), eigvals_only=True)
    assert ev.min() > 0 and ev.max() < 2


def test_block_sweep_row_by_row(div4):
    """A plain loop over the rows of every block in (colour, row) order, forward then
    backward, reading x0 across blocks, gives the same sweep."""
    A = div4.A[1].tocsr()
    n = A.shape[0]
    blk = contiguous_blocks(n, 8)
    color = block_coloring(A, blk)
    b, x0 = _vecs(n, 4)
    x = x0.copy()
    Ad = A.toarray()
    for B in range(int(blk.max()) + 1):
        rows = np.nonzero(blk == B)[0]
        seq = rows[np.lexsort((rows, color[rows]))]
        inside = np.zeros(n, dtype=bool)
        inside[rows] = True
        for i in list(seq) + list(seq[::-1]):
            d = Ad[i, i] + abs(Ad[i, ~inside]).sum()
            x[i] += (b[i] - Ad[i, inside] @ x[inside] - Ad[i, ~inside] @ x0[~inside]) / d
    got = BlockGS(A, blk).sweep(b, x0)
    assert abs(got - x).max() <= 1e-12 * abs(x).max()


@pytest.mark.parametrize("which", ["curl4", "div4"])
def test_block_gs_vcycle_symmetric_and_between_smoothers(which, request):
    """The V-cycle with block sweeps is symmetric with lambda(BA) in (0, 1]; PCG takes
    fewer iterations than with l1-Jacobi."""
    H = request.getfixturevalue(which)
    ml = Multilevel.from_hierarchy(H, smoother="l1blockgs", gs_block=16)
    n = H.A[0].shape[0]
    B = np.column_stack([ml.vcycle(np.eye(n)[:, j]) for j in range(n)])
    assert abs(B - B.T).max() <= 1e-11 * abs(B).max()
    ev = sla.eigh(H.A[0].toarray(), np.linalg.inv(B), eigvals_only=True)
    assert ev.min() > 0 and ev.max() <= 1 + 1e-10
    b = W.rhs(n, 0)[:, 0]
    _, it_b, _ = pcg(H.A[0], b, ml, rtol=1e-8)
    _, it_j, _ = pcg(H.A[0], b, Multilevel.from_hierarchy(H), rtol=1e-8)
    assert it_b < it_j
