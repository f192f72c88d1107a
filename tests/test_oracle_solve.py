"""Pins of the oracle's solve phase (paper section 4, Algorithm 4.1, eq. (4.1)).

Checks against mathematics the paper fixes: the l1-Jacobi spectrum bound, the
error-propagation factorisation of the hybrid smoother (section 4.1), symmetry
and positivity of the V-cycle preconditioner built from the M / M^T pair of
Algorithm 4.1, PCG against a dense direct solve, the B = I case against
textbook CG (scipy), and the one-level case reducing to a Cholesky solve.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle.hierarchy import build_hierarchy
from oracle.solve import Multilevel, pcg, cg_plain, l1_diag
from paper_2107_05613_amd import workloads as W


def _hier(kind, n, L, coef="unit", seed=0):
    w = W.Workload("t", kind, n, L, coef, coef_seed=seed)
    a, b = W.coefficients(w)
    return build_hierarchy(kind, n, L, a, b)


@pytest.fixture(scope="module")
def curl4():
    return _hier("curl", 4, 3, "blocks")


@pytest.fixture(scope="module")
def div4():
    return _hier("div", 4, 3, "blocks")


def test_l1_jacobi_spectrum(curl4, div4):
    """d_i = sum_j |a_ij| gives lambda(d^{-1} A) in (0, 1] (no damping needed)."""
    for H in (curl4, div4):
        for A in H.A[:2]:
            d = l1_diag(A)
            Ad = A.toarray()
            ev = sla.eigh(Ad, np.diag(d), eigvals_only=True)
            assert ev.min() > 0 and ev.max() <= 1 + 1e-12


def _explicit(op, n):
    return np.column_stack([op(np.eye(n)[:, j]) for j in range(n)])


@pytest.mark.parametrize("which", ["curl4", "div4"])
def test_vcycle_symmetric_and_positive(which, request):
    """B = V-cycle(., x0=0) is symmetric (M^{-T} post-smoother) and lambda(BA) in (0, 1]."""
    H = request.getfixturevalue(which)
    ml = Multilevel.from_hierarchy(H)
    n = H.A[0].shape[0]
    B = _explicit(ml.vcycle, n)
    # coefficients jump by up to 1e6 inside this hierarchy; rounding asymmetry stays ~1e-13
    assert abs(B - B.T).max() <= 1e-11 * abs(B).max()
    ev = sla.eigh(H.A[0].toarray(), np.linalg.inv(B), eigvals_only=True)
    assert ev.min() > 0 and ev.max() <= 1 + 1e-10


@pytest.mark.parametrize("which", ["curl4", "div4"])
def test_hybrid_error_propagation_factorises(which, request):
    """I - Mbar^{-1} A = [I - D Mhat^{-1} D^T A][I - M^{-1} A] (section 4.1), with the
    two-sweep l1-Jacobi operators written out as explicit matrices."""
    H = request.getfixturevalue(which)
    ml = Multilevel.from_hierarchy(H)
    lv = ml.levels[0]
    A = lv.A.toarray(); D = lv.D.toarray(); Ah = D.T @ A @ D
    n = A.shape[0]
    di, dhi = np.diag(1 / l1_diag(lv.A)), np.diag(1 / l1_diag(sp.csr_matrix(Ah)))
    Minv = 2 * di - di @ A @ di               # two sweeps from zero
    Mhinv = 2 * dhi - dhi @ Ah @ dhi
    E_ref = (np.eye(n) - D @ Mhinv @ D.T @ A) @ (np.eye(n) - Minv @ A)
    # the oracle's smoother as a black box: e_new = e - S(A e, 0)
    E = np.eye(n) - _explicit(lambda e: ml.smooth(lv, A @ e, np.zeros(n)), n)
    assert abs(E - E_ref).max() < 1e-12
    # transpose smoother: reversed order
    Et_ref = (np.eye(n) - Minv @ A) @ (np.eye(n) - D @ Mhinv @ D.T @ A)
    Et = np.eye(n) - _explicit(lambda e: ml.smooth_transpose(lv, A @ e, np.zeros(n)), n)
    assert abs(Et - Et_ref).max() < 1e-12


def test_pcg_matches_dense_direct_solve():
    """Configuration 1 (n=8 H(curl), 2 levels): PCG to 1e-14 equals a dense solve."""
    H = _hier("curl", 8, 2)
    ml = Multilevel.from_hierarchy(H)
    b = W.rhs(H.A[0].shape[0], 0)[:, 0]
    x, it, hist = pcg(H.A[0], b, ml, rtol=1e-14, maxit=200)
    xd = sla.cho_solve(sla.cho_factor(H.A[0].toarray()), b)
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)
    assert it < 60


def test_identity_preconditioner_is_textbook_cg():
    """With B = I the loop reproduces scipy's CG iterates."""
    H = _hier("div", 4, 1)
    A = H.A[0]
    b = W.rhs(A.shape[0], 3)[:, 0]
    seen = []
    spla.cg(A, b, rtol=1e-30, atol=0, maxiter=12, callback=lambda xk: seen.append(xk.copy()))
    for k in (1, 5, 12):
        x, it, _ = cg_plain(A, b, fixed_iters=k)
        assert it == k
        assert np.linalg.norm(x - seen[k - 1]) <= 1e-10 * np.linalg.norm(seen[k - 1])


def test_one_level_is_cholesky():
    H = _hier("curl", 3, 1)
    ml = Multilevel.from_hierarchy(H)
    b = W.rhs(H.A[0].shape[0], 1)[:, 0]
    x, it, _ = pcg(H.A[0], b, ml, rtol=1e-8)
    assert it == 1
    assert np.linalg.norm(H.A[0] @ x - b) <= 1e-12 * np.linalg.norm(b)


def test_pcg_stops_on_preconditioner_norm(div4):
    """Stop rule: sqrt(r.z / r0.z0) <= tol; the count is the number of A-products."""
    ml = Multilevel.from_hierarchy(div4)
    A = div4.A[0]
    b = W.rhs(A.shape[0], 0)[:, 0]
    x, it, hist = pcg(A, b, ml, rtol=1e-8)
    assert hist[-1] <= 1e-8 < hist[-2]
    assert len(hist) == it + 1
    r = b - A @ x
    z = ml.vcycle(r)
    r0z0 = b @ ml.vcycle(b)
    assert np.isclose(np.sqrt(r @ z / r0z0), hist[-1], rtol=1e-6)
    # fixed-iteration mode runs exactly that many products
    x2, it2, _ = pcg(A, b, ml, fixed_iters=it)
    assert it2 == it and np.allclose(x2, x, rtol=0, atol=1e-14 * abs(x).max())


# ----------------------------------------------------------------------------
# symmetric Gauss-Seidel in colour order
# ----------------------------------------------------------------------------
def test_greedy_coloring_is_proper_and_first_fit(curl4):
    """No two coupled rows share a colour, and every row's colour is the smallest one
    its earlier neighbours leave free (checked by brute force over the dense pattern)."""
    from oracle.solve import greedy_coloring
    for A in (curl4.A[0], curl4.A[1]):
        color = greedy_coloring(A)
        Ad = A.toarray()
        for i in range(A.shape[0]):
            nb = np.nonzero(Ad[i])[0]
            nb = nb[nb != i]
            assert np.all(color[nb] != color[i])
            earlier = set(color[nb[nb < i]].tolist())
            assert color[i] == min(set(range(len(earlier) + 1)) - earlier)


def test_gs_sweep_is_textbook_symmetric_gauss_seidel(div4):
    """One colour-order sweep equals textbook symmetric Gauss-Seidel on the matrix with
    its rows and columns permuted into colour order: a forward triangular solve with
    (D + L) then a backward one with (D + U), L / U the strict triangles in that order."""
    from oracle.solve import greedy_coloring, gs_sweep
    A = div4.A[0].tocsr()
    color = greedy_coloring(A)
    order = np.argsort(color, kind="stable")
    classes = [np.nonzero(color == c)[0] for c in range(color.max() + 1)]
    rng = np.random.default_rng(3)
    b, x = rng.uniform(-1, 1, A.shape[0]), rng.uniform(-1, 1, A.shape[0])
    got = gs_sweep(A, A.diagonal(), classes, b, x)
    Ap = A[order][:, order].toarray()
    bp, xp = b[order], x[order]
    lower, upper = np.tril(Ap), np.triu(Ap)
    xp = xp + sla.solve_triangular(lower, bp - Ap @ xp, lower=True)
    xp = xp + sla.solve_triangular(upper, bp - Ap @ xp, lower=False)
    ref = np.empty_like(xp)
    ref[order] = xp
    assert abs(got - ref).max() <= 1e-12 * abs(ref).max()


@pytest.mark.parametrize("which", ["curl4", "div4"])
def test_gs_vcycle_symmetric_and_positive(which, request):
    """With symmetric Gauss-Seidel point smoothers the V-cycle is again symmetric and
    lambda(BA) lies in (0, 1], and PCG needs fewer iterations than with l1-Jacobi."""
    H = request.getfixturevalue(which)
    ml = Multilevel.from_hierarchy(H, smoother="symgs")
    n = H.A[0].shape[0]
    B = _explicit(ml.vcycle, n)
    assert abs(B - B.T).max() <= 1e-11 * abs(B).max()
    ev = sla.eigh(H.A[0].toarray(), np.linalg.inv(B), eigvals_only=True)
    assert ev.min() > 0 and ev.max() <= 1 + 1e-10
    b = W.rhs(n, 0)[:, 0]
    _, it_gs, _ = pcg(H.A[0], b, ml, rtol=1e-8)
    _, it_j, _ = pcg(H.A[0], b, Multilevel.from_hierarchy(H), rtol=1e-8)
    assert it_gs < it_j
