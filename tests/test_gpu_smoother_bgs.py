"""GPU parity of the l1-scaled symmetric block Gauss-Seidel smoother (opts.smoother =
AMGE_SMOOTHER_BLOCK_GS: 64-row blocks, greedy colours over couplings inside a block,
forward then backward through all colours, couplings across blocks frozen at the start
of the sweep and their l1 weight on the diagonal; the smoother of the paper's
experiments, section 4.1 last paragraph and section 5.1) against the oracle's
(oracle.solve, smoother="l1blockgs", gs_block=64), through the C ABI, on hierarchies set
up from the oracle's own level matrices.  Bars as in test_gpu_parity.py: FP64 within
max(1e-10, 3 s), s the oracle's reformulation spread for this smoother; iteration counts
+-1; the FP32 V-cycle within +3 iterations and 1e-6 of the oracle solution.  The
library forms r = b - A x0 first and solves the two in-block triangular systems for the
correction (the same sweep, different rounding).  Sizes span many blocks with a ragged
last block (n not a multiple of 64) on every level."""
import numpy as np
import pytest

from paper_2107_05613_amd import workloads as W
from reformulation import fp64_bar, spreads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relerr(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


_CASES = {}


class BgsCase:
    def __init__(self, kind, n, L, coef):
        from oracle.hierarchy import build_hierarchy
        from oracle.solve import Multilevel, pcg
        from paper_2107_05613_amd import amge
        print(f"\n[block gs case] {kind} n={n} levels={L} coef={coef}", flush=True)
        a, b = W.coefficients(W.Workload("t", kind, n, L, coef))
        self.H = build_hierarchy(kind, n, L, a, b, check_targets=False)
        self.levels = [(self.H.A[k], self.H.D[k], self.H.P[k] if k < L - 1 else None) for k in range(L)]
        self.ml = Multilevel.from_hierarchy(self.H, smoother="l1blockgs", gs_block=64)
        self.b = W.rhs(self.H.A[0].shape[0], 0)[:, 0]
        self.xo, self.ito, _ = pcg(self.H.A[0], self.b, self.ml, rtol=1e-8)
        self.bar = {k: fp64_bar(v) for k, v in spreads(self.H, self.b, self.ito, smoother="l1blockgs").items()}
        self.gpu = {bits: amge.Hierarchy(self.levels, precond_bits=bits, smoother="l1blockgs") for bits in (64, 32)}
        print(f"[block gs case] sizes {[A.shape[0] for A in self.H.A]}, oracle {self.ito} iterations; "
              f"bars {self.bar}", flush=True)


def case(*spec):
    if spec not in _CASES:
        _CASES[spec] = BgsCase(*spec)
    return _CASES[spec]


SPECS = [("curl", 8, 3, "blocks"), ("div", 8, 3, "blocks"), ("curl", 12, 3, "unit"), ("div", 16, 3, "unit"),
         ("curl", 16, 4, "blocks")]


@pytest.mark.parametrize("spec", SPECS)
def test_bgs_smoother_application(spec):
    """One application of the hybrid smoother with block Gauss-Seidel point smoothers, and
    of its transpose, on every non-coarsest level (sweeps from a nonzero x0)."""
    from paper_2107_05613_amd import amge
    c = case(*spec)
    rng = np.random.default_rng(8)
    for k in range(len(c.H.A) - 1):
        lv = c.ml.levels[k]
        b = rng.uniform(-1, 1, lv.A.shape[0])
        x0 = rng.uniform(-1, 1, lv.A.shape[0])
        for op, fn in ((amge.OP_SMOOTH, c.ml.smooth), (amge.OP_SMOOTHT, c.ml.smooth_transpose)):
            ref = fn(lv, b, x0)
            out = torch.empty_like(dev(b))
            c.gpu[64].level_apply(k, op, dev(b), out, x2=dev(x0), precision=64)
            e64 = relerr(host(out), ref)
            c.gpu[64].level_apply(k, op, dev(b), out, x2=dev(x0), precision=32)
            e32 = relerr(host(out), ref)
            print(f"level {k} (n={lv.A.shape[0]}) op {op}: block GS smoother error fp64 {e64:.1e} fp32 {e32:.1e}")
            assert e64 <= c.bar["smooth"] and e32 <= 1e-4, (k, op)


@pytest.mark.parametrize("spec", SPECS)
def test_bgs_vcycle_and_pcg(spec):
    """Algorithm 4.1 with the block Gauss-Seidel hybrid smoother (folded and unfolded
    coarse tail: the host sweep of the fold and the kernels), and PCG around it: FP64
    parity, FP32 convergence."""
    from paper_2107_05613_amd import amge
    c = case(*spec)
    ref = c.ml.vcycle(c.b)
    z = torch.empty_like(dev(c.b))
    H0 = amge.Hierarchy(c.levels, precond_bits=64, smoother="l1blockgs", tail_rows=0)
    for name, H in (("folded", c.gpu[64]), ("unfolded", H0)):
        H.vcycle(dev(c.b), z)
        e = relerr(host(z), ref)
        print(f"{spec} {name} V-cycle error {e:.1e} (bar {c.bar['vcycle']:.1e})")
        assert e <= c.bar["vcycle"]
    H0.close()
    x = torch.zeros_like(dev(c.b))
    st, it, _ = c.gpu[64].pcg(dev(c.b), x, rtol=1e-8, maxit=500)
    assert st == 0 and abs(it[0] - c.ito) <= 1, (it, c.ito)
    c.gpu[64].pcg(dev(c.b), x, rtol=0.0, maxit=c.ito)
    err = np.linalg.norm(host(x) - c.xo) / np.linalg.norm(c.xo)
    st, it32, rr32 = c.gpu[32].pcg(dev(c.b), x, rtol=1e-8, maxit=500)
    e32 = np.linalg.norm(host(x) - c.xo) / np.linalg.norm(c.xo)
    print(f"{spec}: oracle {c.ito} iterations, GPU FP64 {it[0]}, fixed-count error {err:.1e}; "
          f"FP32 {it32[0]} iterations, error {e32:.1e}")
    assert err <= c.bar["pcg"]
    assert st == 0 and it32[0] <= c.ito + 3 and e32 <= 1e-6


def test_bgs_fewer_iterations_than_l1_jacobi():
    """The block smoother takes fewer PCG iterations than l1-Jacobi on the same hierarchy
    (both on the GPU, FP64 V-cycles)."""
    from paper_2107_05613_amd import amge
    c = case("curl", 16, 4, "blocks")
    x = torch.zeros_like(dev(c.b))
    Hj = amge.Hierarchy(c.levels, precond_bits=64)
    _, itj, _ = Hj.pcg(dev(c.b), x, rtol=1e-8, maxit=500)
    _, itb, _ = c.gpu[64].pcg(dev(c.b), x, rtol=1e-8, maxit=500)
    Hj.close()
    print(f"iterations: l1-Jacobi {itj[0]}, block Gauss-Seidel {itb[0]}")
    assert itb[0] < itj[0]


def test_bgs_smoother_arguments():
    """A matrix with a zero diagonal entry is refused at set-up (AMGE_ERR_NOT_SPD)."""
    import scipy.sparse as sp
    from paper_2107_05613_amd import amge
    c = case("curl", 8, 3, "blocks")
    A = c.levels[0][0].tolil(copy=True)
    A[5, 5] = 0.0
    bad = [(sp.csr_matrix(A),) + tuple(c.levels[0][1:])] + list(c.levels[1:])
    with pytest.raises(amge.AmgeError) as e:
        amge.Hierarchy(bad, smoother="l1blockgs")
    assert e.value.code == -3


@pytest.mark.parametrize("spec", SPECS)
def test_bgs_single_sweep_and_residual(spec):
    """One block sweep from a nonzero x (amge_level_apply SWEEP: the kernel the V-cycle
    launches after its first sweep) and the residual on the block layout (RESID) on every
    non-coarsest level, against the oracle's block sweep and b - A x; FP64 within 1e-13
    of |A||x| + |b| per entry (sweep: relative to the largest entry), FP32 within 1e-5."""
    from oracle.solve import BlockGS, contiguous_blocks
    from paper_2107_05613_amd import amge
    c = case(*spec)
    rng = np.random.default_rng(11)
    for k in range(len(c.H.A) - 1):
        A = c.H.A[k].tocsr()
        n = A.shape[0]
        b, x0 = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
        ref = BlockGS(A, contiguous_blocks(n, 64)).sweep(b, x0)
        rres = b - A @ x0
        scale = abs(A) @ abs(x0) + abs(b)
        out = torch.empty_like(dev(b))
        for bits, tol in ((64, 1e-13), (32, 1e-5)):
            c.gpu[64].level_apply(k, amge.OP_SWEEP, dev(b), out, x2=dev(x0), precision=bits)
            es = relerr(host(out), ref)
            c.gpu[64].level_apply(k, amge.OP_RESID, dev(b), out, x2=dev(x0), precision=bits)
            er = float(np.max(np.abs(host(out) - rres) / scale))
            print(f"level {k} (n={n}) fp{bits}: block sweep {es:.1e}, residual {er:.1e}")
            assert es <= (1e-12 if bits == 64 else 1e-4) and er <= tol, (k, bits)


def test_bgs_row_length_limit():
    """A row of more than 255 entries is refused at set-up with AMGE_ERR_SHAPE (the block
    layout stores a row's length in 8 bits); the matrix stays SPD (the extra couplings are
    weak and symmetric, diagonals raised to keep dominance)."""
    import scipy.sparse as sp
    from paper_2107_05613_amd import amge
    c = case("curl", 8, 3, "blocks")
    A = c.levels[0][0].tocsr()
    n = A.shape[0]
    cols = np.arange(1, 301) * (n // 301)
    E = sp.coo_matrix((np.full(cols.size, 1e-3), (np.zeros(cols.size, dtype=int), cols)), shape=(n, n))
    E = (E + E.T).tocsr()
    Aw = (A + E + sp.diags(np.asarray(abs(E).sum(axis=1)).ravel())).tocsr()
    assert np.diff(Aw.indptr).max() > 255
    bad = [(Aw,) + tuple(c.levels[0][1:])] + list(c.levels[1:])
    with pytest.raises(amge.AmgeError) as e:
        amge.Hierarchy(bad, smoother="l1blockgs")
    assert e.value.code == -2


def _dense_block_levels(n=337, nc=12, m=90, seed=5):
    """A two-level hierarchy whose fine matrix has dense 64-row diagonal blocks (rows with
    up to 64 entries inside their block: the largest register bound of the block sweep),
    a few couplings across blocks, and a positive, dominant diagonal (SPD); D an
    incidence with two +-1 entries per row that touches every column; P piecewise
    constant; the coarse matrix P^T A P."""
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    rows, cols, vals = [], [], []
    for b0 in range(0, n, 64):
        b1 = min(n, b0 + 64)
        for i in range(b0, b1):
            for j in range(b0, i):
                if rng.random() < 0.8:
                    rows.append(i), cols.append(j), vals.append(rng.uniform(-1, 1))
    for _ in range(3 * n):
        i, j = rng.integers(0, n, 2)
        if i // 64 != j // 64 and i > j:
            rows.append(i), cols.append(j), vals.append(rng.uniform(-1, 1))
    L = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    L.sum_duplicates()
    S = L + L.T
    A = (S + sp.diags(np.asarray(abs(S).sum(axis=1)).ravel() + 1.0)).tocsr()
    e0 = np.arange(n) % m
    e1 = (e0 + 1 + np.arange(n) % (m - 1)) % m
    D = sp.csr_matrix((np.r_[np.ones(n), -np.ones(n)], (np.r_[np.arange(n), np.arange(n)], np.r_[e0, e1])),
                      shape=(n, m))
    P = sp.csr_matrix((np.ones(n), (np.arange(n), np.arange(n) * nc // n)), shape=(n, nc))
    Ac = (P.T @ A @ P).tocsr()
    ec = np.arange(nc)
    Dc = sp.csr_matrix((np.r_[np.ones(nc), -np.ones(nc)], (np.r_[ec, ec], np.r_[ec, (ec + 1) % nc])), shape=(nc, nc))
    return [(A, D, P), (Ac, Dc, None)]


def test_bgs_dense_blocks_largest_bound():
    """One block sweep and the residual on a fine matrix with dense 64-row blocks (inside
    widths above 32: the NIN = 64 instances) against the oracle's block sweep and b - A x,
    FP64 and FP32, as in test_bgs_single_sweep_and_residual."""
    from oracle.solve import BlockGS, contiguous_blocks
    from paper_2107_05613_amd import amge
    levels = _dense_block_levels()
    A = levels[0][0]
    n = A.shape[0]
    inside = [sum(1 for j in A.indices[A.indptr[i]:A.indptr[i + 1]] if j // 64 == i // 64) for i in range(n)]
    assert max(inside) > 32
    H = amge.Hierarchy(levels, precond_bits=64, smoother="l1blockgs", tail_rows=0)
    rng = np.random.default_rng(13)
    b, x0 = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
    ref = BlockGS(A, contiguous_blocks(n, 64)).sweep(b, x0)
    rres = b - A @ x0
    scale = abs(A) @ abs(x0) + abs(b)
    out = torch.empty_like(dev(b))
    for bits, tol in ((64, 1e-13), (32, 1e-5)):
        H.level_apply(0, amge.OP_SWEEP, dev(b), out, x2=dev(x0), precision=bits)
        es = relerr(host(out), ref)
        H.level_apply(0, amge.OP_RESID, dev(b), out, x2=dev(x0), precision=bits)
        er = float(np.max(np.abs(host(out) - rres) / scale))
        print(f"dense blocks (n={n}, widest inside row {max(inside)}) fp{bits}: block sweep {es:.1e}, residual {er:.1e}")
        assert es <= (1e-12 if bits == 64 else 1e-4) and er <= tol, bits
    H.close()


def _wide_span_levels(n=70000, nc=40, m=3000, seed=7):
    """A two-level hierarchy whose fine matrix couples rows 65,600 apart (a block's
    outside columns then span more than 65,536, so the block layout stores 32-bit
    outside columns): a tridiagonal band, symmetric long-range couplings, a dominant
    diagonal; D, P and the coarse matrix as in _dense_block_levels."""
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    i = np.arange(n - 1)
    far = rng.integers(0, n - 65600, 200)
    rows = np.r_[i + 1, far + 65600]
    cols = np.r_[i, far]
    L = sp.coo_matrix((rng.uniform(-1, 1, rows.size), (rows, cols)), shape=(n, n)).tocsr()
    L.sum_duplicates()
    S = L + L.T
    A = (S + sp.diags(np.asarray(abs(S).sum(axis=1)).ravel() + 1.0)).tocsr()
    e0 = np.arange(n) % m
    e1 = (e0 + 1 + np.arange(n) % (m - 1)) % m
    D = sp.csr_matrix((np.r_[np.ones(n), -np.ones(n)], (np.r_[np.arange(n), np.arange(n)], np.r_[e0, e1])),
                      shape=(n, m))
    P = sp.csr_matrix((np.ones(n), (np.arange(n), np.arange(n) * nc // n)), shape=(n, nc))
    Ac = (P.T @ A @ P).tocsr()
    ec = np.arange(nc)
    Dc = sp.csr_matrix((np.r_[np.ones(nc), -np.ones(nc)], (np.r_[ec, ec], np.r_[ec, (ec + 1) % nc])), shape=(nc, nc))
    return [(A, D, P), (Ac, Dc, None)]


def test_bgs_wide_column_span():
    """One block sweep and the residual with 32-bit outside columns (a block's outside
    columns span more than 65,536) against the oracle's block sweep and b - A x, FP64
    and FP32, as in test_bgs_single_sweep_and_residual."""
    from oracle.solve import BlockGS, contiguous_blocks
    from paper_2107_05613_amd import amge
    levels = _wide_span_levels()
    A = levels[0][0]
    n = A.shape[0]
    span = 0
    for b0 in range(0, n, 64):
        cols = [j for r in range(b0, min(n, b0 + 64)) for j in A.indices[A.indptr[r]:A.indptr[r + 1]]
                if j // 64 != r // 64]
        span = max(span, max(cols) - min(cols))
    assert span >= 65536
    H = amge.Hierarchy(levels, precond_bits=64, smoother="l1blockgs", tail_rows=0)
    rng = np.random.default_rng(17)
    b, x0 = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
    ref = BlockGS(A, contiguous_blocks(n, 64)).sweep(b, x0)
    rres = b - A @ x0
    scale = abs(A) @ abs(x0) + abs(b)
    out = torch.empty_like(dev(b))
    for bits, tol in ((64, 1e-13), (32, 1e-5)):
        H.level_apply(0, amge.OP_SWEEP, dev(b), out, x2=dev(x0), precision=bits)
        es = relerr(host(out), ref)
        H.level_apply(0, amge.OP_RESID, dev(b), out, x2=dev(x0), precision=bits)
        er = float(np.max(np.abs(host(out) - rres) / scale))
        print(f"wide column span (n={n}) fp{bits}: block sweep {es:.1e}, residual {er:.1e}")
        assert es <= (1e-12 if bits == 64 else 1e-4) and er <= tol, bits
    H.close()
