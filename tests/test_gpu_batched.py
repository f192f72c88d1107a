"""GPU parity of the batched path (several right-hand sides per call) through the C ABI.

A hierarchy set up with max_rhs > 1 runs the V-cycle and PCG on n x NC row-major
blocks (NC = max_rhs rounded up to a power of two, padding columns zero) with SpMM
kernels; PCG keeps one set of recurrences per column and stops each column on its own
(section 5.1 per column), replaying a captured graph of one iteration.

Bars (the single-column ones of test_gpu_parity.py, per column):
* The GPU hierarchies are set up from the oracle's own level matrices (same inputs).
* FP64: every column of the batched V-cycle within max(1e-10, 3 s) of the oracle
  V-cycle on that column, s being the oracle's reformulation spread
  (tests/reformulation.py; below 1e-11 on these cases, so the bar is 1e-10); PCG
  columns within the same bound of the oracle's iterate after the same number of
  iterations, iteration counts at rtol 1e-8 within +-1.
* FP32 preconditioner: each column converges to rtol 1e-8 within 3 iterations of the
  oracle's FP64 count, solution within 1e-6 of the oracle's.
* Graph replays: three batched solves with eager work between them each match their
  reference, and a repeated solve is bitwise identical.
"""
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


class BCase:
    def __init__(self, kind, n, L, coef, max_rhs):
        from oracle.hierarchy import build_hierarchy
        from oracle.solve import Multilevel
        from paper_2107_05613_amd import amge
        print(f"\n[bcase] {kind} n={n} levels={L} coef={coef} max_rhs={max_rhs}", flush=True)
        w = W.Workload("t", kind, n, L, coef)
        self.alpha, self.beta = W.coefficients(w)
        self.L = L
        self.H = build_hierarchy(kind, n, L, self.alpha, self.beta, check_targets=False)
        self.levels = [(self.H.A[k], self.H.D[k], self.H.P[k] if k < L - 1 else None) for k in range(L)]
        self.ml = Multilevel.from_hierarchy(self.H)
        self.gpu = {bits: amge.Hierarchy(self.levels, precond_bits=bits, max_rhs=max_rhs) for bits in (64, 32)}
        self.n1 = self.H.A[0].shape[0]
        kap = 1.0
        for k in range(L - 1):
            A, D = self.H.A[k], self.H.D[k]
            num = abs(D).T @ (abs(A) @ (abs(D) @ np.ones(D.shape[1])))
            den = abs((D.T @ A @ D).tocsr()) @ np.ones(D.shape[1])
            kap = max(kap, float(np.max(num / den)))
        self.kappa = kap
        sp = spreads(self.H, W.rhs(self.n1, 11)[:, 0], 20)
        self.tol64 = fp64_bar(max(sp.values()))
        print(f"[bcase] reformulation spread {max(sp.values()):.1e}, FP64 bar {self.tol64:.1e}", flush=True)


_CASES = {}


def bcase(kind, n, L, coef, max_rhs):
    key = (kind, n, L, coef, max_rhs)
    if key not in _CASES:
        _CASES[key] = BCase(*key)
    return _CASES[key]


# (hierarchy, nrhs): a ragged block (5 of 8 padded columns) and a full 32-column block
SPECS = [(("curl", 8, 3, "blocks", 8), 5), (("div", 12, 3, "unit", 32), 32), (("div", 8, 3, "blocks", 4), 4)]


@pytest.mark.parametrize("spec,nrhs", SPECS)
def test_batched_vcycle(spec, nrhs):
    """a8: one V-cycle on an n x nrhs block equals the oracle V-cycle column by column."""
    c = bcase(*spec)
    B = W.rhs(c.n1, 11, nrhs)
    Z = torch.zeros(c.n1 * nrhs, dtype=torch.float64, device="cuda")
    c.gpu[64].vcycle(dev(B), Z, nrhs=nrhs)
    z64 = host(Z).reshape(c.n1, nrhs)
    c.gpu[32].vcycle(dev(B), Z, nrhs=nrhs)
    z32 = host(Z).reshape(c.n1, nrhs)
    A = c.H.A[0]
    worst64 = worst_en = 0.0
    for j in range(nrhs):
        ref = c.ml.vcycle(B[:, j])
        worst64 = max(worst64, relerr(z64[:, j], ref))
        d = z32[:, j] - ref
        worst_en = max(worst_en, float(np.sqrt(d @ (A @ d)) / np.sqrt(ref @ (A @ ref))))
    print(f"{spec} nrhs={nrhs}: FP64 worst column error {worst64:.2e} (tol {c.tol64:.1e}); "
          f"FP32 worst energy-norm error {worst_en:.2e}")
    assert worst64 <= c.tol64
    assert worst_en <= (1e-3 if c.kappa < 1e6 else 5e-2)


@pytest.mark.parametrize("spec,nrhs", SPECS[:2])
def test_batched_folded_tail(spec, nrhs):
    """The batched V-cycle applies the folded coarse tail as a dense block product; with
    tail_rows = 0 it runs every level.  Both match the oracle column by column (FP64) and
    agree to FP64 rounding, also in FP32."""
    from paper_2107_05613_amd import amge
    c = bcase(*spec)
    B = W.rhs(c.n1, 12, nrhs)
    Z = torch.zeros(c.n1 * nrhs, dtype=torch.float64, device="cuda")
    for bits in (64, 32):
        H0 = amge.Hierarchy(c.levels, precond_bits=bits, max_rhs=spec[-1], tail_rows=0)
        H0.vcycle(dev(B), Z, nrhs=nrhs)
        z0 = host(Z).reshape(c.n1, nrhs)
        c.gpu[bits].vcycle(dev(B), Z, nrhs=nrhs)
        zf = host(Z).reshape(c.n1, nrhs)
        H0.close()
        worst0 = max(relerr(z0[:, j], c.ml.vcycle(B[:, j])) for j in range(nrhs))
        diff = relerr(zf, z0)
        print(f"{spec} nrhs={nrhs} FP{bits}: unfolded vs oracle {worst0:.2e}, folded vs unfolded {diff:.2e}")
        if bits == 64:
            assert worst0 <= c.tol64 and diff <= c.tol64
        else:
            assert diff <= 1e-3


@pytest.mark.parametrize("spec,nrhs", SPECS[:2])
def test_batched_pcg_fp64(spec, nrhs):
    """a7 + a8: per-column inexact PCG in FP64; counts within +-1 of the oracle's, and the
    oracle's iterate after the same fixed count."""
    from oracle.solve import pcg
    c = bcase(*spec)
    B = W.rhs(c.n1, 21, nrhs)
    X = torch.zeros(c.n1 * nrhs, dtype=torch.float64, device="cuda")
    status, its, rrs = c.gpu[64].pcg(dev(B), X, rtol=1e-8, maxit=500, nrhs=nrhs)
    assert status == 0 and max(rrs) <= 1e-8
    ito = []
    for j in range(nrhs):
        _, it, _ = pcg(c.H.A[0], B[:, j], c.ml, rtol=1e-8)
        ito.append(it)
    print(f"{spec}: gpu iters {its}, oracle iters {ito}")
    assert all(abs(a - b) <= 1 for a, b in zip(its, ito))
    # fixed count: rtol <= 0 runs exactly maxit iterations in every column
    k = max(ito)
    status, its2, _ = c.gpu[64].pcg(dev(B), X, rtol=0.0, maxit=k, nrhs=nrhs)
    assert its2 == [k] * nrhs
    Xs = host(X).reshape(c.n1, nrhs)
    worst = 0.0
    for j in range(nrhs):
        xo, _, _ = pcg(c.H.A[0], B[:, j], c.ml, fixed_iters=k)
        worst = max(worst, np.linalg.norm(Xs[:, j] - xo) / np.linalg.norm(xo))
    print(f"{spec}: fixed {k} iterations, worst column error {worst:.2e} (tol {c.tol64:.1e})")
    assert worst <= c.tol64


@pytest.mark.parametrize("spec,nrhs", SPECS[:2])
def test_batched_pcg_fp32(spec, nrhs):
    """FP32 batched V-cycle inside FP64 per-column PCG: every column reaches rtol 1e-8."""
    from oracle.solve import pcg
    c = bcase(*spec)
    B = W.rhs(c.n1, 31, nrhs)
    X = torch.zeros(c.n1 * nrhs, dtype=torch.float64, device="cuda")
    status, its, rrs = c.gpu[32].pcg(dev(B), X, rtol=1e-8, maxit=500, nrhs=nrhs)
    assert status == 0 and max(rrs) <= 1e-8
    Xs = host(X).reshape(c.n1, nrhs)
    worst = 0.0
    for j in range(nrhs):
        xo, ito, _ = pcg(c.H.A[0], B[:, j], c.ml, rtol=1e-8)
        assert its[j] <= ito + 3, (j, its[j], ito)
        worst = max(worst, np.linalg.norm(Xs[:, j] - xo) / np.linalg.norm(xo))
    print(f"{spec}: FP32-precond iters {its}; worst error vs oracle {worst:.2e}")
    assert worst <= 1e-6


def test_batched_matches_single_column_path():
    """The batched solve of a block and single-column solves of its columns agree (the
    two paths use different kernels, so to rounding: FP64 preconditioner, fixed count)."""
    c = bcase("div", 8, 3, "blocks", 4)
    nrhs = 4
    B = W.rhs(c.n1, 41, nrhs)
    X = torch.zeros(c.n1 * nrhs, dtype=torch.float64, device="cuda")
    c.gpu[64].pcg(dev(B), X, rtol=0.0, maxit=12, nrhs=nrhs)
    Xs = host(X).reshape(c.n1, nrhs)
    x1 = torch.zeros(c.n1, dtype=torch.float64, device="cuda")
    for j in range(nrhs):
        c.gpu[64].pcg(dev(B[:, j]), x1, rtol=0.0, maxit=12)
        e = np.linalg.norm(Xs[:, j] - host(x1)) / np.linalg.norm(host(x1))
        assert e <= c.tol64, (j, e)


def test_graph_replays_with_eager_work_between():
    """The captured iteration is replayed by three batched solves on different blocks,
    with eager GPU work (torch and single-column solves) between them; every replay is
    checked against its own reference and a repeated solve is bitwise identical."""
    from oracle.solve import pcg
    c = bcase("curl", 8, 3, "blocks", 8)
    nrhs = 6
    refs = []
    outs = []
    for seed in (51, 52, 53):
        B = W.rhs(c.n1, seed, nrhs)
        X = torch.zeros(c.n1 * nrhs, dtype=torch.float64, device="cuda")
        status, its, _ = c.gpu[64].pcg(dev(B), X, rtol=0.0, maxit=10, nrhs=nrhs)
        assert status == 0 and its == [10] * nrhs
        outs.append(host(X).reshape(c.n1, nrhs))
        refs.append([pcg(c.H.A[0], B[:, j], c.ml, fixed_iters=10)[0] for j in range(nrhs)])
        # eager work in between: a torch reduction and a single-column solve
        y = torch.ones(1 << 20, dtype=torch.float64, device="cuda")
        assert float(y.sum()) == float(1 << 20)
        x1 = torch.zeros(c.n1, dtype=torch.float64, device="cuda")
        c.gpu[64].pcg(dev(B[:, 0]), x1, rtol=1e-8)
    for Xs, R in zip(outs, refs):
        for j in range(nrhs):
            assert np.linalg.norm(Xs[:, j] - R[j]) <= c.tol64 * np.linalg.norm(R[j])
    B = W.rhs(c.n1, 51, nrhs)
    X = torch.zeros(c.n1 * nrhs, dtype=torch.float64, device="cuda")
    c.gpu[64].pcg(dev(B), X, rtol=0.0, maxit=10, nrhs=nrhs)
    assert np.array_equal(host(X).reshape(c.n1, nrhs), outs[0])


def test_batched_edge_cases():
    """Zero columns finish with 0 iterations and a zero solution; a NaN column is
    rejected; maxit = 1 is honoured per column; nrhs beyond max_rhs is rejected."""
    from paper_2107_05613_amd import amge
    c = bcase("curl", 8, 3, "blocks", 8)
    nrhs = 3
    B = W.rhs(c.n1, 61, nrhs)
    B[:, 1] = 0.0
    X = torch.full((c.n1 * nrhs,), 7.0, dtype=torch.float64, device="cuda")
    status, its, rrs = c.gpu[32].pcg(dev(B), X, rtol=1e-8, nrhs=nrhs)
    Xs = host(X).reshape(c.n1, nrhs)
    assert status == 0 and its[1] == 0 and rrs[1] == 0.0 and not np.any(Xs[:, 1])
    assert its[0] > 0 and its[2] > 0
    status, its, _ = c.gpu[32].pcg(dev(B), X, rtol=1e-8, maxit=1, nrhs=nrhs)
    assert status == 1 and its == [1, 0, 1]
    Bn = B.copy()
    Bn[3, 2] = np.nan
    with pytest.raises(amge.AmgeError) as e:
        c.gpu[32].pcg(dev(Bn), X, nrhs=nrhs)
    assert e.value.code == -7
    big = torch.zeros(c.n1 * 9, dtype=torch.float64, device="cuda")
    with pytest.raises(amge.AmgeError) as e:
        c.gpu[32].pcg(big, big.clone(), nrhs=9)
    assert e.value.code == -1
    # the hierarchy still solves after the rejected calls
    status, its, rrs = c.gpu[32].pcg(dev(B), X, rtol=1e-8, nrhs=nrhs)
    assert status == 0 and max(rrs) <= 1e-8


@pytest.mark.parametrize("nrhs", [33, 64])
def test_batched_widest_block(nrhs):
    """The widest block (max_rhs = 64, the largest supported): 33 columns (padded to 64)
    and 64 columns; sampled columns against the oracle's fixed-count PCG iterate."""
    from oracle.solve import pcg
    c = bcase("div", 8, 3, "blocks", 64)
    B = W.rhs(c.n1, 71, nrhs)
    X = torch.zeros(c.n1 * nrhs, dtype=torch.float64, device="cuda")
    k = 10
    status, its, _ = c.gpu[64].pcg(dev(B), X, rtol=0.0, maxit=k, nrhs=nrhs)
    assert its == [k] * nrhs
    Xs = host(X).reshape(c.n1, nrhs)
    for j in (0, nrhs // 2, nrhs - 1):
        xo, _, _ = pcg(c.H.A[0], B[:, j], c.ml, fixed_iters=k)
        assert np.linalg.norm(Xs[:, j] - xo) <= c.tol64 * np.linalg.norm(xo), j
    # FP32 preconditioner converges in every column
    status, its, rrs = c.gpu[32].pcg(dev(B), X, rtol=1e-8, nrhs=nrhs)
    assert status == 0 and max(rrs) <= 1e-8


def test_batched_fp64_fine_residual():
    """The batched FP32 V-cycle with the fine-level residual in FP64 (resid_bits = 64) on
    the 24^3 H(curl) jump workload: every column converges within 3 iterations of the
    same column's FP64 batched solve, and each column's solution is within 1e-6 of the
    single-column FP32 + FP64-residual solve (both FP32 preconditioners, FP64 PCG)."""
    from paper_2107_05613_amd import amge
    w = W.Workload("t", "curl", 24, W.default_levels(24), "blocks", coef_seed=0)
    a, b = W.coefficients(w)
    prod = amge.build_problem(w.kind, w.n, w.levels, a, b)
    k = 4
    H64 = amge.Hierarchy(prod, precond_bits=64, max_rhs=k)
    Hm = amge.Hierarchy(prod, precond_bits=32, resid_bits=64, max_rhs=k)
    n = Hm.rows[0]
    B = W.rhs(n, 21, k)
    X = torch.zeros(n * k, dtype=torch.float64, device="cuda")
    st, it64, _ = H64.pcg(dev(B), X, rtol=1e-8, maxit=1000, nrhs=k)
    X.zero_()
    st, itm, rrm = Hm.pcg(dev(B), X, rtol=1e-8, maxit=1000, nrhs=k)
    Xm = host(X).reshape(n, k)
    H1 = amge.Hierarchy(prod, precond_bits=32, resid_bits=64)
    errs = []
    for j in range(k):
        x = torch.zeros(n, dtype=torch.float64, device="cuda")
        H1.pcg(dev(np.ascontiguousarray(B[:, j])), x, rtol=1e-8, maxit=1000)
        xj = host(x)
        errs.append(float(np.linalg.norm(Xm[:, j] - xj) / np.linalg.norm(xj)))
    print(f"batched curl n=24 jumps: FP64 {it64}, FP32 + FP64 fine residual {itm}; vs single column "
          f"{[f'{e:.1e}' for e in errs]}")
    assert st == 0 and max(rrm) <= 1e-8
    assert all(itm[j] <= it64[j] + 3 for j in range(k))
    assert max(errs) <= 1e-6
    for H in (H64, Hm, H1):
        H.close()
