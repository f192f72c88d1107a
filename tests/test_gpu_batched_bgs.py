"""GPU parity of the batched path with the l1-scaled symmetric block Gauss-Seidel
smoother (AMGE_SMOOTHER_BLOCK_GS, max_rhs > 1) through the C ABI.

Each wave of a batched sweep holds a 64-row block and V consecutive columns; every
column goes through the arithmetic of the single-column sweep.  Bars, per column, as
in test_gpu_batched.py, against the oracle's block Gauss-Seidel V-cycle and PCG
(oracle.solve, smoother="l1blockgs", gs_block=64) on the oracle's own level matrices:
FP64 V-cycle and fixed-count PCG iterate within max(1e-10, 3 s) (s: the oracle's
reformulation spread for this smoother), iteration counts +-1; FP32 V-cycle energy-norm
error 1e-3 (5e-2 where the cancellation factor reaches 1e6); FP32 preconditioner within
3 iterations of the oracle's count and 1e-6 of its solution.  A column's result does not
depend on the other columns or on the block width (bitwise).
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


class Case:
    def __init__(self, kind, n, L, coef, max_rhs):
        from oracle.hierarchy import build_hierarchy
        from oracle.solve import Multilevel
        from paper_2107_05613_amd import amge
        print(f"\n[batched block gs] {kind} n={n} levels={L} coef={coef} max_rhs={max_rhs}", flush=True)
        a, b = W.coefficients(W.Workload("t", kind, n, L, coef))
        self.H = build_hierarchy(kind, n, L, a, b, check_targets=False)
        self.levels = [(self.H.A[k], self.H.D[k], self.H.P[k] if k < L - 1 else None) for k in range(L)]
        self.ml = Multilevel.from_hierarchy(self.H, smoother="l1blockgs", gs_block=64)
        self.gpu = {bits: amge.Hierarchy(self.levels, precond_bits=bits, max_rhs=max_rhs, smoother="l1blockgs")
                    for bits in (64, 32)}
        self.n1 = self.H.A[0].shape[0]
        # cancellation factor of the auxiliary matrices (FP32 V-cycle bar, as in test_gpu_batched.py)
        kap = 1.0
        for k in range(L - 1):
            A, D = self.H.A[k], self.H.D[k]
            num = abs(D).T @ (abs(A) @ (abs(D) @ np.ones(D.shape[1])))
            den = abs((D.T @ A @ D).tocsr()) @ np.ones(D.shape[1])
            kap = max(kap, float(np.max(num / den)))
        self.kappa = kap
        sp = spreads(self.H, W.rhs(self.n1, 11)[:, 0], 15, smoother="l1blockgs")
        self.tol = fp64_bar(max(sp.values()))
        print(f"[batched block gs] sizes {[A.shape[0] for A in self.H.A]}, FP64 bar {self.tol:.1e}", flush=True)


_CASES = {}


def case(*key):
    if key not in _CASES:
        _CASES[key] = Case(*key)
    return _CASES[key]


SPECS = [(("curl", 8, 3, "blocks", 8), 5), (("div", 12, 3, "unit", 32), 32), (("curl", 16, 4, "blocks", 4), 3)]


@pytest.mark.parametrize("spec,nrhs", SPECS)
def test_batched_bgs_vcycle(spec, nrhs):
    c = case(*spec)
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
    print(f"{spec} nrhs={nrhs}: FP64 worst column error {worst64:.2e} (bar {c.tol:.1e}); "
          f"FP32 worst energy-norm error {worst_en:.2e}")
    assert worst64 <= c.tol
    assert worst_en <= (1e-3 if c.kappa < 1e6 else 5e-2)


@pytest.mark.parametrize("spec,nrhs", SPECS)
def test_batched_bgs_pcg(spec, nrhs):
    from oracle.solve import pcg
    c = case(*spec)
    B = W.rhs(c.n1, 13, nrhs)
    ref = [pcg(c.H.A[0], np.ascontiguousarray(B[:, j]), c.ml, rtol=1e-8) for j in range(nrhs)]
    X = torch.zeros(c.n1 * nrhs, dtype=torch.float64, device="cuda")
    st, its, rrs = c.gpu[64].pcg(dev(B), X, rtol=1e-8, maxit=500, nrhs=nrhs)
    assert st == 0
    for j in range(nrhs):
        assert abs(its[j] - ref[j][1]) <= 1, (j, its[j], ref[j][1])
    kfix = max(r[1] for r in ref)
    c.gpu[64].pcg(dev(B), X, rtol=0.0, maxit=kfix, nrhs=nrhs)
    Xs = host(X).reshape(c.n1, nrhs)
    e64 = max(np.linalg.norm(Xs[:, j] - pcg(c.H.A[0], np.ascontiguousarray(B[:, j]), c.ml, fixed_iters=kfix)[0])
              / np.linalg.norm(ref[j][0]) for j in range(nrhs))
    st32, its32, rr32 = c.gpu[32].pcg(dev(B), X, rtol=1e-8, maxit=500, nrhs=nrhs)
    X32 = host(X).reshape(c.n1, nrhs)
    e32 = max(np.linalg.norm(X32[:, j] - ref[j][0]) / np.linalg.norm(ref[j][0]) for j in range(nrhs))
    print(f"{spec} nrhs={nrhs}: oracle iterations {[r[1] for r in ref]}, FP64 {list(its)}, fixed-count error "
          f"{e64:.1e}; FP32 {list(its32)}, error {e32:.1e}")
    assert e64 <= c.tol
    assert st32 == 0 and all(its32[j] <= ref[j][1] + 3 for j in range(nrhs)) and e32 <= 1e-6


def test_batched_bgs_column_independent_of_block():
    """Column 2 of a 3-column V-cycle (active width 4) equals the same right-hand side as
    column 0 of a 2-column V-cycle (width 2) next to other data, and column 2 of a
    4-column block equals it in a block whose other columns differ, bit for bit, in both
    precisions."""
    c = case("curl", 16, 4, "blocks", 4)
    B = W.rhs(c.n1, 17, 3)
    B2 = np.ascontiguousarray(np.stack([B[:, 2], W.rhs(c.n1, 18)[:, 0]], 1))
    for bits in (64, 32):
        Z = torch.zeros(c.n1 * 3, dtype=torch.float64, device="cuda")
        c.gpu[bits].vcycle(dev(B), Z, nrhs=3)
        Z2 = torch.zeros(c.n1 * 2, dtype=torch.float64, device="cuda")
        c.gpu[bits].vcycle(dev(B2), Z2, nrhs=2)
        assert np.array_equal(host(Z).reshape(c.n1, 3)[:, 2], host(Z2).reshape(c.n1, 2)[:, 0]), bits


def test_batched_bgs_wide_block_matches_narrow():
    """Column 21 of a 32-column V-cycle (FP32: four waves per block share its rows, four
    lanes per row; FP64: one row per lane, four columns) equals the same right-hand side
    as column 0 of a 2-column V-cycle (one column per wave), bit for bit, in both
    precisions."""
    c = case("div", 12, 3, "unit", 32)
    B = W.rhs(c.n1, 19, 32)
    B2 = np.ascontiguousarray(np.stack([B[:, 21], W.rhs(c.n1, 20)[:, 0]], 1))
    for bits in (64, 32):
        Z = torch.zeros(c.n1 * 32, dtype=torch.float64, device="cuda")
        c.gpu[bits].vcycle(dev(B), Z, nrhs=32)
        Z2 = torch.zeros(c.n1 * 2, dtype=torch.float64, device="cuda")
        c.gpu[bits].vcycle(dev(B2), Z2, nrhs=2)
        assert np.array_equal(host(Z).reshape(c.n1, 32)[:, 21], host(Z2).reshape(c.n1, 2)[:, 0]), bits


def test_batched_bgs_two_column_groups_match_narrow():
    """Column 45 of a 64-column V-cycle (FP32: two groups of 32 columns per block, each
    over four waves) equals the same right-hand side as column 0 of a 2-column V-cycle,
    bit for bit, in both precisions."""
    c = case("div", 12, 3, "unit", 64)
    B = W.rhs(c.n1, 23, 64)
    B2 = np.ascontiguousarray(np.stack([B[:, 45], W.rhs(c.n1, 24)[:, 0]], 1))
    for bits in (64, 32):
        Z = torch.zeros(c.n1 * 64, dtype=torch.float64, device="cuda")
        c.gpu[bits].vcycle(dev(B), Z, nrhs=64)
        Z2 = torch.zeros(c.n1 * 2, dtype=torch.float64, device="cuda")
        c.gpu[bits].vcycle(dev(B2), Z2, nrhs=2)
        assert np.array_equal(host(Z).reshape(c.n1, 64)[:, 45], host(Z2).reshape(c.n1, 2)[:, 0]), bits


def test_batched_bgs_dense_blocks_largest_bound():
    """A 32-column batched V-cycle on a two-level hierarchy whose fine matrix has dense
    64-row blocks (inside widths above 32: the NIN = 64 batched bodies, FP32 over four
    waves per block, FP64 one row per lane) against the oracle's block Gauss-Seidel
    V-cycle on the same level matrices: FP64 within 1e-10 (a diagonally dominant
    problem), FP32 energy-norm error within 1e-3."""
    from oracle.solve import Multilevel
    from paper_2107_05613_amd import amge
    from test_gpu_smoother_bgs import _dense_block_levels
    levels = _dense_block_levels()
    A = levels[0][0]
    n = A.shape[0]
    ml = Multilevel([lv[0] for lv in levels], [lv[1] for lv in levels], [lv[2] for lv in levels],
                    smoother="l1blockgs", gs_block=64)
    B = W.rhs(n, 29, 32)
    refs = [ml.vcycle(B[:, j]) for j in range(32)]
    for bits in (64, 32):
        H = amge.Hierarchy(levels, precond_bits=bits, max_rhs=32, smoother="l1blockgs", tail_rows=0)
        Z = torch.zeros(n * 32, dtype=torch.float64, device="cuda")
        H.vcycle(dev(B), Z, nrhs=32)
        z = host(Z).reshape(n, 32)
        if bits == 64:
            err = max(relerr(z[:, j], refs[j]) for j in range(32))
            print(f"dense blocks batched FP64: worst column error {err:.1e}")
            assert err <= 1e-10
        else:
            err = max(float(np.sqrt((z[:, j] - refs[j]) @ (A @ (z[:, j] - refs[j])) / (refs[j] @ (A @ refs[j]))))
                      for j in range(32))
            print(f"dense blocks batched FP32: worst energy-norm error {err:.1e}")
            assert err <= 1e-3
        H.close()


def test_batched_bgs_wide_column_span():
    """An 8-column batched V-cycle with 32-bit outside columns in the block layout (a
    block's outside columns span more than 65,536) against the oracle's block
    Gauss-Seidel V-cycle: FP64 within 1e-10, FP32 energy-norm error within 1e-3."""
    from oracle.solve import Multilevel
    from paper_2107_05613_amd import amge
    from test_gpu_smoother_bgs import _wide_span_levels
    levels = _wide_span_levels()
    A = levels[0][0]
    n = A.shape[0]
    ml = Multilevel([lv[0] for lv in levels], [lv[1] for lv in levels], [lv[2] for lv in levels],
                    smoother="l1blockgs", gs_block=64)
    B = W.rhs(n, 31, 8)
    refs = [ml.vcycle(B[:, j]) for j in range(8)]
    for bits in (64, 32):
        H = amge.Hierarchy(levels, precond_bits=bits, max_rhs=8, smoother="l1blockgs", tail_rows=0)
        Z = torch.zeros(n * 8, dtype=torch.float64, device="cuda")
        H.vcycle(dev(B), Z, nrhs=8)
        z = host(Z).reshape(n, 8)
        if bits == 64:
            err = max(relerr(z[:, j], refs[j]) for j in range(8))
            print(f"wide column span batched FP64: worst column error {err:.1e}")
            assert err <= 1e-10
        else:
            err = max(float(np.sqrt((z[:, j] - refs[j]) @ (A @ (z[:, j] - refs[j])) / (refs[j] @ (A @ refs[j]))))
                      for j in range(8))
            print(f"wide column span batched FP32: worst energy-norm error {err:.1e}")
            assert err <= 1e-3
        H.close()
