"""Full-size parity in the launch configuration of the benchmark, through the C ABI:
the 64^3 H(curl) 5-level problem (one right-hand side; FP32 and FP64 V-cycles) and the
48^3 H(div) 5-level problem with a 32-column block.

Same inputs: the GPU hierarchies are set up from the oracle's own level matrices (built
by oracle.hierarchy at full size), so only the solve phase differs.  Both workloads have
unit coefficients, where the oracle's reformulation spread (tests/reformulation.py) is
~1e-13, so the FP64 bar is the plain 1e-10:
* the fine-level kernels the benchmark times (A_1 product, l1-Jacobi sweep and residual;
  A_1 has 30.3 M entries, so the eight-deep unrolled instances run) per entry against
  the oracle's A_1, FP64 1e-13 and FP32 1e-5 relative to |A||x| + |b|;
* one V-cycle (FP64 <= 1e-10 relative; FP32 energy-norm error printed, <= 1e-3);
* PCG: iteration counts at rtol 1e-8 within +-1, and the iterate after the oracle's count
  within 1e-10 (FP64 preconditioner); FP32 preconditioner within +3 iterations and 1e-6
  of the oracle solution (printed);
* the batched block: sampled columns (first, middle, last) of the 32-column FP64 solve
  against the oracle's single-column PCG, the FP32 block the same way to 1e-6;
* properties that need no oracle: symmetry and positivity of B;
* the symmetric Gauss-Seidel smoothers at full size (colour order; l1-scaled block): one
  smoother application and PCG against the oracle's sweeps.
"""
import numpy as np
import pytest

from paper_2107_05613_amd import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

torch = pytest.importorskip("torch")

SAMPLED = (0, 16, 31)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


class Full:
    def __init__(self, name, max_rhs=1):
        import time
        from oracle.hierarchy import build_hierarchy
        from oracle.solve import Multilevel
        from paper_2107_05613_amd import amge
        w = W.WORKLOADS[name]
        print(f"\n[fullsize] {w.name}: building the oracle hierarchy", flush=True)
        t0 = time.perf_counter()
        a, b = W.coefficients(w)
        H = build_hierarchy(w.kind, w.n, w.levels, a, b, check_targets=False)
        self.ml = Multilevel.from_hierarchy(H)
        L = len(H.A)
        levels = [(H.A[k], H.D[k], H.P[k] if k < L - 1 else None) for k in range(L)]
        print(f"[fullsize] oracle hierarchy {[A.shape[0] for A in H.A]} in {time.perf_counter() - t0:.0f} s; "
              f"GPU set-up from its matrices", flush=True)
        self.gpu = {bits: amge.Hierarchy(levels, precond_bits=bits, max_rhs=max_rhs) for bits in (32, 64)}
        self.w, self.H, self.A = w, H, H.A[0]
        self._sol = {}

    def oracle_pcg(self, b, key, **kw):
        """Oracle PCG on b (cached by key): (x, iterations)."""
        from oracle.solve import pcg
        if key not in self._sol:
            x, it, _ = pcg(self.A, b, self.ml, **kw)
            self._sol[key] = (x, it)
        return self._sol[key]


@pytest.fixture(scope="module")
def curl64():
    return Full("curl_n64_l5")


@pytest.fixture(scope="module")
def div48():
    return Full("div_n48_l5_rhs32", max_rhs=32)


def test_fullsize_fine_kernels(curl64):
    """a1 + a2 at full size: the A_1 product, the l1-Jacobi sweep and the residual (the
    launches the benchmark times) on every row against the oracle's A_1."""
    from paper_2107_05613_amd import amge
    f = curl64
    A, ml = f.A, f.ml
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 1, A.shape[0])
    b = rng.uniform(-1, 1, A.shape[0])
    Ax = A @ x
    dinv = 1.0 / ml.levels[0].d
    refs = {amge.OP_A: Ax, amge.OP_SWEEP: x + dinv * (b - Ax), amge.OP_RESID: b - Ax}
    absAx = abs(A) @ np.abs(x)
    scales = {amge.OP_A: absAx, amge.OP_SWEEP: np.abs(x) + dinv * (np.abs(b) + absAx),
              amge.OP_RESID: np.abs(b) + absAx}
    out = torch.empty(A.shape[0], dtype=torch.float64, device="cuda")
    for op, ref in refs.items():
        for bits, tol in ((64, 1e-13), (32, 1e-5)):
            if op == amge.OP_A:
                f.gpu[32].level_apply(0, op, dev(x), out, precision=bits)
            else:
                f.gpu[32].level_apply(0, op, dev(b), out, x2=dev(x), precision=bits)
            e = float(np.max(np.abs(host(out) - ref) / scales[op]))
            print(f"A_1 ({A.shape[0]} rows, {A.nnz} nnz) op {op} FP{bits}: max error / scale = {e:.1e}")
            assert e <= tol, (op, bits)


def test_fullsize_vcycle(curl64):
    """Algorithm 4.1 at full size against the oracle's V-cycle."""
    f = curl64
    b = W.rhs(f.A.shape[0], f.w.rhs_seed)[:, 0]
    ref = f.ml.vcycle(b)
    z = torch.empty(f.A.shape[0], dtype=torch.float64, device="cuda")
    f.gpu[64].vcycle(dev(b), z)
    e64 = float(np.max(np.abs(host(z) - ref)) / np.max(np.abs(ref)))
    f.gpu[32].vcycle(dev(b), z)
    d = host(z) - ref
    en = float(np.sqrt(d @ (f.A @ d)) / np.sqrt(ref @ (f.A @ ref)))
    print(f"V-cycle vs oracle: FP64 {e64:.1e} (max-norm relative), FP32 {en:.1e} (energy norm)")
    assert e64 <= 1e-10
    assert en <= 1e-3


def test_fullsize_pcg(curl64):
    """a7 at full size: FP64 PCG takes the oracle's iteration count (+-1) and, after that
    count, matches its iterate to 1e-10; the FP32-preconditioned solve (the benchmark
    step) converges within +3 iterations and 1e-6 of the oracle's solution."""
    f = curl64
    b = W.rhs(f.A.shape[0], f.w.rhs_seed)[:, 0]
    xo, ito = f.oracle_pcg(b, "rhs0", rtol=f.w.rtol)
    x = torch.zeros(f.A.shape[0], dtype=torch.float64, device="cuda")
    status, it, rr = f.gpu[64].pcg(dev(b), x, rtol=f.w.rtol, maxit=500)
    assert status == 0 and abs(it[0] - ito) <= 1, (it, ito)
    f.gpu[64].pcg(dev(b), x, rtol=0.0, maxit=ito)
    e64 = float(np.linalg.norm(host(x) - xo) / np.linalg.norm(xo))
    status, it32, rr32 = f.gpu[32].pcg(dev(b), x, rtol=f.w.rtol, maxit=500)
    x32 = host(x)
    e32 = float(np.linalg.norm(x32 - xo) / np.linalg.norm(xo))
    res = float(np.linalg.norm(b - f.A @ x32) / np.linalg.norm(b))
    print(f"oracle {ito} iterations; FP64 {it[0]} iterations, fixed-count error {e64:.1e}; "
          f"FP32-preconditioned {it32[0]} iterations, error vs oracle {e32:.1e}, true l2 residual {res:.1e}")
    assert e64 <= 1e-10
    assert status == 0 and rr32[0] <= f.w.rtol and it32[0] <= ito + 3
    assert e32 <= 1e-6


def test_fullsize_vcycle_symmetric(curl64):
    """Algorithm 4.1 at full size (FP64): r2 . B r1 = r1 . B r2 and r . B r > 0."""
    f = curl64
    n = f.A.shape[0]
    rng = np.random.default_rng(5)
    r1, r2 = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
    z1 = torch.empty(n, dtype=torch.float64, device="cuda")
    z2 = torch.empty_like(z1)
    f.gpu[64].vcycle(dev(r1), z1)
    f.gpu[64].vcycle(dev(r2), z2)
    b1, b2 = host(z1), host(z2)
    s12, s21 = r2 @ b1, r1 @ b2
    scale = np.sqrt((r1 @ b1) * (r2 @ b2))
    print(f"symmetry defect {abs(s12 - s21) / scale:.1e}")
    assert r1 @ b1 > 0 and r2 @ b2 > 0
    assert abs(s12 - s21) <= 1e-10 * scale


def test_fullsize_symgs(curl64):
    """f2 at full size: the symmetric Gauss-Seidel smoother (the launches the benchmark's
    Gauss-Seidel leg times) on hierarchies set up from the oracle's matrices.  One hybrid
    smoother application on the fine level against the oracle's colour-order sweep (FP64
    within 1e-10, FP32 within 1e-4, max-norm relative), and PCG: FP64 iteration count
    +-1 and the iterate after the oracle's count within 1e-10; FP32 within +3 iterations
    and 1e-6 of the oracle's solution."""
    import time
    from oracle.solve import Multilevel, pcg
    from paper_2107_05613_amd import amge
    f = curl64
    H = f.H
    L = len(H.A)
    t0 = time.perf_counter()
    ml = Multilevel(H.A, H.D, H.P, smoother="symgs")
    print(f"oracle Gauss-Seidel set-up (colourings) {time.perf_counter() - t0:.0f} s", flush=True)
    levels = [(H.A[k], H.D[k], H.P[k] if k < L - 1 else None) for k in range(L)]
    gpu = {bits: amge.Hierarchy(levels, precond_bits=bits, smoother="symgs") for bits in (32, 64)}
    n = f.A.shape[0]
    rng = np.random.default_rng(6)
    b, x0 = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
    ref = ml.smooth(ml.levels[0], b, x0)
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    err = {}
    for bits in (64, 32):
        gpu[bits].level_apply(0, amge.OP_SMOOTH, dev(b), out, x2=dev(x0), precision=bits)
        err[bits] = float(np.max(np.abs(host(out) - ref)) / np.max(np.abs(ref)))
    rhs = W.rhs(n, f.w.rhs_seed)[:, 0]
    t0 = time.perf_counter()
    xo, ito, _ = pcg(f.A, rhs, ml, rtol=f.w.rtol)
    print(f"oracle Gauss-Seidel PCG {ito} iterations in {time.perf_counter() - t0:.0f} s", flush=True)
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    status, it, _ = gpu[64].pcg(dev(rhs), x, rtol=f.w.rtol, maxit=500)
    assert status == 0 and abs(it[0] - ito) <= 1, (it, ito)
    gpu[64].pcg(dev(rhs), x, rtol=0.0, maxit=ito)
    e64 = float(np.linalg.norm(host(x) - xo) / np.linalg.norm(xo))
    status32, it32, rr32 = gpu[32].pcg(dev(rhs), x, rtol=f.w.rtol, maxit=500)
    e32 = float(np.linalg.norm(host(x) - xo) / np.linalg.norm(xo))
    print(f"Gauss-Seidel smoother vs oracle: FP64 {err[64]:.1e}, FP32 {err[32]:.1e}; PCG oracle {ito}, FP64 "
          f"{it[0]} (fixed-count error {e64:.1e}), FP32 {it32[0]} (error {e32:.1e})")
    assert err[64] <= 1e-10 and err[32] <= 1e-4
    assert e64 <= 1e-10
    assert status32 == 0 and rr32[0] <= f.w.rtol and it32[0] <= ito + 3 and e32 <= 1e-6
    for h in gpu.values():
        h.close()


def test_fullsize_blockgs(curl64):
    """The l1-scaled symmetric block Gauss-Seidel smoother at full size (the launches the
    benchmark times with that smoother: 64-row blocks over 1,872,064 rows) on
    hierarchies set up from the oracle's matrices.  One hybrid smoother application on
    the fine level against the oracle's block sweep (FP64 within 1e-10, FP32 within 1e-4,
    max-norm relative), and PCG: FP64 iteration count +-1 and the iterate after the
    oracle's count within 1e-10; FP32 within +3 iterations and 1e-6 of the oracle's
    solution."""
    import time
    from oracle.solve import Multilevel, pcg
    from paper_2107_05613_amd import amge
    f = curl64
    H = f.H
    L = len(H.A)
    t0 = time.perf_counter()
    ml = Multilevel(H.A, H.D, H.P, smoother="l1blockgs", gs_block=64)
    print(f"oracle block Gauss-Seidel set-up (colourings) {time.perf_counter() - t0:.0f} s", flush=True)
    levels = [(H.A[k], H.D[k], H.P[k] if k < L - 1 else None) for k in range(L)]
    gpu = {bits: amge.Hierarchy(levels, precond_bits=bits, smoother="l1blockgs") for bits in (32, 64)}
    n = f.A.shape[0]
    rng = np.random.default_rng(6)
    b, x0 = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
    ref = ml.smooth(ml.levels[0], b, x0)
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    err = {}
    for bits in (64, 32):
        gpu[bits].level_apply(0, amge.OP_SMOOTH, dev(b), out, x2=dev(x0), precision=bits)
        err[bits] = float(np.max(np.abs(host(out) - ref)) / np.max(np.abs(ref)))
    rhs = W.rhs(n, f.w.rhs_seed)[:, 0]
    t0 = time.perf_counter()
    xo, ito, _ = pcg(f.A, rhs, ml, rtol=f.w.rtol)
    print(f"oracle block Gauss-Seidel PCG {ito} iterations in {time.perf_counter() - t0:.0f} s", flush=True)
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    status, it, _ = gpu[64].pcg(dev(rhs), x, rtol=f.w.rtol, maxit=500)
    assert status == 0 and abs(it[0] - ito) <= 1, (it, ito)
    gpu[64].pcg(dev(rhs), x, rtol=0.0, maxit=ito)
    e64 = float(np.linalg.norm(host(x) - xo) / np.linalg.norm(xo))
    status32, it32, rr32 = gpu[32].pcg(dev(rhs), x, rtol=f.w.rtol, maxit=500)
    e32 = float(np.linalg.norm(host(x) - xo) / np.linalg.norm(xo))
    print(f"block Gauss-Seidel smoother vs oracle: FP64 {err[64]:.1e}, FP32 {err[32]:.1e}; PCG oracle {ito}, "
          f"FP64 {it[0]} (fixed-count error {e64:.1e}), FP32 {it32[0]} (error {e32:.1e})")
    assert err[64] <= 1e-10 and err[32] <= 1e-4
    assert e64 <= 1e-10
    assert status32 == 0 and rr32[0] <= f.w.rtol and it32[0] <= ito + 3 and e32 <= 1e-6
    for h in gpu.values():
        h.close()


def test_fullsize_batched_pcg(div48):
    """a8 at full size: the 32-column block in one batched call.  FP64: sampled columns
    take the oracle's count (+-1) at rtol 1e-8 and match its iterate after that count to
    1e-10.  FP32 (the benchmark's block solve): every column converges, sampled columns
    within +3 iterations and 1e-6 of the oracle's solution."""
    f = div48
    n, k = f.A.shape[0], f.w.nrhs
    B = W.rhs(n, f.w.rhs_seed, k)
    X = torch.zeros(n * k, dtype=torch.float64, device="cuda")
    ref = {j: f.oracle_pcg(np.ascontiguousarray(B[:, j]), j, rtol=f.w.rtol) for j in SAMPLED}
    status, its, rrs = f.gpu[64].pcg(dev(B), X, rtol=f.w.rtol, maxit=500, nrhs=k)
    assert status == 0 and max(rrs) <= f.w.rtol
    for j in SAMPLED:
        assert abs(its[j] - ref[j][1]) <= 1, (j, its[j], ref[j][1])
    kfix = max(r[1] for r in ref.values())
    f.gpu[64].pcg(dev(B), X, rtol=0.0, maxit=kfix, nrhs=k)
    Xs = host(X).reshape(n, k)
    e64 = {}
    for j in SAMPLED:
        xo = ref[j][0] if ref[j][1] == kfix else f.oracle_pcg(np.ascontiguousarray(B[:, j]), ("fixed", j),
                                                                 fixed_iters=kfix)[0]
        e64[j] = float(np.linalg.norm(Xs[:, j] - xo) / np.linalg.norm(xo))
    status, its32, rrs32 = f.gpu[32].pcg(dev(B), X, rtol=f.w.rtol, maxit=500, nrhs=k)
    Xs = host(X).reshape(n, k)
    e32 = {j: float(np.linalg.norm(Xs[:, j] - ref[j][0]) / np.linalg.norm(ref[j][0])) for j in SAMPLED}
    print(f"oracle iterations {[ref[j][1] for j in SAMPLED]}; FP64 block {min(its)}..{max(its)}, fixed-count "
          f"errors {[f'{e:.1e}' for e in e64.values()]}; FP32 block {min(its32)}..{max(its32)}, errors vs oracle "
          f"{[f'{e:.1e}' for e in e32.values()]}")
    assert max(e64.values()) <= 1e-10
    assert status == 0 and max(rrs32) <= f.w.rtol
    assert all(its32[j] <= ref[j][1] + 3 for j in SAMPLED)
    assert max(e32.values()) <= 1e-6


def test_fullsize_batched_vcycle_symmetric(div48):
    """Batched Algorithm 4.1 at full size (FP64): R^T (B R) is symmetric with a positive
    diagonal."""
    f = div48
    n = f.A.shape[0]
    k = 8
    R = np.random.default_rng(9).uniform(-1, 1, (n, k))
    Z = torch.empty(n * k, dtype=torch.float64, device="cuda")
    f.gpu[64].vcycle(dev(R), Z, nrhs=k)
    S = R.T @ host(Z).reshape(n, k)
    d = np.sqrt(np.abs(np.diag(S)))
    defect = np.max(np.abs(S - S.T) / np.outer(d, d))
    print(f"batched V-cycle symmetry defect {defect:.1e}")
    assert np.all(np.diag(S) > 0)
    assert defect <= 1e-10
