"""GPU parity of the symmetric Gauss-Seidel smoother (opts.smoother = AMGE_SMOOTHER_SYM_GS:
rows coloured greedily, colours relaxed in increasing then decreasing order; the
smoother of the paper's experiments, section 4.1) against the oracle's
(oracle.solve, smoother="symgs"), through the C ABI, on hierarchies set up from the
oracle's own level matrices.  Bars as in test_gpu_parity.py: FP64 within max(1e-10, 3 s),
s the oracle's reformulation spread for this smoother; iteration counts +-1; the FP32
V-cycle within +3 iterations and 1e-6 of the oracle solution.  The library relaxes the
colour that ends a half-sweep once instead of twice (the second relaxation has a zero
residual): the same operator, different rounding."""
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


class GsCase:
    def __init__(self, kind, n, L, coef):
        from oracle.hierarchy import build_hierarchy
        from oracle.solve import Multilevel, pcg
        from paper_2107_05613_amd import amge
        print(f"\n[gs case] {kind} n={n} levels={L} coef={coef}", flush=True)
        a, b = W.coefficients(W.Workload("t", kind, n, L, coef))
        self.H = build_hierarchy(kind, n, L, a, b, check_targets=False)
        self.levels = [(self.H.A[k], self.H.D[k], self.H.P[k] if k < L - 1 else None) for k in range(L)]
        self.ml = Multilevel.from_hierarchy(self.H, smoother="symgs")
        self.b = W.rhs(self.H.A[0].shape[0], 0)[:, 0]
        self.xo, self.ito, _ = pcg(self.H.A[0], self.b, self.ml, rtol=1e-8)
        self.bar = {k: fp64_bar(v) for k, v in spreads(self.H, self.b, self.ito, smoother="symgs").items()}
        self.gpu = {bits: amge.Hierarchy(self.levels, precond_bits=bits, smoother="symgs") for bits in (64, 32)}
        print(f"[gs case] oracle {self.ito} iterations; bars {self.bar}", flush=True)


def case(*spec):
    if spec not in _CASES:
        _CASES[spec] = GsCase(*spec)
    return _CASES[spec]


SPECS = [("curl", 8, 3, "blocks"), ("div", 8, 3, "blocks"), ("curl", 12, 3, "unit"), ("div", 16, 3, "unit")]


@pytest.mark.parametrize("spec", SPECS)
def test_gs_smoother_application(spec):
    """One application of the hybrid smoother with Gauss-Seidel point smoothers, and of
    its transpose, on every non-coarsest level."""
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
            print(f"level {k} op {op}: GS smoother error fp64 {e64:.1e} fp32 {e32:.1e}")
            assert e64 <= c.bar["smooth"] and e32 <= 1e-4, (k, op)


@pytest.mark.parametrize("spec", SPECS)
def test_gs_vcycle_and_pcg(spec):
    """Algorithm 4.1 with the Gauss-Seidel hybrid smoother (folded and unfolded coarse
    tail), and PCG around it: FP64 parity, FP32 convergence."""
    from paper_2107_05613_amd import amge
    c = case(*spec)
    ref = c.ml.vcycle(c.b)
    z = torch.empty_like(dev(c.b))
    H0 = amge.Hierarchy(c.levels, precond_bits=64, smoother="symgs", tail_rows=0)
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


def test_gs_smoother_arguments():
    """The Gauss-Seidel smoother runs single-column contexts: max_rhs > 1 is refused."""
    from paper_2107_05613_amd import amge
    c = case("curl", 8, 3, "blocks")
    with pytest.raises(amge.AmgeError) as e:
        amge.Hierarchy(c.levels, smoother="symgs", max_rhs=2)
    assert e.value.code == -1
