"""The no-allocation V-cycle (amge_vcycle_static), through the C ABI.

It computes what amge_vcycle computes on one column, with the level work vectors in the
library's static device scratch instead of a context's buffers; the kernels and their
order are the same, so the bar is bitwise equality with amge_vcycle (with the l1-Jacobi
and with the block Gauss-Seidel point smoother).  Checked on two
calls in a row, the second on a smaller hierarchy (the scratch keeps the first call's
contents), then again on the first; a hierarchy whose work vectors exceed the scratch
is refused with AMGE_ERR_ARG before anything runs; torch's allocator sees no
allocation during the calls.
"""
import numpy as np
import pytest

from paper_2107_05613_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def build(kind, n, L, coef, bits, smoother="l1jacobi"):
    from paper_2107_05613_amd import amge
    w = W.Workload("t", kind, n, L, coef)
    a, b = W.coefficients(w)
    print(f"\n[no-alloc] {kind} n={n} levels={L} FP{bits} smoother {smoother}", flush=True)
    return amge.Hierarchy(amge.build_problem(kind, n, L, a, b), precond_bits=bits, smoother=smoother)


@pytest.mark.parametrize("smoother", ["l1jacobi", "l1blockgs"])
def test_static_vcycle_matches_vcycle(smoother):
    big = build("curl", 12, 3, "unit", 32, smoother)
    small = build("div", 8, 3, "blocks", 64, smoother)
    ref = {}
    rhs = {}
    for name, H in (("big", big), ("small", small)):
        n = H.rows[0]
        rhs[name] = torch.from_numpy(W.rhs(n, 5)[:, 0]).cuda()
        ref[name] = torch.empty_like(rhs[name])
        H.vcycle(rhs[name], ref[name])
    torch.cuda.synchronize()
    out = {k: torch.full_like(v, np.nan) for k, v in rhs.items()}
    m0 = torch.cuda.memory_allocated()
    for name, H in (("big", big), ("small", small), ("big", big)):
        out[name].fill_(np.nan)
        H.vcycle_static(rhs[name], out[name])
        torch.cuda.synchronize()
        assert torch.equal(out[name], ref[name]), name
    assert torch.cuda.memory_allocated() == m0
    big.close()
    small.close()


def test_static_vcycle_refuses_oversized_work():
    from paper_2107_05613_amd import amge
    # 48^3 H(div) in FP64: 1,340,928 fine rows, ~80 MB of single-column work vectors
    H = build("div", 48, 5, "unit", 64)
    r = torch.ones(H.rows[0], dtype=torch.float64, device="cuda")
    z = torch.zeros_like(r)
    with pytest.raises(amge.AmgeError) as e:
        H.vcycle_static(r, z)
    assert e.value.code == -1
    torch.cuda.synchronize()
    assert not torch.any(z != 0)
    H.close()
