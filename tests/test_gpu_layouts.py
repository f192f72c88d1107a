"""Set-up work on the device against the same work on the host, bit for bit.

* Sliced-ELL entry arrays (k_slice_range, k_sell_fill) filled from a staged copy of each
  CSR matrix; AMGE_HOST_LAYOUT=1 builds the same layout on the host.  Layouts are
  integer and byte work.
* The set-up products D^T A, D^T A D and P^T A (spgemm_device.hip); AMGE_HOST_PRODUCTS=1
  forms them on the host.  The device products sum in the host product's order with
  separately rounded operations, so they are equal bit for bit.

Every level operator, smoother, V-cycle and PCG result of a hierarchy set up either way
must be identical bit for bit (same kernels, same arrays).  Covered: 16-bit column
offsets and 32-bit indices (AMGE_INDEX32=1), split-row operators, incidence matrices,
the colour blocks of the Gauss-Seidel smoother and the batched layouts."""
import os

import numpy as np
import pytest

from paper_2107_05613_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


SWITCHES = ("AMGE_HOST_LAYOUT", "AMGE_HOST_PRODUCTS")


def _hier(levels, host, **kw):
    """Hierarchy set up with every set-up step on the host (host=True) or the device."""
    from paper_2107_05613_amd import amge
    old = {k: os.environ.get(k) for k in SWITCHES}
    for k in SWITCHES:
        os.environ[k] = "1" if host else "0"
    try:
        return amge.Hierarchy(levels, **kw)
    finally:
        for k, v in old.items():
            if v is None:
                del os.environ[k]
            else:
                os.environ[k] = v


def _levels(kind, n, L, coef):
    from paper_2107_05613_amd import amge
    a, b = W.coefficients(W.Workload("t", kind, n, L, coef))
    return amge.build_problem(kind, n, L, a, b)


def _same(a, b):
    return torch.equal(a, b)


SPECS = [("curl", 12, 3, "unit", "l1jacobi", False), ("div", 16, 4, "blocks", "symgs", False),
         ("curl", 16, 3, "blocks", "l1jacobi", True)]


@pytest.mark.parametrize("kind,n,L,coef,smoother,index32", SPECS)
def test_level_operators_bitwise(kind, n, L, coef, smoother, index32, monkeypatch):
    from paper_2107_05613_amd import amge
    if index32:
        monkeypatch.setenv("AMGE_INDEX32", "1")
    lv = _levels(kind, n, L, coef)
    kw = dict(precond_bits=64, tail_rows=0, smoother=smoother)
    Hh, Hd = _hier(lv, True, **kw), _hier(lv, False, **kw)
    rng = np.random.default_rng(3)
    dev = lambda v: torch.from_numpy(v).cuda()
    ops = 0
    for k in range(L - 1):
        nk, mk, nc = lv[k][0].shape[0], lv[k][1].shape[1], lv[k][2].shape[1]
        x = {s: dev(rng.uniform(-1, 1, s)) for s in {nk, mk, nc}}
        for op, nin, nout, two in ((amge.OP_A, nk, nk, False), (amge.OP_AHAT, mk, mk, False),
                                   (amge.OP_D, mk, nk, False), (amge.OP_DT, nk, mk, False),
                                   (amge.OP_P, nc, nk, False), (amge.OP_PT, nk, nc, False),
                                   (amge.OP_SWEEP, nk, nk, True), (amge.OP_RESID, nk, nk, True),
                                   (amge.OP_SMOOTH, nk, nk, True), (amge.OP_SMOOTHT, nk, nk, True)):
            x2 = dev(rng.uniform(-1, 1, nk)) if two else None
            for prec in (64, 32):
                oh = torch.empty(nout, dtype=torch.float64, device="cuda")
                od = torch.empty_like(oh)
                Hh.level_apply(k, op, x[nin], oh, x2=x2, precision=prec)
                Hd.level_apply(k, op, x[nin], od, x2=x2, precision=prec)
                assert _same(oh, od), (k, op, prec)
                ops += 1
    print(f"{kind} n={n} {smoother}{' int32' if index32 else ''}: {ops} operator results identical")


@pytest.mark.parametrize("kind,n,L,coef,smoother,nrhs", [("curl", 12, 3, "unit", "l1jacobi", 1),
                                                         ("div", 16, 4, "blocks", "symgs", 1),
                                                         ("div", 12, 3, "blocks", "l1jacobi", 8)])
def test_solves_bitwise(kind, n, L, coef, smoother, nrhs):
    lv = _levels(kind, n, L, coef)
    kw = dict(precond_bits=32, smoother=smoother, max_rhs=nrhs)
    Hh, Hd = _hier(lv, True, **kw), _hier(lv, False, **kw)
    n1 = lv[0][0].shape[0]
    b = torch.from_numpy(np.random.default_rng(4).uniform(-1, 1, n1 * nrhs)).cuda()
    zh, zd = torch.empty_like(b), torch.empty_like(b)
    Hh.vcycle(b, zh, nrhs=nrhs)
    Hd.vcycle(b, zd, nrhs=nrhs)
    assert _same(zh, zd)
    xh, xd = torch.zeros_like(b), torch.zeros_like(b)
    rh = Hh.pcg(b, xh, rtol=1e-8, nrhs=nrhs)
    rd = Hd.pcg(b, xd, rtol=1e-8, nrhs=nrhs)
    assert rh == rd and _same(xh, xd)
    print(f"{kind} n={n} {smoother} nrhs={nrhs}: V-cycle and PCG ({rh[1]} iterations) identical")


def test_fine_level_full_size_bitwise():
    """The 64^3 H(curl) hierarchy: the fine-level kernels the solve times (deep-unrolled
    sliced ELL of A_1) from device-built and host-built layouts."""
    from paper_2107_05613_amd import amge
    w = W.WORKLOADS["curl_n64_l5"]
    a, b = W.coefficients(w)
    lv = amge.build_problem(w.kind, w.n, w.levels, a, b)
    kw = dict(precond_bits=32)
    Hh, Hd = _hier(lv, True, **kw), _hier(lv, False, **kw)
    n1 = lv[0][0].shape[0]
    rng = np.random.default_rng(5)
    x, x2 = (torch.from_numpy(rng.uniform(-1, 1, n1)).cuda() for _ in range(2))
    for op in (amge.OP_A, amge.OP_SWEEP, amge.OP_RESID, amge.OP_SMOOTH):
        for prec in (64, 32):
            oh, od = torch.empty_like(x), torch.empty_like(x)
            Hh.level_apply(0, op, x, oh, x2=x2, precision=prec)
            Hd.level_apply(0, op, x, od, x2=x2, precision=prec)
            assert _same(oh, od), (op, prec)
    xh, xd = torch.zeros_like(x), torch.zeros_like(x)
    assert Hh.pcg(x, xh) == Hd.pcg(x, xd) and _same(xh, xd)


@pytest.mark.parametrize("kind,n,L,coef", [("curl", 16, 4, "blocks"), ("div", 16, 4, "unit")])
def test_builder_galerkin_products_bitwise(kind, n, L, coef):
    """Galerkin coarse matrices P^T (A P) formed on the device (AMGE_BUILD_DEVICE) equal the
    host builder's bit for bit (unweighted extensions: the local problems are shared, so
    only the products differ in where they run)."""
    from paper_2107_05613_amd import amge
    a, b = W.coefficients(W.Workload("t", kind, n, L, coef))
    dev = amge.build_problem(kind, n, L, a, b, device=True)
    hst = amge.build_problem(kind, n, L, a, b)
    for k in range(L):
        for i in range(3):
            if hst[k][i] is None:
                continue
            Md, Mh = dev[k][i], hst[k][i]
            assert Md.shape == Mh.shape
            assert np.array_equal(Md.rowptr, Mh.rowptr) and np.array_equal(Md.col, Mh.col), (k, i)
            assert np.array_equal(Md.val.view(np.uint64), Mh.val.view(np.uint64)), (k, i)


def test_permuted_fine_level_uses_32bit_indices():
    """A random renumbering of the fine-level dofs (A -> Q^T A Q, D -> Q^T D, P -> Q^T P)
    spreads every slice's columns over the whole range (238,688 dofs), so the fine-level
    layouts need 32-bit column indices (k_slice_range flags them, k_sell_fill writes
    them).  The device-filled layouts equal the host-built ones bit for bit, and the
    renumbered problem is the same problem: FP64 PCG takes the same iteration count (+-1)
    and its solution, renumbered back, is within 1e-10 of the original one's."""
    import scipy.sparse as sp
    from paper_2107_05613_amd import amge
    lv = _levels("curl", 32, 3, "unit")   # unit coefficients: FP64 reorderings agree to ~1e-13
    n1 = lv[0][0].shape[0]
    perm = np.random.default_rng(17).permutation(n1)
    Q = sp.csr_matrix((np.ones(n1), (perm, np.arange(n1))), shape=(n1, n1))   # Q e_i = e_perm[i]
    A, D, P = (m.to_scipy() for m in lv[0])
    plv = [((Q.T @ A @ Q).tocsr(), (Q.T @ D).tocsr(), (Q.T @ P).tocsr())] + \
          [tuple(None if m is None else m.to_scipy() for m in lk) for lk in lv[1:]]
    kw = dict(precond_bits=64)
    Hh, Hd = _hier(plv, True, **kw), _hier(plv, False, **kw)
    b = W.rhs(n1, 2)[:, 0]
    bp = Q.T @ b
    rng = np.random.default_rng(1)
    x = torch.from_numpy(rng.uniform(-1, 1, n1)).cuda()
    for op in (amge.OP_A, amge.OP_SWEEP, amge.OP_RESID):
        oh, od = torch.empty_like(x), torch.empty_like(x)
        x2 = torch.from_numpy(rng.uniform(-1, 1, n1)).cuda()
        Hh.level_apply(0, op, x, oh, x2=x2, precision=64)
        Hd.level_apply(0, op, x, od, x2=x2, precision=64)
        assert _same(oh, od), op
    H0 = amge.Hierarchy(lv, **kw)
    x0 = torch.zeros(n1, dtype=torch.float64, device="cuda")
    xp = torch.zeros_like(x0)
    _, it0, _ = H0.pcg(torch.from_numpy(b).cuda(), x0, rtol=1e-8)
    _, itp, _ = Hd.pcg(torch.from_numpy(bp).cuda(), xp, rtol=1e-8)
    H0.pcg(torch.from_numpy(b).cuda(), x0, rtol=0.0, maxit=it0[0])
    Hd.pcg(torch.from_numpy(bp).cuda(), xp, rtol=0.0, maxit=it0[0])
    xs = Q @ xp.cpu().numpy()
    e = float(np.linalg.norm(xs - x0.cpu().numpy()) / np.linalg.norm(x0.cpu().numpy()))
    print(f"renumbered fine level: iterations {itp[0]} vs {it0[0]}, solution difference {e:.1e}")
    assert abs(itp[0] - it0[0]) <= 1 and e <= 1e-10
    for h in (Hh, Hd, H0):
        h.close()


def test_set_up_product_with_a_row_beyond_the_device_tables():
    """A set-up product with a row of more distinct columns than the largest device hash
    table (4096): D^T A and D^T A D of a 'star' derivative whose first column touches all
    6000 rows.  That product runs on the host instead; the hierarchy equals the one set up
    with every product on the host, bit for bit (auxiliary operator and V-cycle)."""
    import scipy.sparse as sp
    from paper_2107_05613_amd import amge
    n = 6000
    rng = np.random.default_rng(4)
    off = sp.random(n, n, density=4.0 / n, random_state=5, format="csr")
    off = (off + off.T) * 0.1
    A = (off + sp.diags(np.asarray(abs(off).sum(axis=1)).ravel() + 1.0)).tocsr()
    # D: column 0 touches every row (the star), plus a second entry per row
    rows = np.concatenate([np.arange(n), np.arange(n)])
    cols = np.concatenate([np.zeros(n, dtype=int), 1 + (np.arange(n) % 1999)])
    vals = np.concatenate([np.ones(n), -np.ones(n)])
    D = sp.csr_matrix((vals, (rows, cols)), shape=(n, 2000))
    P = sp.csr_matrix((np.ones(n), (np.arange(n), np.arange(n) // 60)), shape=(n, 100))
    Ac = (P.T @ A @ P).tocsr()
    Dc = sp.identity(100, format="csr")
    levels = [(A, D, P), (Ac, Dc, None)]
    Hh, Hd = _hier(levels, True, precond_bits=64), _hier(levels, False, precond_bits=64)
    y = torch.from_numpy(rng.uniform(-1, 1, 2000)).cuda()
    oh, od = torch.empty_like(y), torch.empty_like(y)
    Hh.level_apply(0, amge.OP_AHAT, y, oh, precision=64)
    Hd.level_apply(0, amge.OP_AHAT, y, od, precision=64)
    ref = (D.T @ A @ D) @ y.cpu().numpy()
    assert _same(oh, od)
    assert np.max(np.abs(od.cpu().numpy() - ref)) <= 1e-12 * np.max(np.abs(ref))
    b = torch.from_numpy(rng.uniform(-1, 1, n)).cuda()
    zh, zd = torch.empty_like(b), torch.empty_like(b)
    Hh.vcycle(b, zh)
    Hd.vcycle(b, zd)
    assert _same(zh, zd)
    Hh.close()
    Hd.close()
