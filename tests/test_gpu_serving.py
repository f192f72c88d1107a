"""Serving engine (amge_server_*, through the C ABI): resident hierarchies, admission by
device memory, continuous batching of single right-hand-side requests.

Bars
* Solo vs mix: every request solved alone (the only request in the server) and inside
  a mix of requests on several hierarchies, arriving while others are in flight, gives
  the same solution, iteration count and residual.  Columns of the batched PCG share no
  arithmetic, so the bar is bitwise equality.
* Parity: requests on an FP64-preconditioner hierarchy (built by the library's own
  builder), stopped after a fixed number of iterations, equal the oracle's PCG iterate
  within max(1e-10, 3 s), s being the oracle's reformulation spread
  (tests/reformulation.py; below 1e-11 here, so the bar is 1e-10).
* Grouped launches: hierarchies added as the server's ensemble (one captured graph of
  grouped launches for an iteration of all of them) give bitwise the results of the
  same hierarchies served one by one.
* Cancellation: cancelled requests complete once, as cancelled, x untouched; the
  others are bitwise unaffected.
* Admission: the in-flight budget caps the admitted requests' work footprint at every
  moment; hierarchies beyond the resident budget and requests beyond the in-flight
  budget are refused with AMGE_ERR_BUSY.
"""
import numpy as np
import pytest

from paper_2107_05613_amd import workloads as W
from reformulation import fp64_bar, spreads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SPECS = [("curl", 8, 3, "blocks", 0), ("div", 8, 3, "blocks", 1), ("curl", 12, 3, "unit", 0)]
SLOTS = 4


class Resident:
    def __init__(self, precond_bits, resid_bits=0, smoother="l1jacobi"):
        from paper_2107_05613_amd import amge
        self.smoother = smoother
        self.prods, self.H, self.n1 = [], [], []
        for kind, n, L, coef, cs in SPECS:
            w = W.Workload("t", kind, n, L, coef, coef_seed=cs)
            a, b = W.coefficients(w)
            prod = amge.build_problem(kind, n, L, a, b)
            self.prods.append((w, a, b))
            self.H.append(amge.Hierarchy(prod, precond_bits=precond_bits, max_rhs=SLOTS, resid_bits=resid_bits,
                                         smoother=smoother))
            self.n1.append(self.H[-1].rows[0])


_RES = {}


def resident(bits, resid_bits=0, smoother="l1jacobi"):
    if (bits, resid_bits, smoother) not in _RES:
        _RES[(bits, resid_bits, smoother)] = Resident(bits, resid_bits, smoother)
    return _RES[(bits, resid_bits, smoother)]


def requests(res, num, seed=0):
    """(hierarchy index, device rhs) per request, hierarchies drawn at random."""
    rng = np.random.default_rng(seed)
    out = []
    for r in range(num):
        h = int(rng.integers(0, len(res.H)))
        out.append((h, torch.from_numpy(W.rhs(res.n1[h], 100 + r)[:, 0]).cuda()))
    torch.cuda.synchronize()
    return out


def serve(res, reqs, order, inflight_budget=0, maxit=None, watch=None, grouped=None, info=None):
    """Serves the requests of `order` (all submitted at once, in that order); returns
    {request: (status, iters, relres, x)}.  grouped[i]: None for a solo hierarchy, else
    the ensemble hierarchy i joins; info (a list) receives the server's ensemble figures."""
    from paper_2107_05613_amd import amge
    srv = amge.Server(inflight_budget=inflight_budget, chunk=2)
    ids = [srv.add(H) if not grouped or grouped[i] is None else srv.add(H, grouped=True, ensemble=grouped[i])
           for i, H in enumerate(res.H)]
    xs = {j: torch.full((res.n1[reqs[j][0]],), 3.0, dtype=torch.float64, device="cuda") for j in order}
    for j in order:
        h, b = reqs[j]
        mi = maxit[j] if maxit and j in maxit else 500
        srv.submit(ids[h], b, xs[j], tag=j, rtol=1e-8, maxit=mi)
    out = {}
    while len(out) < len(order):
        for tag, hid, status, iters, relres in srv.progress(wait=True):
            out[tag] = (status, iters, relres)
        if watch is not None:
            watch(srv)
    if info is not None:
        info.append(srv.ensemble())
    srv.close()
    torch.cuda.synchronize()
    return {j: (*out[j], xs[j].cpu().numpy()) for j in order}


def test_solo_vs_mix_bitwise():
    """a9: each result is the same alone and in the mix (continuous batching: requests
    enter free columns while the other columns of their hierarchy are in flight)."""
    res = resident(32)
    reqs = requests(res, 14, seed=1)
    mix = serve(res, reqs, list(range(len(reqs))))
    for j in range(len(reqs)):
        solo = serve(res, reqs, [j])[j]
        m = mix[j]
        assert m[0] == 0 and solo[0] == 0
        assert m[1] == solo[1] and m[2] == solo[2], (j, m[:3], solo[:3])
        assert np.array_equal(m[3], solo[3]), j
        assert m[2] <= 1e-8
    # the served result is the hierarchy's own batched solve of that column
    j = 0
    h, b = reqs[j]
    x = torch.zeros(res.n1[h] * 2, dtype=torch.float64, device="cuda")
    B = torch.stack([b, torch.zeros_like(b)], 1).reshape(-1).contiguous()
    status, its, rrs = res.H[h].pcg(B, x, rtol=1e-8, nrhs=2)
    assert its[0] == mix[j][1]
    assert np.array_equal(x.view(-1, 2)[:, 0].cpu().numpy(), mix[j][3])


class _Joined:
    def __init__(self, *rs):
        self.H = [H for r in rs for H in r.H]
        self.n1 = [n for r in rs for n in r.n1]


def test_grouped_ensemble_bitwise():
    """a9 grouped launches: the six hierarchies (H(curl) and H(div), FP32 and FP64
    V-cycles) served as one ensemble, as two ensembles, and half of them grouped beside
    solo ones, give every request bitwise the result it gets with every hierarchy served
    on its own; the ensemble's graph has fewer kernels than its members' own graphs
    together."""
    from paper_2107_05613_amd import amge
    res = _Joined(resident(32), resident(64))
    reqs = requests(res, 24, seed=3)
    order = list(range(len(reqs)))
    solo = serve(res, reqs, order)
    info = []
    allg = serve(res, reqs, order, grouped=[0] * len(res.H), info=info)
    two = serve(res, reqs, order, grouped=[i % 2 for i in range(len(res.H))])
    half = serve(res, reqs, order, grouped=[3 if i % 2 == 0 else None for i in range(len(res.H))])
    for j in order:
        for other in (allg, two, half):
            o = other[j]
            assert o[0] == solo[j][0] == 0, (j, o[:3], solo[j][:3])
            assert o[1] == solo[j][1] and o[2] == solo[j][2], (j, o[:3], solo[j][:3])
            assert np.array_equal(o[3], solo[j][3]), j
    members, launches, solo_launches = info[0]
    print(f"\n[ensemble] {members} members: {launches} kernels per iteration vs {solo_launches} alone", flush=True)
    assert members == len(res.H)
    assert 0 < launches < solo_launches
    srv = amge.Server()
    with pytest.raises(amge.AmgeError) as ei:
        srv.add(res.H[0], grouped=True, ensemble=16)
    assert ei.value.code == -1
    with pytest.raises(amge.AmgeError):
        srv.add(res.H[0], grouped=True, ensemble=-1)
    srv.close()


def test_grouped_ensemble_recapture_and_split():
    """An ensemble that grows while it serves (members join after its first chunks, so
    its graph is captured again) and has more members than one grouped launch takes (the
    launches are split): every request bitwise equal to the same request served on a
    server of solo hierarchies."""
    from paper_2107_05613_amd import amge
    hs, n1 = [], []
    for i in range(18):
        kind = "curl" if i % 2 == 0 else "div"
        w = W.Workload("t", kind, 8, 3, "blocks", coef_seed=10 + i)
        a, b = W.coefficients(w)
        hs.append(amge.Hierarchy(amge.build_problem(kind, 8, 3, a, b), precond_bits=32 if i % 3 else 64,
                                 max_rhs=2))
        n1.append(hs[-1].rows[0])
    reqs = []
    for j in range(36):
        h = j % 18 if j < 18 else (j * 7) % 18
        reqs.append((h, torch.from_numpy(W.rhs(n1[h], 500 + j)[:, 0]).cuda()))
    torch.cuda.synchronize()

    def run(srv, ids, order, xs, out):
        for j in order:
            h, b = reqs[j]
            srv.submit(ids[h], b, xs[j], tag=j, rtol=1e-8, maxit=500)
        got = 0
        while got < len(order):
            for tag, hid, status, iters, relres in srv.progress(wait=True):
                out[tag] = (status, iters, relres)
                got += 1

    def fresh():
        return {j: torch.full((n1[reqs[j][0]],), 3.0, dtype=torch.float64, device="cuda") for j in range(36)}

    solo_x, solo = fresh(), {}
    srv = amge.Server(chunk=2)
    ids = [srv.add(H) for H in hs]
    run(srv, ids, range(36), solo_x, solo)
    srv.close()

    grp_x, grp = fresh(), {}
    srv = amge.Server(chunk=2)
    ids = [srv.add(H, grouped=True) for H in hs[:10]]
    first = [j for j in range(36) if reqs[j][0] < 10]
    run(srv, ids, first, grp_x, grp)
    m0 = srv.ensemble()
    ids += [srv.add(H, grouped=True) for H in hs[10:]]
    run(srv, ids, [j for j in range(36) if j not in grp], grp_x, grp)
    m1 = srv.ensemble()
    srv.close()
    torch.cuda.synchronize()
    print(f"\n[ensemble] 10 members: {m0[1]} kernels vs {m0[2]}; 18 members: {m1[1]} vs {m1[2]}", flush=True)
    assert m0[0] == 10 and m1[0] == 18 and m1[2] > m0[2] and 0 < m1[1] < m1[2]
    for j in range(36):
        assert grp[j] == solo[j] and grp[j][0] == 0, (j, grp[j], solo[j])
        assert torch.equal(grp_x[j], solo_x[j]), j


def test_served_fp64_matches_oracle():
    """Served requests on FP64-preconditioner hierarchies, fixed iteration count, against
    the oracle's PCG iterate."""
    from oracle.hierarchy import build_hierarchy
    from oracle.solve import Multilevel, pcg
    res = resident(64)
    reqs = requests(res, 6, seed=2)
    k = 9
    out = serve(res, reqs, list(range(len(reqs))), maxit={j: k for j in range(len(reqs))})
    oracles = {}
    for j, (h, b) in enumerate(reqs):
        w, a, be = res.prods[h]
        if h not in oracles:
            H = build_hierarchy(w.kind, w.n, w.levels, a, be, check_targets=False)
            oracles[h] = (H, Multilevel.from_hierarchy(H))
        H, ml = oracles[h]
        tol = fp64_bar(spreads(H, b.cpu().numpy(), k)["pcg"])
        status, iters, relres, x = out[j]
        assert status == 1 and iters == k    # rtol 1e-8 not reached in k steps
        xo, _, _ = pcg(H.A[0], b.cpu().numpy(), ml, fixed_iters=k)
        err = np.linalg.norm(x - xo) / np.linalg.norm(xo)
        print(f"request {j} (hierarchy {h}): {k} iterations, error vs oracle {err:.1e} (tol {tol:.1e})")
        assert err <= tol


@pytest.mark.parametrize("resid_bits", [32, 64])
def test_served_fp32_matches_oracle(resid_bits):
    """Served requests on FP32-preconditioner hierarchies (fine-level residual in FP32, or
    in FP64 as the precision trial picks for high-contrast hierarchies), run to rtol 1e-8:
    within 3 iterations of the oracle's FP64 count and within 1e-6 of its solution
    (printed)."""
    from oracle.hierarchy import build_hierarchy
    from oracle.solve import Multilevel, pcg
    res = resident(32, resid_bits)
    assert all(H.resid_bits() == resid_bits for H in res.H)
    reqs = requests(res, 6, seed=4)
    out = serve(res, reqs, list(range(len(reqs))))
    oracles = {}
    for j, (h, b) in enumerate(reqs):
        w, a, be = res.prods[h]
        if h not in oracles:
            H = build_hierarchy(w.kind, w.n, w.levels, a, be, check_targets=False)
            oracles[h] = (H, Multilevel.from_hierarchy(H))
        H, ml = oracles[h]
        status, iters, relres, x = out[j]
        xo, ito, _ = pcg(H.A[0], b.cpu().numpy(), ml, rtol=1e-8)
        err = np.linalg.norm(x - xo) / np.linalg.norm(xo)
        print(f"request {j} (hierarchy {h}): {iters} iterations (oracle {ito}), error vs oracle {err:.1e}")
        assert status == 0 and relres <= 1e-8 and iters <= ito + 3
        assert err <= 1e-6


class _OracleResident:
    """The SPECS hierarchies set up from the oracle's own level matrices (the block
    smoother's colours depend on which couplings are nonzero, so both sides take the
    same matrices), with the oracle's block Gauss-Seidel V-cycle beside them."""

    def __init__(self, precond_bits, smoother):
        from oracle.hierarchy import build_hierarchy
        from oracle.solve import Multilevel
        from paper_2107_05613_amd import amge
        self.H, self.n1, self.oracle = [], [], []
        for kind, n, L, coef, cs in SPECS:
            a, b = W.coefficients(W.Workload("t", kind, n, L, coef, coef_seed=cs))
            Ho = build_hierarchy(kind, n, L, a, b, check_targets=False)
            levels = [(Ho.A[k], Ho.D[k], Ho.P[k] if k < L - 1 else None) for k in range(L)]
            self.H.append(amge.Hierarchy(levels, precond_bits=precond_bits, max_rhs=SLOTS, smoother=smoother))
            self.n1.append(self.H[-1].rows[0])
            self.oracle.append((Ho, Multilevel.from_hierarchy(Ho, smoother=smoother, gs_block=64)))


def test_served_block_gs():
    """Served requests on hierarchies with the l1-scaled symmetric block Gauss-Seidel
    smoother (set up from the oracle's level matrices): FP64 preconditioner at a fixed
    iteration count against the oracle's block Gauss-Seidel PCG iterate (max(1e-10, 3 s));
    FP32 preconditioner to rtol 1e-8 within 3 iterations of the oracle's count and 1e-6
    of its solution; and the same requests with the hierarchies as one ensemble (grouped
    launches of the batched block sweeps) bitwise as served one by one."""
    from oracle.solve import pcg
    r64, r32 = _OracleResident(64, "l1blockgs"), _OracleResident(32, "l1blockgs")
    reqs = requests(r64, 6, seed=5)
    k = 7
    out64 = serve(r64, reqs, list(range(len(reqs))), maxit={j: k for j in range(len(reqs))})
    out32 = serve(r32, reqs, list(range(len(reqs))))
    grouped = serve(r32, reqs, list(range(len(reqs))), grouped=[0] * len(r32.H))
    for j, (h, b) in enumerate(reqs):
        H, ml = r64.oracle[h]
        bb = b.cpu().numpy()
        tol = fp64_bar(spreads(H, bb, k, smoother="l1blockgs")["pcg"])
        xk, _, _ = pcg(H.A[0], bb, ml, fixed_iters=k)
        xo, ito, _ = pcg(H.A[0], bb, ml, rtol=1e-8)
        s64, it64, _, x64 = out64[j]
        s32, it32, rr32, x32 = out32[j]
        e64 = np.linalg.norm(x64 - xk) / np.linalg.norm(xk)
        e32 = np.linalg.norm(x32 - xo) / np.linalg.norm(xo)
        print(f"request {j} (hierarchy {h}): FP64 {k} iterations, error {e64:.1e} (tol {tol:.1e}); FP32 {it32} "
              f"iterations (oracle {ito}), error {e32:.1e}")
        assert s64 == 1 and it64 == k and e64 <= tol
        assert s32 == 0 and rr32 <= 1e-8 and it32 <= ito + 3 and e32 <= 1e-6
        g = grouped[j]
        assert g[:3] == out32[j][:3] and np.array_equal(g[3], x32), j
    for r in (r64, r32):
        for H in r.H:
            H.close()


def test_admission_by_inflight_budget():
    """At most two requests' work footprint admitted at any moment; the results are still
    those of the unconstrained mix."""
    from paper_2107_05613_amd import amge
    res = resident(32)
    reqs = requests(res, 8, seed=3)
    srv = amge.Server()
    ids = [srv.add(H) for H in res.H]
    per = [srv.request_bytes(i) for i in ids]
    srv.close()
    budget = 2 * max(per)
    seen = []

    def watch(s):
        st = s.stats()
        seen.append(st["inflight_bytes"])
        assert st["inflight_bytes"] <= budget

    lim = serve(res, reqs, list(range(len(reqs))), inflight_budget=budget, watch=watch)
    free = serve(res, reqs, list(range(len(reqs))))
    for j in range(len(reqs)):
        assert lim[j][1] == free[j][1] and np.array_equal(lim[j][3], free[j][3])
    assert max(seen) <= budget


def test_budget_refusals_and_failed_requests():
    """AMGE_ERR_BUSY for a hierarchy beyond the resident budget and for a request beyond
    the in-flight budget; a NaN right-hand side and a maxit cut finish with their own
    status while the other requests of the batch are unaffected."""
    from paper_2107_05613_amd import amge
    res = resident(32)
    fp = [H.footprint() for H in res.H]
    srv = amge.Server(hierarchy_budget=fp[0] + fp[1])
    srv.add(res.H[0])
    srv.add(res.H[1])
    with pytest.raises(amge.AmgeError) as e:
        srv.add(res.H[2])
    assert e.value.code == -8
    srv.close()
    srv = amge.Server(inflight_budget=1024)
    hid = srv.add(res.H[0])
    b = torch.ones(res.n1[0], dtype=torch.float64, device="cuda")
    with pytest.raises(amge.AmgeError) as e:
        srv.submit(hid, b, torch.zeros_like(b), tag=0)
    assert e.value.code == -8
    srv.close()
    # failures stay in their own column
    reqs = [(0, torch.from_numpy(W.rhs(res.n1[0], 500 + i)[:, 0]).cuda()) for i in range(5)]
    bad = reqs[1][1].clone()
    bad[7] = float("nan")
    reqs_bad = list(reqs)
    reqs_bad[1] = (0, bad)
    got = serve(res, reqs_bad, list(range(5)), maxit={3: 2})
    ref = serve(res, reqs, [0, 2, 4])
    assert got[1][0] == -7
    assert got[3][0] == 1 and got[3][1] == 2
    for j in (0, 2, 4):
        assert got[j][0] == 0 and np.array_equal(got[j][3], ref[j][3])


@pytest.mark.parametrize("grouped", [False, True])
def test_cancellation(grouped):
    """amge_server_cancel: a queued request and one whose chunk is running each complete
    once with status CANCELLED and their x untouched; every other request gives bitwise
    the result it gives when nothing is cancelled; an unknown tag cancels nothing; the
    server holds no request or in-flight bytes afterwards."""
    from paper_2107_05613_amd import amge
    res = resident(32)
    reqs = requests(res, 12, seed=3)
    order = list(range(12))
    grp = [0, 0, 0] if grouped else None
    ref = serve(res, reqs, order, grouped=grp)
    srv = amge.Server(chunk=2)
    ids = [srv.add(H) if not grouped else srv.add(H, grouped=True, ensemble=0) for H in res.H]
    xs = {j: torch.full((res.n1[reqs[j][0]],), float("nan"), dtype=torch.float64, device="cuda") for j in order}
    for j in order:
        srv.submit(ids[reqs[j][0]], reqs[j][1], xs[j], tag=j, rtol=1e-8, maxit=500)
    assert srv.cancel(5) == 1          # still queued
    assert srv.cancel(999) == 0
    out = {}

    def take(done):
        for tag, hid, status, iters, relres in done:
            assert tag not in out, f"request {tag} completed twice"
            out[tag] = (status, iters, relres)

    take(srv.progress(wait=False))     # admits the first requests and starts their chunks
    assert srv.cancel(0) == 1          # admitted first, its chunk in flight
    while len(out) < len(order):
        take(srv.progress(wait=True))
    st = srv.stats()
    srv.close()
    torch.cuda.synchronize()
    assert st["queued"] == 0 and st["inflight"] == 0 and st["inflight_bytes"] == 0
    for j in order:
        x = xs[j].cpu().numpy()
        if j in (0, 5):
            assert out[j][0] == amge.CANCELLED, (j, out[j])
            assert np.isnan(x).all(), j
            continue
        assert out[j] == ref[j][:3], (j, out[j], ref[j][:3])
        assert np.array_equal(x, ref[j][3]), j
    print(f"grouped={grouped}: 2 of 12 requests cancelled, the other 10 bitwise as uncancelled")
