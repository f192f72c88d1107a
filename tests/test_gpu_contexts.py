"""Contexts and the caller's allocator (amge_ctx_create, amge_opts.alloc, amge_footprint),
through the C ABI.

Algorithm 4.1 takes the hierarchy ({A_k}, {P}, the smoothers' inputs, the coarsest
solver) as read-only input; a context holds what one caller mutates.  Bars:
* two contexts of one hierarchy used at the same time (V-cycles queued on two streams;
  PCG solves from two host threads) give bitwise the results of the same calls made one
  after the other on one context;
* with torch's caching allocator as the library's allocator, the bytes the library
  requests from torch for a hierarchy and for a context are exactly the footprint it
  reports (set-up staging included in nothing that stays), and they are returned when
  the hierarchy and context are destroyed;
* the library's own hipMalloc path (allocator=None) gives bitwise the same results.
"""
import threading

import numpy as np
import pytest

from paper_2107_05613_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


@pytest.fixture(scope="module")
def problem():
    from paper_2107_05613_amd import amge
    w = W.Workload("t", "div", 12, 3, "blocks")
    a, b = W.coefficients(w)
    print("\n[contexts] div n=12 3 levels, jump coefficients", flush=True)
    return amge.build_problem(w.kind, w.n, w.levels, a, b)


@pytest.mark.parametrize("bits", [32, 64])
def test_concurrent_vcycles_on_two_streams(problem, bits):
    from paper_2107_05613_amd import amge
    H = amge.Hierarchy(problem, precond_bits=bits, max_rhs=4)
    n = H.rows[0]
    r1, r2 = dev(W.rhs(n, 1)[:, 0]), dev(W.rhs(n, 2)[:, 0])
    B = dev(W.rhs(n, 3, 4))
    # serial references on one context
    c0 = H.context(4)
    ref1, ref2, refB = torch.empty_like(r1), torch.empty_like(r2), torch.empty_like(B)
    c0.vcycle(r1, ref1)
    c0.vcycle(r2, ref2)
    c0.vcycle(B, refB, nrhs=4)
    torch.cuda.synchronize()
    # two contexts, queued on two streams, each several times
    c1, c2 = H.context(1), H.context(4)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    z1, z2, zB = torch.empty_like(r1), torch.empty_like(r2), torch.empty_like(B)
    torch.cuda.synchronize()
    for _ in range(5):
        with torch.cuda.stream(s1):
            c1.vcycle(r1, z1, stream=s1)
        with torch.cuda.stream(s2):
            c2.vcycle(B, zB, nrhs=4, stream=s2)
            c2.vcycle(r2, z2, stream=s2)
    torch.cuda.synchronize()
    assert torch.equal(z1, ref1) and torch.equal(z2, ref2) and torch.equal(zB, refB)
    for c in (c0, c1, c2):
        c.close()
    H.close()


def test_concurrent_pcg_from_two_threads(problem):
    from paper_2107_05613_amd import amge
    H = amge.Hierarchy(problem, precond_bits=32, max_rhs=4)
    n = H.rows[0]
    rhs = [dev(W.rhs(n, 10 + i)[:, 0]) for i in range(2)]
    B = dev(W.rhs(n, 20, 3))
    c0 = H.context(4)
    refs = []
    for b in rhs:
        x = torch.zeros_like(b)
        refs.append((c0.pcg(b, x, rtol=1e-8), x))
    X = torch.zeros_like(B)
    refB = (c0.pcg(B, X, rtol=1e-8, nrhs=3), X)
    torch.cuda.synchronize()
    ctxs = [H.context(1), H.context(4)]
    out = {}

    def worker(i):
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            for rep in range(3):
                if i == 0:
                    x = torch.zeros_like(rhs[0])
                    out[(i, rep)] = (ctxs[0].pcg(rhs[0], x, rtol=1e-8, stream=s), x)
                else:
                    X = torch.zeros_like(B)
                    out[(i, rep)] = (ctxs[1].pcg(B, X, rtol=1e-8, nrhs=3, stream=s), X)
            s.synchronize()

    th = [threading.Thread(target=worker, args=(i,)) for i in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    torch.cuda.synchronize()
    for rep in range(3):
        (st, it, rr), x = out[(0, rep)]
        assert st == 0 and it == refs[0][0][1] and rr == refs[0][0][2] and torch.equal(x, refs[0][1])
        (st, it, rr), X = out[(1, rep)]
        assert st == 0 and it == refB[0][1] and rr == refB[0][2] and torch.equal(X, refB[1])
    print(f"[contexts] threads: {refs[0][0][1]} / {refB[0][1]} iterations, bitwise equal to serial", flush=True)
    for c in ctxs + [c0]:
        c.close()
    H.close()


def test_torch_allocator_and_footprint(problem):
    from paper_2107_05613_amd import amge
    def requested():
        # bytes requested from torch's allocator and not yet returned (its block sizes,
        # memory_allocated, add its rounding, which depends on what it holds cached)
        return torch.cuda.memory_stats()["requested_bytes.all.current"]

    torch.cuda.synchronize()
    m0 = requested()
    H = amge.Hierarchy(problem, precond_bits=32, max_rhs=8)
    torch.cuda.synchronize()
    m1 = requested()
    hb, cb8 = H.footprint_parts(8)
    _, cb1 = H.footprint_parts(1)
    c = H.context(8)
    m2 = requested()
    print(f"[contexts] hierarchy {hb} B (requested from torch {m1 - m0}), context of 8 {cb8} B "
          f"(requested {m2 - m1}), context of 1 {cb1} B", flush=True)
    # set-up staging (layouts, products) is returned before the call ends: what stays
    # is exactly the footprint
    assert m1 - m0 == hb
    assert m2 - m1 == cb8
    assert 0 < cb1 < cb8
    n = H.rows[0]
    b = dev(W.rhs(n, 4)[:, 0])
    x = torch.zeros_like(b)
    st, it, rr = c.pcg(b, x, rtol=1e-8)
    # the same solve on a hipMalloc hierarchy: bitwise equal
    G = amge.Hierarchy(problem, precond_bits=32, max_rhs=8, allocator=None)
    assert G.footprint_parts(8) == (hb, cb8)
    y = torch.zeros_like(b)
    st2, it2, rr2 = G.pcg(b, y, rtol=1e-8)
    assert (st, it, rr) == (st2, it2, rr2) and torch.equal(x, y)
    G.close()
    c.close()
    H.close()
    del b, x, y
    torch.cuda.synchronize()
    assert requested() == m0


def test_context_arguments(problem):
    from paper_2107_05613_amd import amge
    H = amge.Hierarchy(problem, precond_bits=64, max_rhs=2)
    with pytest.raises(amge.AmgeError) as e:
        H.context(3)
    assert e.value.code == -1
    with pytest.raises(amge.AmgeError) as e:
        H.context(0)
    assert e.value.code == -1
    c = H.context(1)
    n = H.rows[0]
    B = torch.zeros(2 * n, dtype=torch.float64, device="cuda")
    with pytest.raises(amge.AmgeError) as e:
        c.vcycle(B, B.clone(), nrhs=2)     # more columns than the context holds
    assert e.value.code == -1
    with pytest.raises(amge.AmgeError):
        H.footprint_parts(3)
    c.close()
    H.close()
