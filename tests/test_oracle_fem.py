"""Pins of the oracle's fine level (paper section 2) against closed forms.

Nothing here re-types an oracle formula: each check uses an independent
characterisation (Stokes / divergence theorem on polynomial fields, the
classical 7-point stencil of the Kuhn triangulation, quadrature of Whitney's
own barycentric formulas, topological invariants).
"""
import itertools

import numpy as np
import pytest

from oracle.fem import FineMesh, assemble, fine_problem, TET_EDGES, TET_FACES, TRI_EDGES
from paper_2107_05613_amd.workloads import entity_counts


@pytest.mark.parametrize("n", [1, 2, 3, 5])
def test_counts_and_euler(n):
    m = FineMesh(n)
    c = m.counts
    assert c == entity_counts(n)
    # contractible domain: V - E + F - T = 1
    assert c["V"] - c["E"] + c["F"] - c["T"] == 1


@pytest.mark.parametrize("n", [1, 2, 4])
def test_complex_property_exact(n):
    """D_{i+1} D_i = 0 exactly (section 2.2.1)."""
    m = FineMesh(n)
    G, C, Dv = m.grad(), m.curl(), m.div()
    assert abs(C @ G).max() == 0
    assert abs(Dv @ C).max() == 0


@pytest.mark.parametrize("n", [1, 2])
def test_exactness_ranks(n):
    """Range(D_i) = Ker(D_{i+1}) (eq. (2.4)) via ranks on a contractible mesh."""
    m = FineMesh(n)
    G, C, Dv = (x.toarray() for x in (m.grad(), m.curl(), m.div()))
    V, E, F, T = (m.counts[k] for k in "VEFT")
    assert np.linalg.matrix_rank(G) == V - 1
    assert np.linalg.matrix_rank(C) == E - (V - 1)
    assert np.linalg.matrix_rank(Dv) == T       # div onto
    assert F - np.linalg.matrix_rank(Dv) == np.linalg.matrix_rank(C)


def _linear_field(rng):
    B = rng.standard_normal((3, 3))
    c = rng.standard_normal(3)
    return B, c


@pytest.mark.parametrize("n", [2, 3])
def test_stokes_commutation_on_linear_fields(n):
    """Interpolants of polynomial fields commute with G, C, Dv (Stokes / Gauss)."""
    rng = np.random.default_rng(1)
    m = FineMesh(n)
    x = m.X * m.h
    B, c = _linear_field(rng)
    # potential phi = x.S x / 2 + g.x, grad phi = S x + g (linear)
    S = rng.standard_normal((3, 3)); S = S + S.T
    g = rng.standard_normal(3)
    phi = 0.5 * np.einsum("vi,ij,vj->v", x, S, x) + x @ g
    a, b = m.edges[:, 0], m.edges[:, 1]
    mid = 0.5 * (x[a] + x[b])
    t = x[b] - x[a]
    u_grad = np.einsum("ei,ei->e", mid @ S.T + g, t)       # exact line integrals
    assert np.allclose(m.grad() @ phi, u_grad, atol=1e-13)
    # curl of F = B x + c is the constant vector w
    u_nd = np.einsum("ei,ei->e", mid @ B.T + c, t)
    w = np.array([B[2, 1] - B[1, 2], B[0, 2] - B[2, 0], B[1, 0] - B[0, 1]])
    fa, fb, fc = m.faces[:, 0], m.faces[:, 1], m.faces[:, 2]
    nrm = np.cross(x[fb] - x[fa], x[fc] - x[fa]) / 2.0       # area vector, orientation normal
    assert np.allclose(m.curl() @ u_nd, nrm @ w, atol=1e-13)
    # div: fluxes of F through faces, integral of div F = tr(B) |tau|
    cen = (x[fa] + x[fb] + x[fc]) / 3.0
    u_rt = np.einsum("fi,fi->f", cen @ B.T + c, nrm)
    assert np.allclose(m.div() @ u_rt, np.trace(B) * m.volumes(), atol=1e-13)


@pytest.mark.parametrize("n", [2, 3])
def test_constant_field_energies(n):
    """|c|^2 |Omega| for the ND and RT interpolants of a constant field."""
    m = FineMesh(n)
    one = np.ones(len(m.tets))
    Mnd = assemble(m.tet_edges, m.nd_element_mass(), one, len(m.edges))
    Mrt = assemble(m.tet_faces, m.rt_element_mass(), one, len(m.faces))
    rng = np.random.default_rng(2)
    c = rng.standard_normal(3)
    u = m.edge_vectors() @ c * m.h
    f = m.face_normals() @ c * m.h ** 2 / 2
    assert np.isclose(u @ Mnd @ u, c @ c, rtol=1e-13)
    assert np.isclose(f @ Mrt @ f, c @ c, rtol=1e-13)


def test_p1_stiffness_is_seven_point_stencil():
    """G^T M_ND G is the P1 stiffness; on the Kuhn triangulation it is the 7-point
    Laplacian times h at interior vertices (classical result)."""
    n = 4
    m = FineMesh(n)
    Mnd = assemble(m.tet_edges, m.nd_element_mass(), np.ones(len(m.tets)), len(m.edges))
    G = m.grad()
    K = (G.T @ Mnd @ G).toarray()
    M1 = n + 1
    for (i, j, k) in [(1, 1, 1), (2, 1, 3), (3, 3, 2)]:
        v = i + M1 * (j + M1 * k)
        expect = np.zeros(M1 ** 3)
        expect[v] = 6.0
        for d in (1, M1, M1 * M1):
            expect[v + d] = expect[v - d] = -1.0
        assert np.allclose(K[v] / m.h, expect, atol=1e-12)


def _bary(xs, p):
    """Barycentric coordinates of points p in the tet with vertices xs (independent solve)."""
    Amat = np.vstack([xs.T, np.ones(4)])
    return np.linalg.solve(Amat, np.vstack([p.T, np.ones(len(p))])).T


def _bary_grads(xs):
    Amat = np.vstack([xs.T, np.ones(4)])
    inv = np.linalg.inv(Amat)          # lambda(x) = inv @ [x; 1]
    return inv[:, :3]                  # rows: grad lambda_i


def test_element_masses_by_quadrature():
    """Closed-form Whitney masses equal a degree-2-exact quadrature of Whitney's
    barycentric formulas (ND: l_i grad l_j - l_j grad l_i; RT: 2 sum of
    l_a grad l_b x grad l_c over the cyclic shifts of the face (a<b<c))."""
    m = FineMesh(2)
    Mnd, Mrt = m.nd_element_mass(), m.rt_element_mass()
    a, b = 0.5854101966249685, 0.1381966011250105
    qb = np.full((4, 4), b) + np.eye(4) * (a - b)       # 4-point rule, weights |tau|/4
    for t in [0, 7, 23, 47]:
        xs = m.X[m.tets[t]].astype(float) * m.h
        vol = abs(np.linalg.det((xs[1:] - xs[0]).T)) / 6
        pts = qb @ xs
        lam = _bary(xs, pts)
        gl = _bary_grads(xs)
        nd = np.stack([lam[:, i, None] * gl[j] - lam[:, j, None] * gl[i] for i, j in TET_EDGES], 1)
        Q = np.einsum("qad,qbd->ab", nd, nd) * vol / 4
        assert np.allclose(Q, Mnd[t], rtol=1e-12, atol=1e-14)
        rt = []
        for i, f in enumerate(TET_FACES):
            aa, bb, cc = f
            w = 2 * (lam[:, aa, None] * np.cross(gl[bb], gl[cc]) + lam[:, bb, None] * np.cross(gl[cc], gl[aa])
                     + lam[:, cc, None] * np.cross(gl[aa], gl[bb]))
            rt.append(w)
        rt = np.stack(rt, 1)
        Q = np.einsum("qad,qbd->ab", rt, rt) * vol / 4
        assert np.allclose(Q, Mrt[t], rtol=1e-12, atol=1e-14)


def test_face_trace_mass_by_quadrature_and_constant_fields():
    """The tangential-trace mass of a face (the mass the ND extension minimises on
    coarse faces, section 3.3.3) against two independent facts.
    (a) An edge-midpoint quadrature (exact for degree 2) of the 2-D Whitney edge
        functions l_i grad_F l_j - l_j grad_F l_i, the surface gradients taken from the
        cross-product formula grad_F l_i = n x (x_{i+2} - x_{i+1}) / (2 |F|).
    (b) Every constant field c: with u_e = c . (x_b - x_a) on the face's edges,
        u^T M u = |F| |c - (c . n) n|^2, the L2 norm of its tangential part."""
    m = FineMesh(2)
    M = m.nd_face_trace_mass()
    rng = np.random.default_rng(0)
    mids = np.array([[0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]])
    for f in range(len(m.faces)):
        xs = m.X[m.faces[f]].astype(float) * m.h
        nv = np.cross(xs[1] - xs[0], xs[2] - xs[0])
        area = np.linalg.norm(nv) / 2
        nu = nv / np.linalg.norm(nv)
        g = np.stack([np.cross(nu, xs[(i + 2) % 3] - xs[(i + 1) % 3]) / (2 * area) for i in range(3)])
        w = np.stack([mids[:, i, None] * g[j] - mids[:, j, None] * g[i] for i, j in TRI_EDGES], 1)  # (q, e, 3)
        Q = np.einsum("qad,qbd->ab", w, w) * area / 3
        assert np.allclose(Q, M[f], rtol=1e-12, atol=1e-15), f
        for c in rng.uniform(-1, 1, (3, 3)):
            u = np.array([c @ (xs[j] - xs[i]) for i, j in TRI_EDGES])
            ct = c - (c @ nu) * nu
            assert abs(u @ M[f] @ u - area * (ct @ ct)) <= 1e-12 * area * (c @ c), f


def test_nd_basis_unit_circulation():
    """The closed-form ND mass uses basis functions whose tangential integral on
    their own edge is 1: check via Gauss-Legendre on the edges."""
    m = FineMesh(1)
    xs = m.X[m.tets[0]].astype(float) * m.h
    gl = _bary_grads(xs)
    gp = np.array([-1, 1]) / np.sqrt(3)
    for p, (i, j) in enumerate(TET_EDGES):
        for q, (k, l) in enumerate(TET_EDGES):
            pts = xs[k] + np.outer((gp + 1) / 2, xs[l] - xs[k])
            lam = _bary(xs, pts)
            w = lam[:, i, None] * gl[j] - lam[:, j, None] * gl[i]
            circ = np.mean(w @ (xs[l] - xs[k]))
            assert np.isclose(circ, 1.0 if p == q else 0.0, atol=1e-13)


def test_curlcurl_element_formula():
    """C^T M_RT C equals the element curl-curl matrix with curl w_ij = 2 grad l_i x grad l_j."""
    m = FineMesh(2)
    one = np.ones(len(m.tets))
    Mrt = assemble(m.tet_faces, m.rt_element_mass(), one, len(m.faces))
    C = m.curl()
    K1 = (C.T @ Mrt @ C).toarray()
    K2 = np.zeros_like(K1)
    for t in range(len(m.tets)):
        xs = m.X[m.tets[t]].astype(float) * m.h
        vol = abs(np.linalg.det((xs[1:] - xs[0]).T)) / 6
        gl = _bary_grads(xs)
        cu = np.stack([2 * np.cross(gl[i], gl[j]) for i, j in TET_EDGES])
        idx = m.tet_edges[t]
        K2[np.ix_(idx, idx)] += vol * cu @ cu.T
    assert np.allclose(K1, K2, rtol=1e-12, atol=1e-12)


def test_div_div_and_fine_operators_spd():
    m = FineMesh(2)
    rng = np.random.default_rng(3)
    a, b = 10 ** rng.uniform(-3, 3, 8), np.ones(8)
    for kind in ("curl", "div"):
        A, G, C, Dv = fine_problem(m, kind, a, b)
        Ad = A.toarray()
        assert np.allclose(Ad, Ad.T, rtol=0, atol=1e-12 * abs(Ad).max())
        assert np.linalg.eigvalsh(Ad).min() > 0
    # div-div part: Dv^T diag(alpha/|tau|) Dv = int alpha div w_f div w_g with div w_f = +-1/|tau|
    A, G, C, Dv = fine_problem(m, "div", a, np.zeros(8))
    vol = m.volumes()
    al = a[m.tet_hex]
    ref = np.zeros((len(m.faces), len(m.faces)))
    s = m.tet_face_signs()
    for t in range(len(m.tets)):
        d = s[t] / vol[t]
        ref[np.ix_(m.tet_faces[t], m.tet_faces[t])] += al[t] * vol[t] * np.outer(d, d)
    assert np.allclose(A.toarray(), ref, rtol=1e-12, atol=1e-10)


def test_translated_elements_bitwise_equal():
    """Element matrices depend only on integer lattice differences (needed for the
    identical-local-problem shortcut of the coarsening)."""
    m = FineMesh(6)
    Mnd = m.nd_element_mass()
    # the 6 Kuhn tets of hex 0 and of hex (3, 2, 5), in the same local order
    def hex_tets(i, j, k):
        h = i + 6 * (j + 6 * k)
        return np.nonzero(m.tet_hex == h)[0]
    t0, t1 = hex_tets(0, 0, 0), hex_tets(3, 2, 5)
    assert np.array_equal(Mnd[t0], Mnd[t1])
