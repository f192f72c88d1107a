"""Oracle, fine level: Kuhn mesh, signed incidences, Whitney masses, fine operators.

Test infrastructure only (see the package docstring).

Paper anchors
-------------
* Section 2.1, eq. (2.2): a_D(u, v) = (alpha D u, D v) + (beta u, v) for D = curl, div.
* Section 2.2: lowest-order spaces H1 -> ND -> RT -> L2 with one dof per vertex,
  edge, face, cell; the discrete derivatives D_1^h, D_2^h, D_3^h map vertices to
  edges, edges to faces and faces to cells (signed incidences).

The fine system matrices are assembled exactly from Whitney forms:
curl maps the Whitney edge space onto the Whitney face space with the incidence
C as matrix, and div maps the face space onto piecewise constants with Dv, so

    A_curl = C^T M_RT(alpha) C + M_ND(beta),
    A_div  = Dv^T M_L2(alpha) Dv + M_RT(beta).

Geometry is computed in integer lattice units and scaled by powers of h, so that
translated elements have bitwise identical element matrices.
"""
from __future__ import annotations

import itertools
import numpy as np
import scipy.sparse as sp

# Local edge (i, j) and face (omitting vertex i) numbering inside a tetrahedron.
TET_EDGES = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
TET_FACES = [(1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2)]   # face i omits vertex i
TRI_EDGES = [(0, 1), (0, 2), (1, 2)]


def _keys(tuples, nv):
    """Encode sorted integer tuples as int64 keys (lexicographic order preserved)."""
    tuples = np.asarray(tuples, dtype=np.int64)
    key = np.zeros(tuples.shape[0], dtype=np.int64)
    for c in range(tuples.shape[1]):
        key = key * nv + tuples[:, c]
    return key


class FineMesh:
    """Kuhn triangulation of the unit cube with n^3 hexes, 6 tetrahedra each.

    Vertex (i, j, k) has index i + (n+1)(j + (n+1)k).  Edges, faces and tets are
    sorted tuples of vertex indices; each entity list is sorted lexicographically.
    Orientation of edges and faces is by increasing vertex index: an edge runs
    from its smaller to its larger vertex, a face (a, b, c) has normal
    (x_b - x_a) x (x_c - x_a).
    """

    def __init__(self, n: int):
        self.n = n
        self.h = 1.0 / n
        m = n + 1
        nv = m ** 3
        if nv ** 3 >= 2 ** 62:
            raise ValueError("mesh too large for the key encoding")
        self.nv = nv
        v = np.arange(nv)
        self.X = np.stack([v % m, (v // m) % m, v // (m * m)], axis=1).astype(np.int64)

        # Six Kuhn tets per hex: the monotone lattice paths from corner (0,0,0)
        # to corner (1,1,1), one per permutation of the axes.
        hx = np.arange(n ** 3)
        i, j, k = hx % n, (hx // n) % n, hx // (n * n)
        base = i + m * (j + m * k)
        step = [1, m, m * m]
        tets, thex = [], []
        for perm in itertools.permutations(range(3)):
            off = np.cumsum([0] + [step[a] for a in perm])
            tets.append(base[:, None] + off[None, :])
            thex.append(hx)
        tets = np.concatenate(tets)
        thex = np.concatenate(thex)
        order = np.lexsort(tets.T[::-1])
        self.tets = tets[order]
        self.tet_hex = thex[order]

        # unique sorted entities: the int64 key order is the lexicographic tuple order
        ekeys = np.unique(np.concatenate([_keys(self.tets[:, list(e)], nv) for e in TET_EDGES]))
        self.edges = np.stack([ekeys // nv, ekeys % nv], axis=1)
        fkeys = np.unique(np.concatenate([_keys(self.tets[:, list(f)], nv) for f in TET_FACES]))
        self.faces = np.stack([fkeys // (nv * nv), (fkeys // nv) % nv, fkeys % nv], axis=1)
        self.ekey = ekeys
        self.fkey = fkeys
        self._signs = None

        # element -> global entity maps
        self.tet_edges = np.stack([np.searchsorted(self.ekey, _keys(self.tets[:, list(e)], nv))
                                   for e in TET_EDGES], axis=1)
        self.tet_faces = np.stack([np.searchsorted(self.fkey, _keys(self.tets[:, list(f)], nv))
                                   for f in TET_FACES], axis=1)
        self.face_edges = np.stack([np.searchsorted(self.ekey, _keys(self.faces[:, list(e)], nv))
                                    for e in TRI_EDGES], axis=1)

    # ------------------------------------------------------------------ counts
    @property
    def counts(self):
        return dict(V=self.nv, E=len(self.edges), F=len(self.faces), T=len(self.tets))

    # ------------------------------------------------------------ incidences
    def grad(self):
        """G (E x V): G[e, a] = -1, G[e, b] = +1 for e = (a < b)."""
        ne = len(self.edges)
        r = np.repeat(np.arange(ne), 2)
        c = self.edges.reshape(-1)
        val = np.tile([-1.0, 1.0], ne)
        return sp.csr_matrix((val, (r, c)), shape=(ne, self.nv))

    def curl(self):
        """C (F x E): boundary of face (a, b, c) is (b, c) - (a, c) + (a, b)."""
        nf = len(self.faces)
        fe = self.face_edges  # columns: (a,b), (a,c), (b,c)
        r = np.repeat(np.arange(nf), 3)
        c = fe.reshape(-1)
        val = np.tile([1.0, -1.0, 1.0], nf)
        return sp.csr_matrix((val, (r, c)), shape=(nf, len(self.edges)))

    def tet_face_signs(self):
        """+1 where the face's orientation normal points out of the tet, else -1."""
        if self._signs is not None:
            return self._signs
        X = self.X
        sgn = np.empty((len(self.tets), 4))
        for i, f in enumerate(TET_FACES):
            a, b, c = (X[self.tets[:, f[0]]], X[self.tets[:, f[1]]], X[self.tets[:, f[2]]])
            nrm = np.cross(b - a, c - a)
            # face centroid minus opposite vertex points outward (times 3 to stay integral)
            outward = (a + b + c) - 3 * X[self.tets[:, i]]
            s = np.einsum("ij,ij->i", nrm, outward)
            assert np.all(s != 0)
            sgn[:, i] = np.sign(s)
        self._signs = sgn
        return sgn

    def div(self):
        """Dv (T x F): +1/-1 for outward/inward face orientation, so Dv u = integral of div."""
        nt = len(self.tets)
        r = np.repeat(np.arange(nt), 4)
        c = self.tet_faces.reshape(-1)
        return sp.csr_matrix((self.tet_face_signs().reshape(-1), (r, c)),
                             shape=(nt, len(self.faces)))

    # ------------------------------------------------------------- geometry
    def tet_geometry(self):
        """Lattice-unit edge matrix J (T,3,3), 6*volume in lattice units, bary gradients."""
        X = self.X[self.tets]                      # (T, 4, 3) int
        J = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
        vol6 = np.abs(np.round(np.linalg.det(J.astype(np.float64))))
        Jinv = np.linalg.inv(J.astype(np.float64))           # rows: grad lambda_1..3
        grads = np.concatenate([-Jinv.sum(axis=1, keepdims=True), Jinv], axis=1)  # (T,4,3)
        return X, vol6, grads

    def volumes(self):
        _, vol6, _ = self.tet_geometry()
        return vol6 * self.h ** 3 / 6.0

    # -------------------------------------------------------- element masses
    def nd_element_mass(self):
        """Whitney edge mass per tet, (T, 6, 6), unit coefficient.

        w_ij = l_i grad l_j - l_j grad l_i,  int l_a l_b = |tau| (1 + delta_ab) / 20.
        """
        _, vol6, g = self.tet_geometry()
        h = self.h
        vol = vol6 * h ** 3 / 6.0
        I = (np.ones((4, 4)) + np.eye(4)) / 20.0
        gg = np.einsum("tad,tbd->tab", g, g) / h ** 2   # grad l_a . grad l_b, true units
        M = np.empty((len(self.tets), 6, 6))
        for p, (i, j) in enumerate(TET_EDGES):
            for q, (k, l) in enumerate(TET_EDGES):
                M[:, p, q] = vol * (I[i, k] * gg[:, j, l] - I[i, l] * gg[:, j, k]
                                    - I[j, k] * gg[:, i, l] + I[j, l] * gg[:, i, k])
        return M

    def rt_element_mass(self):
        """Whitney face mass per tet, (T, 4, 4), unit coefficient.

        The face function with unit flux through face i (opposite vertex x_i) is
        s_i (x - x_i) / (3|tau|), s_i = +-1 the sign of the face orientation.
        """
        X, vol6, _ = self.tet_geometry()
        h = self.h
        vol = vol6 * h ** 3 / 6.0
        s = self.tet_face_signs()
        # int (x - x_i).(x - x_j) = |tau| sum_ab I_ab (x_a - x_i).(x_b - x_j), I_ab = (1 + d_ab)/20.
        # With the Gram matrix Gr_ab = y_a.y_b of y_a = x_a - x_0 (integers) and
        # sum_b I_ab = 1/4, sum_ab I_ab = 1 this is
        #   sum_ab I_ab Gr_ab - (colsum_j + rowsum_i) / 4 + Gr_ij.
        Y = (X - X[:, :1, :]).astype(np.float64)
        Gr = np.einsum("tad,tbd->tab", Y, Y)
        I = (np.ones((4, 4)) + np.eye(4)) / 20.0
        c0 = np.einsum("ab,tab->t", I, Gr)
        rs = Gr.sum(axis=2)                                  # sum_b Gr_ib
        acc = (c0[:, None, None] - 0.25 * (rs[:, None, :] + rs[:, :, None]) + Gr) * h * h
        return s[:, :, None] * s[:, None, :] * acc * (vol / (9.0 * vol ** 2))[:, None, None]

    def nd_face_trace_mass(self):
        """Tangential-trace (2D Whitney edge) mass per face, (F, 3, 3), local edges TRI_EDGES."""
        X = self.X[self.faces].astype(np.float64)    # (F, 3, 3)
        J = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0]], axis=2)   # (F, 3, 2)
        Gm = np.einsum("fdi,fdj->fij", J, J)
        area2 = np.sqrt(np.linalg.det(Gm))            # twice the area, lattice units
        G12 = np.einsum("fdi,fij->fdj", J, np.linalg.inv(Gm))   # grads of l_1, l_2 (as columns)
        g = np.stack([-G12[:, :, 0] - G12[:, :, 1], G12[:, :, 0], G12[:, :, 1]], axis=1)  # (F,3,3)
        area = area2 / 2.0 * self.h ** 2
        gg = np.einsum("fad,fbd->fab", g, g) / self.h ** 2
        I = (np.ones((3, 3)) + np.eye(3)) / 12.0
        M = np.empty((len(self.faces), 3, 3))
        for p, (i, j) in enumerate(TRI_EDGES):
            for q, (k, l) in enumerate(TRI_EDGES):
                M[:, p, q] = area * (I[i, k] * gg[:, j, l] - I[i, l] * gg[:, j, k]
                                     - I[j, k] * gg[:, i, l] + I[j, l] * gg[:, i, k])
        return M

    # -------------------------------------------------- measures / orientation
    def edge_vectors(self):
        """Oriented edge vectors x_b - x_a in lattice units."""
        return self.X[self.edges[:, 1]] - self.X[self.edges[:, 0]]

    def face_normals(self):
        """Oriented (x_b - x_a) x (x_c - x_a) in lattice units (twice the area vector)."""
        a, b, c = (self.X[self.faces[:, 0]], self.X[self.faces[:, 1]], self.X[self.faces[:, 2]])
        return np.cross(b - a, c - a)


def assemble(idx, mats, coef, ndof):
    """Global matrix sum_c coef[c] * L_c^T mats[c] L_c from local index lists idx (nc, nl)."""
    nc, nl = idx.shape
    r = np.repeat(idx, nl, axis=1).reshape(-1)
    c = np.tile(idx, (1, nl)).reshape(-1)
    v = (mats * coef[:, None, None]).reshape(-1)
    return sp.coo_matrix((v, (r, c)), shape=(ndof, ndof)).tocsr()


def fine_problem(mesh: FineMesh, kind: str, alpha_hex, beta_hex):
    """Fine system matrix (eq. (2.2)) and the incidences, in canonical dof order."""
    alpha = np.asarray(alpha_hex, dtype=np.float64)[mesh.tet_hex]
    beta = np.asarray(beta_hex, dtype=np.float64)[mesh.tet_hex]
    G, C, Dv = mesh.grad(), mesh.curl(), mesh.div()
    nE, nF = len(mesh.edges), len(mesh.faces)
    if kind == "curl":
        Mrt_a = assemble(mesh.tet_faces, mesh.rt_element_mass(), alpha, nF)
        Mnd_b = assemble(mesh.tet_edges, mesh.nd_element_mass(), beta, nE)
        A = (C.T @ Mrt_a @ C + Mnd_b).tocsr()
    elif kind == "div":
        vol = mesh.volumes()
        ML2 = sp.diags(alpha / vol)
        Mrt_b = assemble(mesh.tet_faces, mesh.rt_element_mass(), beta, nF)
        A = (Dv.T @ ML2 @ Dv + Mrt_b).tocsr()
    else:
        raise ValueError(kind)
    A.sum_duplicates()
    A.sort_indices()
    return A, G, C, Dv
