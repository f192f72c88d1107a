"""Oracle, coarse levels: structured agglomeration and the AMGe de Rham hierarchy.

Test infrastructure only (see the package docstring).

Paper anchors
-------------
* Section 3.1: agglomerates, coarse facets / edges / vertices by intersection,
  orientation vectors of +-1 relating coarse entities to their constituents.
  Here the agglomerates are the 2x2x2 blocks that undo one uniform refinement,
  so level k >= 2 is a cube complex; a finer entity belongs to the coarse entity
  that contains it in its relative interior.
* Section 3.2.1: prolongators P_i (columns = coarse basis functions), Galerkin
  coarse matrices A^H = P^T A P.
* Section 3.2.2, eq. (3.4): co-chain projectors with Pi P = I; for PV-only coarse
  spaces the L2 projection of a trace onto the PV trace is the oriented sum of
  the constituent dofs (the coarse de Rham map).  D^H = Pi D P.
* Section 3.3.1 and 3.3.2, eq. (3.5): PV traces with unit integral; targets are the
  interpolants of polynomials of the fine order (order 0 here: constants),
  orthogonalised against the PV traces with SVD and local masses.
* Section 3.3.3, eqs. (3.6) and (3.8): extension of traces from lower- to
  higher-dimensional coarse entities.  Both systems are the optimality conditions
  of a minimum-L2-norm extension under a derivative constraint,
      min 1/2 u^T M_Z u  subject to  D_Z u = s,  u fixed on the boundary of Z,
  where s is the coarse derivative of the trace expressed with the already
  built next space (the commuting relation D P_i = P_{i+1} D^H restricted to Z).
  At consistent data the stabilisation term of (3.8) vanishes.
* Sections 3.3.3 (bubbles, eqs. (3.7), (3.9)) and 3.3.4: cross-space bubbles
  arise only from targets orthogonal to the PV traces; for order-0 targets none
  survive the filtering, which is asserted.
* Remark closing section 3.3 (coefficients in the local problems): by default the
  extensions minimise the unweighted L2 norm; with extension="coefficient" the element
  masses of the system space are weighted by beta and those of the next space (the
  range of its derivative) by alpha, so each local problem minimises the part of the
  energy (2.2) its space carries.  Coarse element masses follow by RAP, so the weights
  reach every level.  Face trace masses stay unweighted (a face between cells of
  different beta has no single weight; beta = 1 in every workload here).
* Essential boundary conditions (the benchmark of section 5.1; boundary attributes
  tracked on every level, section 3): bc="essential" keeps on every level only the
  entities not lying in the boundary of the cube.  A coarse basis function of an
  interior entity vanishes on the boundary (its extensions reach only entities whose
  closure contains it), so the restricted P maps interior to interior dofs and the
  restricted operators are still Galerkin products.

Local problems are solved by the SVD null-space method: particular solution
from the pseudo-inverse of the constraint block, minimisation over the right
null space.  Entities are processed in batches; a local problem whose inputs
are bitwise equal to another one's in the batch (translates on the structured
mesh) is solved once, which changes no result.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .fem import FineMesh, fine_problem

SPACE_NAMES = ("H1", "ND", "RT", "L2")
SVD_NULL_TOL = 1e-12     # relative singular value below which a direction is null
TARGET_TOL = 1e-10       # relative singular value above which a target survives


# ----------------------------------------------------------------------------
# levels
# ----------------------------------------------------------------------------
class Level:
    """One level of the de Rham hierarchy as a (generalised) cell complex.

    ent[d]      vertex tuples of the d-dimensional entities (canonical order)
    D[d]        incidence from dimension d to d+1 (G, C, Dv)
    X           vertex coordinates in fine lattice units
    measure[d]  length / area / volume (true units), 1 for vertices
    orient[d]   orientation vectors: edge direction (d=1), face normal (d=2)
    cell_mass   {1: (idx, mats), 2: (idx, mats)}  ND / RT mass per cell
    face_mass   (idx, mats)  ND tangential-trace mass per face
    side        cell side in fine lattice units
    """

    def __init__(self, k, X, ent, D, measure, orient, cell_mass, face_mass, side, keys):
        self.k, self.X, self.ent, self.D = k, X, ent, D
        self.measure, self.orient = measure, orient
        self.cell_mass, self.face_mass = cell_mass, face_mass
        self.side, self.keys = side, keys

    def ndofs(self, d):
        return len(self.ent[d])


def fine_level(mesh: FineMesh, weights=None) -> Level:
    """Fine level of the Kuhn mesh; weights: {space: per-tet factor} multiplying that
    space's element masses (coefficient-aware extensions)."""
    h = mesh.h
    ev, fn = mesh.edge_vectors(), mesh.face_normals()
    measure = [np.ones(mesh.nv),
               np.linalg.norm(ev.astype(float), axis=1) * h,
               np.linalg.norm(fn.astype(float), axis=1) / 2.0 * h * h,
               mesh.volumes()]
    ent = [np.arange(mesh.nv)[:, None], mesh.edges, mesh.faces, mesh.tets]
    masses = {1: mesh.nd_element_mass(), 2: mesh.rt_element_mass()}
    for i, w in (weights or {}).items():
        masses[i] = masses[i] * np.asarray(w, dtype=np.float64)[:, None, None]
    return Level(1, mesh.X, ent, [mesh.grad(), mesh.curl(), mesh.div()], measure,
                 [None, ev, fn, None],
                 {1: (mesh.tet_edges, masses[1]), 2: (mesh.tet_faces, masses[2])},
                 (mesh.face_edges, mesh.nd_face_trace_mass()), 1, None)


def boundary_entities(level: Level, d: int):
    """Mask of the d-dimensional entities of a level lying in the boundary of the cube:
    all their vertices on one of its six faces."""
    X = np.asarray(level.X)
    top = X.max(axis=0)
    V = X[np.asarray(level.ent[d])]          # (entities, vertices, 3)
    on = np.zeros(len(V), dtype=bool)
    for a in range(3):
        on |= np.all(V[:, :, a] == 0, axis=1) | np.all(V[:, :, a] == top[a], axis=1)
    return on


def cube_level(k: int, N: int, side: int, h: float) -> Level:
    """Cube complex with N cells per side, cell side `side` fine lattice units.

    Orientation: edge (p, a) runs along +e_a; face (p, a) has normal +e_a with
    boundary edge(p,b) + edge(p+e_b,c) - edge(p+e_c,b) - edge(p,c), (a,b,c) cyclic;
    a cube carries +1 on its upper and -1 on its lower faces.
    """
    M = N + 1
    nv = M ** 3
    lat = np.arange(nv)
    P = np.stack([lat % M, (lat // M) % M, lat // (M * M)], axis=1).astype(np.int64)
    vid = lambda p: p[:, 0] + M * (p[:, 1] + M * p[:, 2])
    e = np.eye(3, dtype=np.int64)

    # edges: (tail, head), sorted lexicographically
    tails, heads, eax = [], [], []
    for a in range(3):
        p = P[P[:, a] < N]
        tails.append(vid(p)); heads.append(vid(p + e[a])); eax.append(np.full(len(p), a))
    E = np.stack([np.concatenate(tails), np.concatenate(heads)], axis=1)
    eax = np.concatenate(eax)
    o = np.lexsort(E.T[::-1]); E, eax = E[o], eax[o]
    ekey = E[:, 0] * nv + E[:, 1]

    # faces: 4 sorted vertices; key (min vertex, 2 - normal axis) matches the tuple order
    fv, fax, fbase = [], [], []
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        p = P[(P[:, b] < N) & (P[:, c] < N)]
        fv.append(np.sort(np.stack([vid(p), vid(p + e[b]), vid(p + e[c]), vid(p + e[b] + e[c])], 1), 1))
        fax.append(np.full(len(p), a)); fbase.append(p)
    F, fax, fbase = np.concatenate(fv), np.concatenate(fax), np.concatenate(fbase)
    o = np.lexsort(F.T[::-1]); F, fax, fbase = F[o], fax[o], fbase[o]
    fkey = 3 * F[:, 0] + (2 - fax)
    assert np.all(np.diff(fkey) > 0)

    # cubes: 8 sorted vertices; key = min vertex
    p = P[np.all(P < N, axis=1)]
    corners = [p + sum(e[a] * bits[a] for a in range(3))
               for bits in np.ndindex(2, 2, 2)]
    T = np.sort(np.stack([vid(q) for q in corners], 1), 1)
    o = np.lexsort(T.T[::-1]); T, tbase = T[o], p[o]
    tkey = T[:, 0]

    def edge_id(p, a):
        return np.searchsorted(ekey, vid(p) * nv + vid(p + e[a]))

    def face_id(p, a):
        return np.searchsorted(fkey, 3 * vid(p) + (2 - a))

    nE, nF, nT = len(E), len(F), len(T)
    G = sp.csr_matrix((np.tile([-1.0, 1.0], nE), (np.repeat(np.arange(nE), 2), E.reshape(-1))),
                      shape=(nE, nv))
    rows, cols, vals = [], [], []
    for a in range(3):
        sel = np.nonzero(fax == a)[0]
        b, c = (a + 1) % 3, (a + 2) % 3
        q = fbase[sel]
        for ids, v in ((edge_id(q, b), 1.0), (edge_id(q + e[b], c), 1.0),
                       (edge_id(q + e[c], b), -1.0), (edge_id(q, c), -1.0)):
            rows.append(sel); cols.append(ids); vals.append(np.full(len(sel), v))
    C = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(nF, nE))
    rows, cols, vals = [], [], []
    for a in range(3):
        for q, v in ((tbase + e[a], 1.0), (tbase, -1.0)):
            rows.append(np.arange(nT)); cols.append(face_id(q, a)); vals.append(np.full(nT, v))
    Dv = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(nT, nF))

    X = P * side
    ev = X[E[:, 1]] - X[E[:, 0]]
    fn = e[fax] * side * side
    hs = h * side
    measure = [np.ones(nv), np.full(nE, hs), np.full(nF, hs * hs), np.full(nT, hs ** 3)]
    ent = [lat[:, None], E, F, T]
    keys = dict(nv=nv, M=M, ekey=ekey, fkey=fkey, tkey=tkey, vid=vid)
    return Level(k, X, ent, [G, C, Dv], measure, [None, ev, fn, None], None, None, side, keys)


# ----------------------------------------------------------------------------
# classification of finer entities into coarse ones
# ----------------------------------------------------------------------------
def classify(fine: Level, coarse: Level):
    """Owner (dimension, index) and orientation sign of every finer entity.

    A finer entity lies in the relative interior of exactly one coarse entity:
    the one whose dimension is the number of non-integer coordinates of the
    finer entity's centroid measured in coarse cells.
    """
    S = coarse.side
    kk = coarse.keys
    nv, M, vid = kk["nv"], kk["M"], kk["vid"]
    e = np.eye(3, dtype=np.int64)
    out = []
    for d in range(4):
        ent = fine.ent[d]
        cnt = ent.shape[1]
        sums = fine.X[ent].sum(axis=1)
        nonint = (sums % (cnt * S)) != 0
        base = sums // (cnt * S)
        dim = nonint.sum(axis=1)
        owner = np.full(len(ent), -1, dtype=np.int64)
        phi = np.ones(len(ent))
        # vertices
        s0 = dim == 0
        owner[s0] = vid(base[s0])
        # edges
        s1 = np.nonzero(dim == 1)[0]
        if len(s1):
            a = np.argmax(nonint[s1], axis=1)
            key = vid(base[s1]) * nv + vid(base[s1] + e[a])
            owner[s1] = np.searchsorted(kk["ekey"], key)
            assert np.all(kk["ekey"][owner[s1]] == key)
            if d == 1:
                phi[s1] = np.sign(fine.orient[1][s1][np.arange(len(s1)), a])
        # faces
        s2 = np.nonzero(dim == 2)[0]
        if len(s2):
            a = np.argmin(nonint[s2], axis=1)          # the integer axis is the normal
            key = 3 * vid(base[s2]) + (2 - a)
            owner[s2] = np.searchsorted(kk["fkey"], key)
            assert np.all(kk["fkey"][owner[s2]] == key)
            if d == 2:
                phi[s2] = np.sign(fine.orient[2][s2][np.arange(len(s2)), a])
        s3 = np.nonzero(dim == 3)[0]
        if len(s3):
            key = vid(base[s3])
            owner[s3] = np.searchsorted(kk["tkey"], key)
            assert np.all(kk["tkey"][owner[s3]] == key)
        assert np.all(phi != 0)
        out.append((dim, owner, phi))
    return out


def _group(dim, owner, dw, n_coarse, n_fine):
    """Boolean CSR: coarse dw-entity -> finer entities in its relative interior."""
    sel = np.nonzero(dim == dw)[0]
    return sp.csr_matrix((np.ones(len(sel)), (owner[sel], sel)), shape=(n_coarse, n_fine))


def _bool(A):
    A = A.tocsr().copy()
    A.data[:] = 1.0
    A.eliminate_zeros()
    A.sort_indices()
    return A


def _rows(A, r):
    return A.indices[A.indptr[r]:A.indptr[r + 1]]


def _rows2d(A, Zs):
    """Rows Zs of a CSR pattern as a 2-D array (all rows must have equal length)."""
    lens = A.indptr[Zs + 1] - A.indptr[Zs]
    if len(Zs) == 0:
        return np.zeros((0, 0), dtype=np.int64)
    assert np.all(lens == lens[0]), "entities of one batch must have equal closures"
    idx = A.indptr[Zs][:, None] + np.arange(lens[0])[None, :]
    return A.indices[idx].astype(np.int64)


def batched_block(A, rows2d, cols2d):
    """out[b] = dense A[rows2d[b], cols2d[b]]; every row of cols2d must be sorted."""
    A = A.tocsr()
    nb, nr = rows2d.shape
    nc = cols2d.shape[1]
    out = np.zeros((nb, nr, nc))
    if nb == 0 or nr == 0 or nc == 0:
        return out
    r = rows2d.reshape(-1)
    starts = A.indptr[r]
    lens = A.indptr[r + 1] - starts
    flat = np.repeat(np.arange(nb * nr), lens)
    pos = np.repeat(starts, lens) + (np.arange(lens.sum()) - np.repeat(np.cumsum(lens) - lens, lens))
    c = A.indices[pos].astype(np.int64)
    b = flat // nr
    big = A.shape[1] + 1
    colkey = (np.arange(nb)[:, None] * big + cols2d).reshape(-1)
    q = b * big + c
    j = np.searchsorted(colkey, q)
    jc = np.minimum(j, len(colkey) - 1)
    ok = colkey[jc] == q
    out.reshape(nb * nr, nc)[flat[ok], j[ok] - b[ok] * nc] = A.data[pos[ok]]
    return out


def batched_mass(cells2d, idx, mats, dofs2d):
    """out[b] = sum over cells c in cells2d[b] of the element mass mats[c] placed on dofs2d[b]."""
    nb, nd = dofs2d.shape
    E = idx[cells2d]                                   # (nb, ncell, nl)
    nl = E.shape[2]
    big = int(max(dofs2d.max(), E.max())) + 1
    key = (np.arange(nb)[:, None] * big + dofs2d).reshape(-1)
    q = np.arange(nb)[:, None, None] * big + E
    loc = np.searchsorted(key, q) - np.arange(nb)[:, None, None] * nd
    assert np.all(dofs2d[np.arange(nb)[:, None, None], loc] == E)
    flat = (np.arange(nb)[:, None, None, None] * nd * nd + loc[:, :, :, None] * nd + loc[:, :, None, :])
    w = mats[cells2d]                                  # (nb, ncell, nl, nl)
    return np.bincount(flat.reshape(-1), weights=w.reshape(-1), minlength=nb * nd * nd).reshape(nb, nd, nd)


def _unique_rows(*arrays):
    """Indices of the distinct rows of the concatenated per-batch inputs, and the inverse map.

    Rows are grouped by an exact integer fingerprint of their bits and then
    compared element by element, so only bitwise-equal rows are merged.
    """
    nb = arrays[0].shape[0]
    parts = [np.ascontiguousarray(a, dtype=np.float64).reshape(nb, -1) for a in arrays]
    # candidate groups from a random projection (rows with equal bits project equally);
    # membership is then confirmed bit for bit below
    fp = np.zeros(nb)
    rng = np.random.default_rng(20210712)
    for b in parts:
        fp += b @ rng.standard_normal(b.shape[1])
    _, first, inv = np.unique(fp, return_index=True, return_inverse=True)
    inv = inv.reshape(-1)
    rep = first[inv]
    def same(b):
        bu = b.view(np.uint64)
        return all(np.array_equal(bu[i:i + 64], bu[rep[i:i + 64]]) for i in range(0, nb, 64))
    if all(same(b) for b in parts):
        return first, inv
    # fingerprint collision between different rows: fall back to exact byte keys
    flat = np.concatenate([b.view(np.uint64) for b in parts], axis=1)
    seen, firsts, inv = {}, [], np.empty(nb, dtype=np.int64)
    for r in range(nb):
        key = flat[r].tobytes()
        j = seen.get(key)
        if j is None:
            j = seen[key] = len(firsts)
            firsts.append(r)
        inv[r] = j
    return np.array(firsts, dtype=np.int64), inv


def _batches(Zs, size=1024):
    for s in range(0, len(Zs), size):
        yield Zs[s:s + size]


# ----------------------------------------------------------------------------
# local minimum-mass extension (eqs. (3.6), (3.8)) by the SVD null-space method
# ----------------------------------------------------------------------------
def _svd_split(KI):
    U, s, Vt = np.linalg.svd(KI, full_matrices=True)
    smax = s.max() if s.size else 0.0
    r = int(np.sum(s > SVD_NULL_TOL * smax)) if smax > 0 else 0
    return U, s, Vt, r


def minmass_extend(M, K, interior, rhs, ub):
    """Solve min 1/2 u^T M u s.t. K[:, I] u_I = rhs - K[:, B] u_B, u_B = ub (column-wise).

    M, K are given on the closure dofs of the entity; `interior` masks its
    interior dofs.  Returns u_I (n_I x ncols).  The constraint must be consistent.
    """
    I, B = interior, ~interior
    KI, KB = K[:, I], K[:, B]
    g = rhs - KB @ ub
    U, s, Vt, r = _svd_split(KI)
    # particular solution u_p = K_I^+ g
    up = Vt[:r].T @ ((U[:, :r].T @ g) / s[:r, None])
    res = np.linalg.norm(KI @ up - g)
    if res > 1e-10 * max(1.0, np.linalg.norm(g)):
        raise AssertionError(f"inconsistent extension constraint, residual {res:g}")
    N = Vt[r:].T
    if N.shape[1] == 0:
        return up
    if M is None:
        raise AssertionError("extension not determined by its constraint and no mass given")
    MII, MIB = M[np.ix_(I, I)], M[np.ix_(I, B)]
    w = -np.linalg.solve(N.T @ MII @ N, N.T @ (MII @ up + MIB @ ub))
    return up + N @ w


def dfree_bubble_projection(M, K, interior, t):
    """L2(Z) projection of the columns of t onto {u: u_B = 0, K_I u_I = 0}; returns (u_I, N)."""
    I, B = interior, ~interior
    U, s, Vt, r = _svd_split(K[:, I])
    N = Vt[r:].T
    if N.shape[1] == 0:
        return np.zeros((int(I.sum()), t.shape[1])), N
    MII, MIB = M[np.ix_(I, I)], M[np.ix_(I, B)]
    w = np.linalg.solve(N.T @ MII @ N, N.T @ (MII @ t[I] + MIB @ t[B]))
    return N @ w, N


def surviving(R, T_raw, Mnorm):
    """Number of independent columns of R (M-norm SVD) above the relative target tolerance."""
    if R.size == 0:
        return 0
    L = np.linalg.cholesky(Mnorm)
    sr = np.linalg.svd(L.T @ R, compute_uv=False)
    st = np.linalg.svd(L.T @ T_raw, compute_uv=False)
    return int(np.sum(sr > TARGET_TOL * max(1.0, st.max() if st.size else 0.0)))


# ----------------------------------------------------------------------------
# one coarsening step
# ----------------------------------------------------------------------------
class _Coarsening:
    """Topological bookkeeping of one agglomeration step (section 3.1)."""

    def __init__(self, fine: Level, h: float):
        if not np.all(np.asarray(fine.X).max(axis=0) % (2 * fine.side) == 0):
            raise ValueError("lattice not divisible by 2")
        N = int(fine.X[:, 0].max() // (2 * fine.side))
        self.fine = fine
        self.coarse = coarse = cube_level(fine.k + 1, N, 2 * fine.side, h)
        self.cls = cls = classify(fine, coarse)
        nc = self.nc = [coarse.ndofs(d) for d in range(4)]
        nf = self.nf = [fine.ndofs(d) for d in range(4)]
        Gh, Ch, Dh = (abs(coarse.D[0]), abs(coarse.D[1]), abs(coarse.D[2]))
        # sub[(dz, dw)]: coarse entities of dim dw in the closure of a dz-entity
        sub = {(d, d): sp.identity(nc[d], format="csr") for d in range(4)}
        sub[(1, 0)] = _bool(Gh)
        sub[(2, 1)] = _bool(Ch)
        sub[(2, 0)] = _bool(Ch @ Gh)
        sub[(3, 2)] = _bool(Dh)
        sub[(3, 1)] = _bool(Dh @ Ch)
        sub[(3, 0)] = _bool(Dh @ Ch @ Gh)
        self.sub = sub
        # interior[i][dw]: coarse dw-entity -> finer i-entities in its relative interior
        self.interior = {i: {dw: _group(cls[i][0], cls[i][1], dw, nc[dw], nf[i]) for dw in range(4)}
                         for i in range(4)}
        self.closure = {}
        for i in range(4):
            for dz in range(i, 4):
                acc = None
                for dw in range(dz + 1):
                    t = sub[(dz, dw)] @ self.interior[i][dw]
                    acc = t if acc is None else acc + t
                self.closure[(i, dz)] = _bool(acc)

    def local(self, i, dz, Zs):
        """Closure dofs (sorted), interior mask and L2 mass of space i on the entities Zs."""
        dofs = _rows2d(self.closure[(i, dz)], Zs)
        intr = self.cls[i][0][dofs] == dz
        M = None
        if i == 1 and dz == 2:          # tangential-trace mass on a coarse face
            cells = _rows2d(self.interior[2][2], Zs)
            M = batched_mass(cells, self.fine.face_mass[0], self.fine.face_mass[1], dofs)
        elif i in (1, 2) and dz == 3:   # full mass on a coarse cell
            cells = _rows2d(self.interior[3][3], Zs)
            idx, mats = self.fine.cell_mass[i]
            M = batched_mass(cells, idx, mats, dofs)
        return dofs, intr, M


def coarsen(fine: Level, h: float, spaces=(0, 1, 2, 3), targets=None, check_targets=True):
    """Build the next level, the prolongators and co-chain projectors for `spaces`.

    Spaces are built in reverse order L2 -> RT -> ND -> H1 (section 3), each one
    from PV traces on its lowest-dimensional coarse entities, then extended to
    entities of increasing dimension.  `targets` maps space -> (ndof x m) target
    vectors on `fine` (order-0 interpolants); they are filtered against the PV
    traces and projected onto D-free bubbles, and the number of survivors is
    asserted to be zero (no higher-order coarse dofs are built).

    Every coarse entity gets its own local problem; entities are visited in
    batches and a local problem whose inputs are bitwise equal to an earlier
    one in the batch is not solved twice.
    """
    cg = _Coarsening(fine, h)
    coarse, cls, nc, nf = cg.coarse, cg.cls, cg.nc, cg.nf
    P, Pi = {}, {}
    for i in sorted(spaces, reverse=True):
        # PV traces, eq. (3.5): unit integral, oriented constituents
        dim_i, own_i, phi_i = cls[i]
        sel = np.nonzero(dim_i == i)[0]
        X = own_i[sel]
        vals = phi_i[sel] * fine.measure[i][sel] / coarse.measure[i][X]
        rows, cols, data = [sel], [X], [vals]
        Pi[i] = sp.csr_matrix((phi_i[sel], (X, sel)), shape=(nc[i], nf[i]))
        Pcur = sp.csr_matrix((vals, (sel, X)), shape=(nf[i], nc[i]))
        # extensions to entities of increasing dimension, eqs. (3.6) and (3.8)
        for dz in range(i + 1, 4):
            # target of the derivative: D P_i = P_{i+1} D^H  restricted to Z
            Q = (P[i + 1] @ coarse.D[i]).tocsr()
            for Zs in _batches(np.arange(nc[dz])):
                dofs, intr, M = cg.local(i, dz, Zs)
                nI = int(intr[0].sum())
                yrows = _rows2d(cg.interior[i + 1][dz], Zs)
                Xs = _rows2d(cg.sub[(dz, i)], Zs)
                K = batched_block(fine.D[i], yrows, dofs)
                S = batched_block(Q, yrows, Xs)
                bdofs = dofs[~intr].reshape(len(Zs), -1)
                UB = batched_block(Pcur, bdofs, Xs)
                parts = [K, S, UB, intr] + ([M] if M is not None else [])
                first, inv = _unique_rows(*parts)
                sol = np.stack([minmass_extend(None if M is None else M[u], K[u], intr[u], S[u], UB[u])
                                for u in first])
                UI = sol[inv]                              # (nb, nI, nX)
                ri = dofs[intr].reshape(len(Zs), nI)
                rows.append(np.repeat(ri[:, :, None], Xs.shape[1], axis=2).reshape(-1))
                cols.append(np.repeat(Xs[:, None, :], nI, axis=1).reshape(-1))
                data.append(UI.reshape(-1))
            r_, c_, v_ = np.concatenate(rows), np.concatenate(cols), np.concatenate(data)
            keep = v_ != 0
            Pcur = sp.csr_matrix((v_[keep], (r_[keep], c_[keep])), shape=(nf[i], nc[i]))
        P[i] = Pcur.tocsr()
        P[i].sort_indices()

        # order-0 targets (sections 3.3.1-3.3.3): filtered against PV, projected on D-free bubbles
        if check_targets and targets is not None and i in targets and i != 0:
            _check_targets(cg, i, targets[i])

    # coarse element masses by RAP (section 3.3.2: trace masses produced by RAP)
    cell_mass, face_mass = {}, None
    for i in (1, 2):
        if i in P:
            idx_l, mats_l = [], []
            for Zs in _batches(np.arange(nc[3])):
                dofs, _, Mt = cg.local(i, 3, Zs)
                cd = _rows2d(cg.sub[(3, i)], Zs)
                PT = batched_block(P[i], dofs, cd)
                idx_l.append(cd); mats_l.append(PT.transpose(0, 2, 1) @ Mt @ PT)
            cell_mass[i] = (np.concatenate(idx_l), np.concatenate(mats_l))
    if 1 in P:
        idx_l, mats_l = [], []
        for Zs in _batches(np.arange(nc[2])):
            dofs, _, Mf = cg.local(1, 2, Zs)
            cd = _rows2d(cg.sub[(2, 1)], Zs)
            PF = batched_block(P[1], dofs, cd)
            idx_l.append(cd); mats_l.append(PF.transpose(0, 2, 1) @ Mf @ PF)
        face_mass = (np.concatenate(idx_l), np.concatenate(mats_l))
    coarse.cell_mass, coarse.face_mass = cell_mass, face_mass
    return coarse, P, Pi


def _check_targets(cg, i, T):
    """Assert that no order-0 target survives PV removal or D-free bubble projection."""
    fine, coarse, cls = cg.fine, cg.coarse, cg.cls
    dim_i, own_i, phi_i = cls[i]
    m = T.shape[1]
    # lowest-dimensional entities: remove the component along the PV trace, using the
    # diagonal trace mass of the PV-type finer space (1 / measure per dof)
    for Zs in _batches(np.arange(cg.nc[i]), 8192):
        dofs = _rows2d(cg.interior[i][i], Zs)
        t = T[dofs]                                           # (nb, nI, m)
        pv = phi_i[dofs] * fine.measure[i][dofs] / coarse.measure[i][Zs][:, None]
        w = 1.0 / fine.measure[i][dofs]
        c = np.einsum("bi,bi,bim->bm", pv, w, t) / np.einsum("bi,bi,bi->b", pv, w, pv)[:, None]
        R = t - pv[:, :, None] * c[:, None, :]
        rn = np.sqrt(np.einsum("bi,bim->b", w, R * R))
        tn = np.sqrt(np.einsum("bi,bim->b", w, t * t))
        for b in np.nonzero(rn > TARGET_TOL * np.maximum(1.0, tn))[0]:
            if surviving(R[b], t[b], np.diag(w[b])):
                raise NotImplementedError("a target survived PV removal: higher-order coarse dofs are not built")
    # higher-dimensional entities: projection onto D-free bubbles
    for dz in range(i + 1, 4):
        for Zs in _batches(np.arange(cg.nc[dz])):
            dofs, intr, M = cg.local(i, dz, Zs)
            yrows = _rows2d(cg.interior[i + 1][dz], Zs)
            K = batched_block(fine.D[i], yrows, dofs)
            t = T[dofs]
            first, inv = _unique_rows(K, intr, M, t)
            for u in first:
                R, N = dfree_bubble_projection(M[u], K[u], intr[u], t[u])
                if N.shape[1] and surviving(R, t[u][intr[u]], M[u][np.ix_(intr[u], intr[u])]):
                    raise NotImplementedError("a target survived the bubble projection")


# ----------------------------------------------------------------------------
# targets
# ----------------------------------------------------------------------------
def order0_targets(level: Level):
    """Interpolants of constants: ND (3 fields), RT (3 fields), L2 (the constant 1)."""
    h = 1.0 / level.X[:, 0].max() * 1.0   # lattice units -> true units (unit cube)
    ev = level.orient[1].astype(float) * h
    fn = level.orient[2].astype(float)
    # face interpolant: flux of c through the face = c . (unit normal) * area
    nrm = fn / np.linalg.norm(fn, axis=1, keepdims=True)
    return {1: ev.copy(), 2: nrm * level.measure[2][:, None], 3: level.measure[3][:, None].copy()}


# ----------------------------------------------------------------------------
# the full hierarchy
# ----------------------------------------------------------------------------
class Hierarchy:
    """Per level: system matrix A, derivative D used by the hybrid smoother,
    prolongator P to the next coarser level, plus the full sequence data."""

    def __init__(self):
        self.levels, self.A, self.D, self.P, self.Pall, self.Piall = [], [], [], [], [], []


def build_hierarchy(kind: str, n: int, nlevels: int, alpha_hex, beta_hex, spaces=None,
                    check_targets=True, extension="l2", bc="natural"):
    """FP64 hierarchy for H(curl) (kind='curl') or H(div) (kind='div').

    spaces: which sequence spaces to coarsen (default: the ones the system
    space needs -- ND needs RT and L2; RT needs L2 -- plus H1 for small meshes).
    extension: "l2" (unweighted local problems) or "coefficient" (masses of the system
    space weighted by beta, of the next space by alpha; the order-0 target check does
    not apply to weighted masses and is skipped).
    bc: "natural", or "essential" (every level restricted to its interior entities;
    H.interior[k] is the kept mask of level k's system space).
    """
    if extension not in ("l2", "coefficient") or bc not in ("natural", "essential"):
        raise ValueError("extension must be 'l2' or 'coefficient', bc 'natural' or 'essential'")
    mesh = FineMesh(n)
    A, G, C, Dv = fine_problem(mesh, kind, alpha_hex, beta_hex)
    sys_space = 1 if kind == "curl" else 2
    weights = None
    if extension == "coefficient":
        a_t = np.asarray(alpha_hex, dtype=np.float64)[mesh.tet_hex]
        b_t = np.asarray(beta_hex, dtype=np.float64)[mesh.tet_hex]
        weights = {sys_space: b_t}
        if sys_space + 1 <= 2:
            weights[sys_space + 1] = a_t
        check_targets = False
    lev = fine_level(mesh, weights)
    if spaces is None:
        spaces = tuple(range(sys_space, 4)) + ((0,) if n <= 16 and kind == "curl" else ())
    H = Hierarchy()
    H.kind, H.n, H.sys_space = kind, n, sys_space
    H.levels.append(lev)
    H.A.append(A)
    H.D.append(lev.D[sys_space - 1])
    targets = order0_targets(lev) if check_targets else None
    h = mesh.h
    for k in range(1, nlevels):
        coarse, P, Pi = coarsen(lev, h, spaces=spaces, targets=targets, check_targets=check_targets)
        Psys = P[sys_space]
        Ac = (Psys.T @ H.A[-1] @ Psys).tocsr()
        Ac.sum_duplicates(); Ac.sort_indices()
        H.P.append(Psys)
        H.Pall.append(P)
        H.Piall.append(Pi)
        H.levels.append(coarse)
        H.A.append(Ac)
        H.D.append(coarse.D[sys_space - 1].tocsr())
        if targets is not None:
            targets = {s: Pi[s] @ targets[s] for s in targets if s in Pi}
        lev = coarse
    H.extension, H.bc = extension, bc
    if bc == "essential":
        keep = [~boundary_entities(L, sys_space) for L in H.levels]
        keepd = [~boundary_entities(L, sys_space - 1) for L in H.levels]
        H.interior = keep
        for k in range(nlevels):
            H.A[k] = H.A[k][keep[k]][:, keep[k]].tocsr()
            H.D[k] = H.D[k][keep[k]][:, keepd[k]].tocsr()
            if k < nlevels - 1:
                H.P[k] = H.P[k][keep[k]][:, keep[k + 1]].tocsr()
    return H
