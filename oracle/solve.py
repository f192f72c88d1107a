"""Oracle, solve phase: hybrid smoother (l1-Jacobi, Gauss-Seidel), V-cycle, inexact PCG (FP64).

Test infrastructure only (see the package docstring).

Paper anchors
-------------
* Section 4.1, eq. (4.1): hybrid smoother -- a point smoother on A, then a point
  smoother on the auxiliary matrix D^T A D applied to D^T times the residual,
  with the correction mapped back through D.  The transpose smoother runs the
  two steps in reverse order with the transposed point smoothers.
* Section 4.1 (smoother choice) and section 5.1: two sweeps for the primary and
  for the auxiliary smoothing.  Three point smoothers:
  - l1-Jacobi (default), d_i = sum_j |a_ij| (the l1 scaling of the cited smoother
    paper with point blocks); its sweeps are symmetric so M^{-T} = M^{-1};
  - symmetric Gauss-Seidel in colour order (smoother="symgs"), the smoother the
    paper's experiments use (l1-scaled symmetric Gauss-Seidel): rows are coloured
    greedily (first fit in increasing row order: the smallest colour no earlier
    neighbour holds), a forward sweep relaxes the colours in increasing order, each
    row i by x_i += (b - A x)_i / a_ii, and the backward sweep in decreasing order.
    Rows of one colour are not coupled, so each colour is one exact block step; the
    l1 term of the cited smoother, which covers couplings to rows relaxed in parallel
    in other blocks, is empty when the colours are the blocks.  One symmetric sweep
    is symmetric, so again M^{-T} = M^{-1}.
  - l1-scaled symmetric block Gauss-Seidel (smoother="l1blockgs"), the smoother of
    the cited smoother paper with row blocks in place of processors: row i belongs
    to block i // gs_block (contiguous ranges of gs_block rows); inside a block the
    rows are coloured greedily over the couplings within the block (first fit in
    increasing row order) and relaxed colour by colour, forward through the colours
    and then backward through all of them again, each row i by
        x_i += (b_i - sum_{j in block} a_ij x_j - sum_{j not in block} a_ij x0_j) / d_i,
        d_i = a_ii + sum_{j not in block} |a_ij|,
    where x holds the current values and x0 the values at the start of the sweep
    (couplings across blocks are relaxed Jacobi-fashion, their weight moved to the
    diagonal: the l1 scaling).  Blocks of one row give a closed form built from
    l1-Jacobi steps, one block holding every row gives the Gauss-Seidel above, and
    the sweep is symmetric, x += Mb^{-1} (D + 2 D_l1) Mf^{-1} (b - A x) with Mf / Mb
    the block lower / upper factors (pinned by tests).
  The auxiliary sweeps start from zero.
* Algorithm 4.1: V-cycle, pre-relax, restrict with P^T, recurse or coarse solve,
  prolong, post-relax with the transposed smoother.
* Section 4.2 / 5.1: the coarsest-level solver; here an exact dense Cholesky
  solve in FP64 (the footnote of section 5.1 allows other coarse solvers).
* Section 4 (use in PCG) and section 5.1: one V-cycle with zero initial guess
  per PCG iteration; inexact (flexible) PCG; stop when the residual measured in
  the preconditioner norm has dropped by the relative tolerance.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def l1_diag(A):
    """Row l1 norms d_i = sum_j |a_ij| of a sparse matrix."""
    return np.asarray(abs(A).sum(axis=1)).ravel()


def greedy_coloring(A):
    """Colour of every row: the smallest non-negative integer not held by any earlier
    row (lower index) coupled to it (a_ij != 0, j != i), rows taken in increasing order."""
    A = A.tocsr()
    n = A.shape[0]
    color = np.full(n, -1, dtype=np.int64)
    for i in range(n):
        used = set()
        lo, hi = A.indptr[i], A.indptr[i + 1]
        for j, v in zip(A.indices[lo:hi], A.data[lo:hi]):
            if j < i and v != 0:
                used.add(int(color[j]))
        c = 0
        while c in used:
            c += 1
        color[i] = c
    return color


def gs_sweep(A, diag, classes, b, x, blocks=None):
    """One symmetric Gauss-Seidel sweep in colour order: colours increasing, then
    decreasing; rows of a colour relaxed together (they are not coupled).  blocks:
    optionally the row blocks A[rows] of the classes, sliced once."""
    x = x.copy()
    blocks = blocks if blocks is not None else [A[rows] for rows in classes]
    for rows, Ar in list(zip(classes, blocks)) + list(zip(classes, blocks))[::-1]:
        x[rows] += (b[rows] - Ar @ x) / diag[rows]
    return x


def block_coloring(A, blk):
    """Colour of every row over the couplings inside its own block (blk[i] is row i's
    block): the smallest non-negative integer not held by an earlier row of the same
    block coupled to it (a_ij != 0, j < i)."""
    A = A.tocsr()
    n = A.shape[0]
    color = np.full(n, -1, dtype=np.int64)
    for i in range(n):
        used = set()
        lo, hi = A.indptr[i], A.indptr[i + 1]
        for j, v in zip(A.indices[lo:hi], A.data[lo:hi]):
            if j < i and v != 0 and blk[j] == blk[i]:
                used.add(int(color[j]))
        c = 0
        while c in used:
            c += 1
        color[i] = c
    return color


class BlockGS:
    """Data of the l1-scaled symmetric block Gauss-Seidel sweep on A for a row partition
    blk: the couplings inside and across blocks, d_i = a_ii + sum_{j not in block}
    |a_ij|, and the rows of every colour (colours taken over couplings inside blocks)."""

    def __init__(self, A, blk):
        A = A.tocsr()
        self.A = A
        blk = np.asarray(blk)
        coo = A.tocoo()
        inside = blk[coo.row] == blk[coo.col]
        n = A.shape[0]
        self.A_in = sp.csr_matrix((coo.data[inside], (coo.row[inside], coo.col[inside])), shape=(n, n))
        self.A_off = sp.csr_matrix((coo.data[~inside], (coo.row[~inside], coo.col[~inside])), shape=(n, n))
        self.d = A.diagonal() + l1_diag(self.A_off)
        color = block_coloring(A, blk)
        C = int(color.max()) + 1 if n else 0
        self.classes = [np.nonzero(color == c)[0] for c in range(C)]
        self.rows_in = [self.A_in[rows] for rows in self.classes]

    def sweep(self, b, x):
        """One symmetric sweep: colours 0..C-1, then C-1..0; couplings across blocks
        read the values x0 at the start of the sweep."""
        x0 = x
        off = self.A_off @ x0
        x = x0.copy()
        order = list(range(len(self.classes)))
        for c in order + order[::-1]:
            rows = self.classes[c]
            x[rows] += (b[rows] - off[rows] - self.rows_in[c] @ x) / self.d[rows]
        return x


def contiguous_blocks(n, block):
    """Block index of every row for contiguous ranges of `block` rows."""
    return np.arange(n) // int(block)


class SolveLevel:
    def __init__(self, A, D, P=None, nu_primary=2, nu_aux=2, smoother="l1jacobi", gs_block=64):
        self.A = A.tocsr()
        self.D = D.tocsr()
        self.Ahat = (self.D.T @ self.A @ self.D).tocsr()
        self.d = l1_diag(self.A)
        self.dhat = l1_diag(self.Ahat)
        self.P = None if P is None else P.tocsr()
        self.nu_primary, self.nu_aux = nu_primary, nu_aux
        self.smoother = smoother
        if smoother == "symgs":
            self.diag, self.diaghat = self.A.diagonal(), self.Ahat.diagonal()
            self.classes = self._classes(greedy_coloring(self.A))
            self.classes_hat = self._classes(greedy_coloring(self.Ahat))
            self.blocks = [self.A[rows] for rows in self.classes]
            self.blocks_hat = [self.Ahat[rows] for rows in self.classes_hat]
        elif smoother == "l1blockgs":
            self.bgs = BlockGS(self.A, contiguous_blocks(self.A.shape[0], gs_block))
            self.bgs_hat = BlockGS(self.Ahat, contiguous_blocks(self.Ahat.shape[0], gs_block))
        elif smoother != "l1jacobi":
            raise ValueError(smoother)

    @staticmethod
    def _classes(color):
        return [np.nonzero(color == c)[0] for c in range(int(color.max()) + 1)] if len(color) else []


class Multilevel:
    """Algorithm 4.1 over a list of levels; the last one is solved by Cholesky."""

    def __init__(self, As, Ds, Ps, nu_primary=2, nu_aux=2, smoother="l1jacobi", gs_block=64):
        L = len(As)
        self.levels = [SolveLevel(As[k], Ds[k], Ps[k] if k < L - 1 else None, nu_primary, nu_aux,
                                  smoother if k < L - 1 else "l1jacobi", gs_block)
                       for k in range(L)]
        self.chol = sla.cho_factor(As[-1].toarray(), lower=True)

    @classmethod
    def from_hierarchy(cls, H, **kw):
        return cls(H.A, H.D, H.P, **kw)

    # --- hybrid smoother, eq. (4.1) -------------------------------------------
    @staticmethod
    def primary(lv, b, x):
        for _ in range(lv.nu_primary):
            if lv.smoother == "symgs":
                x = gs_sweep(lv.A, lv.diag, lv.classes, b, x, lv.blocks)
            elif lv.smoother == "l1blockgs":
                x = lv.bgs.sweep(b, x)
            else:
                x = x + (b - lv.A @ x) / lv.d
        return x

    @staticmethod
    def auxiliary(lv, b, x):
        g = lv.D.T @ (b - lv.A @ x)
        y = np.zeros_like(g)
        for _ in range(lv.nu_aux):
            if lv.smoother == "symgs":
                y = gs_sweep(lv.Ahat, lv.diaghat, lv.classes_hat, g, y, lv.blocks_hat)
            elif lv.smoother == "l1blockgs":
                y = lv.bgs_hat.sweep(g, y)
            else:
                y = y + (g - lv.Ahat @ y) / lv.dhat
        return x + lv.D @ y

    def smooth(self, lv, b, x):
        """x + M^{-1}(b - A x) with the hybrid smoother."""
        return self.auxiliary(lv, b, self.primary(lv, b, x))

    def smooth_transpose(self, lv, b, x):
        """x + M^{-T}(b - A x): the steps in reverse order."""
        return self.primary(lv, b, self.auxiliary(lv, b, x))

    # --- Algorithm 4.1 ----------------------------------------------------------
    def coarse_solve(self, b):
        return sla.cho_solve(self.chol, b)

    def vcycle(self, b, l=0, x0=None):
        if l == len(self.levels) - 1:
            return self.coarse_solve(b)
        lv = self.levels[l]
        x = np.zeros_like(b) if x0 is None else x0.copy()
        x = self.smooth(lv, b, x)
        ec = self.vcycle(lv.P.T @ (b - lv.A @ x), l + 1)
        x = x + lv.P @ ec
        return self.smooth_transpose(lv, b, x)

    __call__ = vcycle


def pcg(A, b, precond, rtol=1e-8, maxit=1000, stop="bnorm", fixed_iters=None):
    """Inexact PCG with x0 = 0.

    beta = (r_{k+1}.z_{k+1} - r_{k+1}.z_k) / (r_k.z_k), the flexible form that
    reduces to the standard one for a fixed symmetric preconditioner.
    stop = "bnorm": stop when sqrt(r.z / r0.z0) <= rtol (preconditioner norm);
    stop = "l2": stop when ||r|| / ||b|| <= rtol.
    fixed_iters: run exactly that many iterations regardless of the test.
    Returns (x, iterations, history) where iterations counts products with A.
    """
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    r = b.copy()
    z = precond(r)
    p = z.copy()
    delta = float(r @ z)
    delta0 = delta
    bnorm = float(np.linalg.norm(b))
    hist = [1.0]
    if delta0 <= 0 or not np.isfinite(delta0):
        raise FloatingPointError("preconditioner not positive on b")
    it = 0
    while True:
        if fixed_iters is not None and it >= fixed_iters:
            break
        if fixed_iters is None and it >= maxit:
            break
        q = A @ p
        pq = float(p @ q)
        if not pq > 0:
            raise FloatingPointError("PCG breakdown: p.q <= 0")
        alpha = delta / pq
        x = x + alpha * p
        r = r - alpha * q
        it += 1
        zn = precond(r)
        dn = float(r @ zn)
        rzo = float(r @ z)
        rel = np.sqrt(max(dn, 0.0) / delta0) if stop == "bnorm" else float(np.linalg.norm(r)) / bnorm
        hist.append(rel)
        if fixed_iters is None and rel <= rtol:
            break
        beta = (dn - rzo) / delta
        p = zn + beta * p
        z = zn
        delta = dn
    return x, it, hist


def cg_plain(A, b, rtol=1e-8, maxit=1000, fixed_iters=None):
    """Unpreconditioned CG (B = I) through the same loop."""
    return pcg(A, b, lambda r: r.copy(), rtol=rtol, maxit=maxit, stop="l2", fixed_iters=fixed_iters)
