"""A second FP64 evaluation of the oracle's arithmetic, for the FP64 parity bar.

Test helper only (not part of the oracle).  `Reformulated` computes the same
preconditioner as `oracle.solve.Multilevel` (Algorithm 4.1 with the hybrid smoother of
eq. (4.1) and an exact coarsest solve) with three steps evaluated differently, each
equal to the oracle's in exact arithmetic:

* the coarsest solve applies the explicit inverse W^T W formed from the Cholesky
  factor (W = L^{-1}) instead of two triangular solves;
* the auxiliary residual D^T (b - A x) is evaluated as D^T b - (D^T A) x;
* below the fine level the restricted residual P^T (b - A x) is evaluated as
  P^T b - (P^T A) x.

These are the evaluation orders the library uses.  The distance between the two
evaluations after the same number of PCG iterations (`spread`) is how closely the
method's FP64 result is determined by its definition: on the 1e6-contrast jump
workloads it is ~3e-10, above the 1e-10 solution-error bar, so no evaluation order
other than the oracle's own can be held to 1e-10 there.  The GPU parity tests hold the
library to max(1e-10, SPREAD_FACTOR * spread).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from oracle.solve import Multilevel, gs_sweep, pcg

SPREAD_FACTOR = 3.0


class Reformulated(Multilevel):
    def __init__(self, As, Ds, Ps, **kw):
        super().__init__(As, Ds, Ps, **kw)
        Ac = As[-1].toarray()
        Wc = sla.solve_triangular(np.linalg.cholesky(Ac), np.eye(Ac.shape[0]), lower=True)
        self.Ainv = Wc.T @ Wc
        for lv in self.levels[:-1]:
            lv.DtA = (lv.D.T @ lv.A).tocsr()
            lv.PtA = (lv.P.T @ lv.A).tocsr()

    def coarse_solve(self, b):
        return self.Ainv @ b

    @staticmethod
    def auxiliary(lv, b, x):
        g = lv.D.T @ b - lv.DtA @ x
        y = np.zeros_like(g)
        for _ in range(lv.nu_aux):
            if lv.smoother == "symgs":
                y = gs_sweep(lv.Ahat, lv.diaghat, lv.classes_hat, g, y, lv.blocks_hat)
            elif lv.smoother == "l1blockgs":
                y = lv.bgs_hat.sweep(g, y)
            else:
                y = y + (g - lv.Ahat @ y) / lv.dhat
        return x + lv.D @ y

    def vcycle(self, b, l=0, x0=None):
        if l == len(self.levels) - 1:
            return self.coarse_solve(b)
        lv = self.levels[l]
        x = np.zeros_like(b) if x0 is None else x0.copy()
        x = self.smooth(lv, b, x)
        bc = lv.P.T @ (b - lv.A @ x) if l == 0 else lv.P.T @ b - lv.PtA @ x
        x = x + lv.P @ self.vcycle(bc, l + 1)
        return self.smooth_transpose(lv, b, x)

    __call__ = vcycle


def relmax(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def spreads(H, b, iters, nu_primary=2, nu_aux=2, smoother="l1jacobi"):
    """Distances between the oracle and its reformulation on right-hand side b: one
    smoother application per level (max-norm relative), one V-cycle (max-norm
    relative) and PCG after `iters` iterations (2-norm relative)."""
    ml = Multilevel.from_hierarchy(H, nu_primary=nu_primary, nu_aux=nu_aux, smoother=smoother)
    rf = Reformulated(H.A, H.D, H.P, nu_primary=nu_primary, nu_aux=nu_aux, smoother=smoother)
    rng = np.random.default_rng(8)
    smooth = 0.0
    for k in range(len(H.A) - 1):
        bk = rng.uniform(-1, 1, H.A[k].shape[0])
        xk = rng.uniform(-1, 1, H.A[k].shape[0])
        for a, c in ((ml.smooth, rf.smooth), (ml.smooth_transpose, rf.smooth_transpose)):
            smooth = max(smooth, relmax(c(rf.levels[k], bk, xk), a(ml.levels[k], bk, xk)))
    vc = relmax(rf.vcycle(b), ml.vcycle(b))
    xo, _, _ = pcg(H.A[0], b, ml, fixed_iters=iters)
    xr, _, _ = pcg(H.A[0], b, rf, fixed_iters=iters)
    pc = float(np.linalg.norm(xr - xo) / np.linalg.norm(xo))
    return {"smooth": smooth, "vcycle": vc, "pcg": pc}


def fp64_bar(spread):
    """The FP64 parity bar for a quantity whose reformulation spread is `spread`."""
    return max(1e-10, SPREAD_FACTOR * spread)
