"""Seeded synthetic workloads for the AMGe solve phase.

This module only draws random numbers and states problem shapes.  It holds no
finite-element, coarsening or solver arithmetic, so both the FP64 oracle and
the HIP path can take their inputs from it without sharing any of the method.

Conventions shared by every consumer (they are part of the input format):

* Mesh: the unit cube split into ``n**3`` hexahedra; hex ``(i, j, k)`` has
  linear index ``i + n*(j + n*k)``.
* Coefficients are piecewise constant on hexes.  Random fields are drawn per
  ``block**3``-hex block, blocks laid out from the origin, block ``(bi, bj, bk)``
  with linear index ``bi + nb*(bj + nb*bk)``; draws are made in that order.
* Right-hand sides are drawn per fine dof in the canonical dof order (entities
  sorted lexicographically by their sorted global vertex indices, vertex
  ``(i, j, k)`` having index ``i + (n+1)*(j + (n+1)*k)``).
"""
from __future__ import annotations

import dataclasses
import numpy as np

CURL = "curl"   # H(curl): lowest-order Nedelec, dofs on edges
DIV = "div"     # H(div): lowest-order Raviart-Thomas, dofs on faces


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    kind: str            # CURL or DIV
    n: int               # hexes per side
    levels: int          # levels in the agglomeration hierarchy
    coef: str            # "unit" or "blocks"
    coef_seed: int = 0
    nrhs: int = 1
    rhs_seed: int = 0
    rtol: float = 1e-8


# The five workloads; sizes follow the configurations the method is measured on.
WORKLOADS = {
    "curl_n8_l2": Workload("curl_n8_l2", CURL, 8, 2, "unit"),
    "div_n32_l4_jumps": Workload("div_n32_l4_jumps", DIV, 32, 4, "blocks"),
    "curl_n64_l5": Workload("curl_n64_l5", CURL, 64, 5, "unit"),
    "div_n48_l5_rhs32": Workload("div_n48_l5_rhs32", DIV, 48, 5, "unit", nrhs=32),
}


def default_levels(n: int) -> int:
    """Number of levels: halve the lattice while it is even and the half is >= 3."""
    levels, m = 1, n
    while m % 2 == 0 and m // 2 >= 3:
        m //= 2
        levels += 1
    return levels


def entity_counts(n: int) -> dict:
    """Closed-form entity counts of the Kuhn mesh (sizes only)."""
    m = n + 1
    return {
        "V": m ** 3,
        "E": 3 * n * m * m + 3 * n * n * m + n ** 3,
        "F": 6 * n * n * m + 6 * n ** 3,
        "T": 6 * n ** 3,
    }


def fine_dofs(kind: str, n: int) -> int:
    c = entity_counts(n)
    return c["E"] if kind == CURL else c["F"]


def block_coefficients(n: int, seed: int, block: int = 4, lo: float = -3.0, hi: float = 3.0):
    """Log-uniform values 10**U(lo, hi), one per block, in block-lexicographic order."""
    if n % block:
        raise ValueError("n must be a multiple of the block size")
    nb = n // block
    rng = np.random.default_rng(seed)
    return 10.0 ** rng.uniform(lo, hi, size=nb ** 3)


def hex_coefficients(n: int, block_values, block: int = 4):
    """Expand per-block values to per-hex values (hex-lexicographic, i fastest)."""
    nb = n // block
    bv = np.asarray(block_values, dtype=np.float64).reshape(nb, nb, nb)  # [bk, bj, bi]
    return np.repeat(np.repeat(np.repeat(bv, block, 0), block, 1), block, 2).reshape(-1)


def coefficients(w: Workload):
    """(alpha, beta) per hex.  alpha multiplies the derivative term, beta the mass term."""
    nh = w.n ** 3
    if w.coef == "unit":
        return np.ones(nh), np.ones(nh)
    if w.coef == "blocks":
        return hex_coefficients(w.n, block_coefficients(w.n, w.coef_seed)), np.ones(nh)
    raise ValueError(w.coef)


def rhs(ndofs: int, seed: int, nrhs: int = 1):
    """Uniform[-1, 1] right-hand sides, shape (ndofs, nrhs), column c drawn after column c-1."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.uniform(-1.0, 1.0, size=(nrhs, ndofs)).T)


def serving_requests(num: int = 256, seed: int = 0, sizes=(16, 24, 32, 48, 64),
                     coef_pool: int = 2, rate: float = 1.0):
    """Request stream for the serving loop: kind, n, coefficient seed, rhs seed, arrival time.

    ``rate`` is the Poisson arrival rate in requests per second.
    """
    rng = np.random.default_rng(seed)
    kinds = rng.integers(0, 2, size=num)
    ns = rng.integers(0, len(sizes), size=num)
    cseeds = rng.integers(0, coef_pool, size=num)
    gaps = rng.exponential(1.0 / rate, size=num)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for r in range(num):
        out.append(dict(id=r, kind=CURL if kinds[r] == 0 else DIV, n=int(sizes[ns[r]]),
                        coef_seed=int(cseeds[r]), rhs_seed=r, t_arrive=float(t[r])))
    return out
