// PCG state records written by the kernels and read by the host.
#pragma once

#include <stdint.h>

namespace amge {
namespace dev {

// Single-column PCG status.
struct PcgStatus {
    double delta0, delta, rr, relres, bnorm;
    double rtol;     // stopping tolerance (<= 0: exactly maxit iterations)
    int iters, done, breakdown, maxit, stop_l2;
    uint32_t epoch;  // number of the solve, tags the host records of its iterations
};

// Host-visible record of one finished single-column PCG iteration, kept in a ring of
// pinned host memory indexed by the iteration number: the status after the iteration,
// then (after a system-scope fence) tag = epoch << 32 | iteration.
constexpr int PCG_RING = 64;
struct alignas(128) PcgRecord {
    PcgStatus st;
    uint64_t tag;
};

// Per-column state of the batched PCG (written only by the single-block finalize
// kernels and by the kernels that load a column).  A column is idle (done = 1), fresh
// (just loaded: its next pass through an iteration computes z0 = B b and the initial
// quantities instead of a step) or live.
struct ColState {
    double delta0, delta, bnorm, relres, pq, rz, rzold, rr, alpha, beta;
    double rtol;      // stopping tolerance of the column (<= 0: exactly maxit iterations)
    int iters;        // PCG steps taken since the column was loaded
    int maxit;
    int stop_l2;      // 0: preconditioner norm, 1: l2 norm of the residual
    int done, fresh, pinit, breakdown, nonfinite;
};

struct BatchStatus {
    int it;          // iterations run since the last load
    int all_done;    // no fresh or live column: every kernel of an iteration returns at once
    int any_breakdown;
    int all_done_next;   // all_done after the current iteration (made current by its last kernel)
};

// One 64-row block of the l1-scaled symmetric block Gauss-Seidel layout: entry base,
// width (entries of its longest row), info = inside width (most inside entries of a
// row) | colours << 8 | shortest row length << 16 | rows << 24, base column of the
// outside 16-bit offsets.
struct alignas(16) BgsBlock {
    int base, width, info, cbase;
};

}  // namespace dev
}  // namespace amge
