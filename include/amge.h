/*
 * amge.h -- C ABI of the MI355X AMGe solve phase for lowest-order H(curl) and
 * H(div) systems (element-based algebraic multigrid on an exact de Rham
 * hierarchy).
 *
 * Method (paper: Kalchev, Vassilevski, Villa, "Parallel element-based algebraic
 * multigrid for H(curl) and H(div) problems using the ParELAG library"):
 *   - the preconditioner is one V-cycle of Algorithm 4.1 with zero initial guess;
 *   - every non-coarsest level is relaxed by the hybrid smoother of eq. (4.1):
 *     l1-Jacobi sweeps on A_k, then l1-Jacobi sweeps on the auxiliary matrix
 *     D_k^T A_k D_k with the correction mapped back through D_k; the
 *     post-smoother applies the two steps in reverse order;
 *   - the coarsest level is solved exactly (dense FP64 Cholesky); the small levels
 *     just above it may be folded with it into one dense FP64 operator formed at
 *     set-up (the same linear map; opts.tail_rows);
 *   - the outer iteration is inexact PCG (section 5.1) stopped on the residual
 *     measured in the preconditioner norm.
 *
 * Conventions for every entry point
 *   - Host CSR inputs are read only during the call; the library copies them.
 *     Column indices must be sorted and in range within each row.
 *   - Device vectors are caller-owned HIP device pointers, row-major
 *     (n x nrhs): entry (i, c) is at i*nrhs + c.
 *   - `stream` is a hipStream_t (0 = the null stream).  Calls are ordered on it;
 *     functions that return host scalars synchronise it before returning.
 *   - Negative return values are errors, amge_last_error() gives a message for
 *     the calling thread.  AMGE_NOT_CONVERGED is a warning: outputs are valid.
 *   - A hierarchy (amge_setup_hierarchy) holds the level operators of Algorithm 4.1
 *     and is read-only after set-up.  The solve calls run on a context
 *     (amge_ctx_create): the work buffers, PCG state, stream and captured graphs of one
 *     caller.  Calls on one context must not overlap in time; contexts of the same
 *     hierarchy may run concurrently on different streams or threads.
 *   - Device memory of hierarchies and contexts comes from the caller's allocator
 *     (amge_opts.alloc) when one is given, else from hipMalloc.
 */
#ifndef AMGE_H
#define AMGE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AMGE_OK = 0,
    AMGE_NOT_CONVERGED = 1,
    AMGE_CANCELLED = 2,       /* serving: the request was cancelled (amge_server_cancel)  */
    AMGE_ERR_ARG = -1,        /* invalid argument (null pointer, bad size, bad option)   */
    AMGE_ERR_SHAPE = -2,      /* matrix dimensions do not chain, indices out of range    */
    AMGE_ERR_NOT_SPD = -3,    /* coarsest matrix not symmetric positive definite         */
    AMGE_ERR_OOM = -4,        /* device or host allocation failed                        */
    AMGE_ERR_HIP = -5,        /* a HIP runtime call failed                               */
    AMGE_ERR_BREAKDOWN = -6,  /* PCG breakdown: p.q <= 0 or preconditioner not positive  */
    AMGE_ERR_NONFINITE = -7,  /* NaN or Inf in an input                                  */
    AMGE_ERR_BUSY = -8        /* resource budget exceeded (serving admission)            */
} amge_status;

enum { AMGE_CURL = 0, AMGE_DIV = 1 };

/* Host CSR matrix, FP64 values, int32 indices. */
typedef struct {
    int32_t nrows, ncols;
    int64_t nnz;
    const int32_t* rowptr;   /* nrows + 1 */
    const int32_t* col;      /* nnz, sorted within each row */
    const double* val;       /* nnz */
} amge_csr;

/* One level k of the hierarchy (Algorithm 4.1 inputs, section 3.2):
 *   A  n_k x n_k    system matrix A_k (SPD); A_1 is the fine matrix, A_{k+1} = P_k^T A_k P_k
 *   D  n_k x m_k    exterior derivative used by the hybrid smoother (eq. (4.1)):
 *                   discrete gradient (H(curl)) or discrete curl (H(div)); entries +-1
 *   P  n_k x n_{k+1} prolongator to the next level (section 3.2.1); nrows = 0 on the
 *                   coarsest level. */
typedef struct {
    amge_csr A, D, P;
} amge_level;

typedef struct {
    int32_t nu_primary;     /* point-smoother sweeps on A_k per smoothing step (paper: 2)   */
    int32_t nu_aux;         /* point-smoother sweeps on D^T A D per smoothing step (paper: 2) */
    int32_t precond_bits;   /* 64: V-cycle in FP64; 32: FP32 values/accumulation in the
                               V-cycle with the coarsest Cholesky solve kept in FP64;
                               0: chosen at set-up by trial PCG solves on a fixed
                               pseudo-random right-hand side to rtol 1e-8: FP32 (with the
                               first resid_bits that works, 32 then 64) if it converges
                               within 3 iterations of the FP64 V-cycle, else FP64            */
    int32_t max_rhs;        /* largest nrhs of a context of this hierarchy (1 <= max_rhs <= 64);
                               > 1 also builds the batched operators                        */
    int32_t tail_rows;      /* coarse-tail folding: while the level above the coarse tail
                               (initially the coarsest level) is not the fine level and has
                               at most tail_rows rows, the V-cycle from that level down (a
                               fixed linear map: zero initial guess) is formed at set-up in
                               FP64, one unit vector at a time, and applied in every V-cycle
                               (single-column and batched) as one dense FP64 product.  Same
                               operator, fewer launches.  0: off (0 <= tail_rows <= 8192). */
    int32_t smoother;       /* point smoother of the hybrid smoother (section 4.1):
                               AMGE_SMOOTHER_L1_JACOBI: x += d^{-1}(b - A x), d_i = sum_j |a_ij|;
                               AMGE_SMOOTHER_SYM_GS: symmetric Gauss-Seidel in colour order:
                               rows coloured greedily (first fit in increasing row order over
                               the rows coupled to earlier ones), a sweep relaxes the colours
                               in increasing then decreasing order, each row by
                               x_i += (b - A x)_i / a_ii;
                               AMGE_SMOOTHER_BLOCK_GS: l1-scaled symmetric block Gauss-Seidel
                               (the smoother of the paper's experiments, section 4.1 last
                               paragraph and section 5.1, with blocks of 64 consecutive rows
                               in place of processors): inside a block, rows coloured greedily
                               over the couplings within the block and relaxed colour by
                               colour, forward then backward through all colours, each row by
                               x_i += (b_i - sum_j a_ij x_j) / d_i, d_i = a_ii + sum of |a_ij|
                               over columns outside the block, where x_j outside the block
                               keeps its value from the start of the sweep.
                               The Gauss-Seidel smoothers need a positive diagonal
                               (AMGE_ERR_NOT_SPD otherwise), the block one rows of at most
                               255 entries (AMGE_ERR_SHAPE otherwise); the colour-order one
                               runs single-column contexts only (max_rhs = 1), the block one
                               also the batched path (every column through the arithmetic of
                               the single-column sweep).                                      */
    int32_t resid_bits;     /* FP32 V-cycles: precision of the fine-level residual b - A x that
                               is restricted to level 2 (Algorithm 4.1).  32: FP32 values and
                               sums; 64: the FP64 values of A_1 summed in FP64, the result
                               rounded to FP32 once (one FP64-value pass over A_1 per V-cycle
                               instead of an FP32 one).  On high-contrast coefficients the
                               FP32 residual loses the small mass part of A x near the range
                               of D (see amge_precision_info); the FP64 one keeps the FP32
                               V-cycle converging like the FP64 one.  0: 32, or chosen by the
                               trial when precond_bits = 0.  Ignored for FP64 V-cycles.      */
    /* Caller's device allocator (both NULL: hipMalloc / hipFree).  alloc(bytes, user)
     * returns device memory of at least `bytes` bytes, 256-byte aligned, or NULL (the
     * call then fails with AMGE_ERR_OOM); dealloc(ptr, user) returns it.  The library
     * calls them from the thread that calls it, during amge_setup_hierarchy (operators),
     * amge_ctx_create (work buffers), the first amge_level_apply of a precision other
     * than the V-cycle's, and the destroy calls (after a device-wide synchronisation, so
     * no queued work still uses the memory).  The hierarchy's contexts use the same
     * allocator. */
    void* (*alloc)(size_t bytes, void* user);
    void (*dealloc)(void* ptr, void* user);
    void* alloc_user;
} amge_opts;

typedef struct amge_hierarchy amge_hierarchy;
typedef struct amge_ctx amge_ctx;

enum { AMGE_SMOOTHER_L1_JACOBI = 0, AMGE_SMOOTHER_SYM_GS = 1, AMGE_SMOOTHER_BLOCK_GS = 2 };

/* Default options: nu = 2 + 2, FP32 preconditioner, max_rhs = 1, tail_rows = 2048,
 * l1-Jacobi, hipMalloc. */
void amge_default_opts(amge_opts* opts);

/* Builds the device hierarchy from host level matrices (section 3.2, Algorithm 4.1 inputs).
 * Host work: validation, D^T, P^T, the products D^T A and D^T A D, and P^T A below the
 * fine level (FP64 sparse products; the auxiliary residual D^T (b - A x) is evaluated as
 * D^T b - (D^T A) x, and below the fine level the restricted residual P^T (b - A x) as
 * P^T b - (P^T A) x), the l1 row sums, the cancellation factor, a dense FP64 Cholesky
 * factor of the coarsest matrix and the inverse it gives (coarsest level at most 8192
 * rows), and the folded coarse tail (tail_rows).  The device layouts are tuned
 * by timing candidate launches on `stream`.  The hierarchy owns the device operators
 * (allocated through opts.alloc when given) and holds no work buffers.
 * Errors: AMGE_ERR_ARG, AMGE_ERR_SHAPE, AMGE_ERR_NONFINITE (NaN/Inf value),
 * AMGE_ERR_NOT_SPD (coarsest matrix not symmetric positive definite, or a zero row),
 * AMGE_ERR_OOM, AMGE_ERR_HIP. */
amge_status amge_setup_hierarchy(const amge_level* levels, int32_t nlevels, const amge_opts* opts,
                                 void* stream, amge_hierarchy** out);

/* Destroys a hierarchy; its contexts must be destroyed first. */
void amge_destroy(amge_hierarchy* h);

/* Context for up to nrhs columns (1 <= nrhs <= opts.max_rhs of h): per-level work
 * vectors of the V-cycle precision, the outer PCG vectors and partial sums (FP64), with
 * nrhs > 1 also the n x NC batched blocks (NC = nrhs rounded up to a power of two), a
 * stream for the captured PCG iterations, events and a pinned host ring of iteration
 * records.  The Algorithm 4.1 inputs themselves stay in h, shared by all its contexts.
 * Errors: AMGE_ERR_ARG (nrhs out of range), AMGE_ERR_OOM, AMGE_ERR_HIP. */
amge_status amge_ctx_create(const amge_hierarchy* h, int32_t nrhs, amge_ctx** out);
/* Waits for the device, then frees the context's buffers (NULL: no-op). */
void amge_ctx_destroy(amge_ctx* c);

/* Device memory of the hierarchy's operators (hier_bytes) and of one context for nrhs
 * columns (ctx_bytes: what amge_ctx_create(h, nrhs) allocates, not counting a level
 * work set that amge_level_apply may add).  Either output may be NULL; nrhs is checked
 * only when ctx_bytes is requested. */
amge_status amge_footprint(const amge_hierarchy* h, int32_t nrhs, size_t* hier_bytes, size_t* ctx_bytes);

/* z = B r: one V-cycle of Algorithm 4.1 with zero initial guess, on nrhs columns.
 * r, z: device FP64, n_1 x nrhs row-major.  1 <= nrhs <= the context's nrhs; nrhs > 1
 * runs the batched kernels (one launch per level operator for all columns).
 * Asynchronous on `stream`. */
amge_status amge_vcycle(amge_ctx* c, const double* r, double* z, int32_t nrhs, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): z = B r on one column, exactly the
 * computation of amge_vcycle with nrhs = 1, with the level work vectors taken from a
 * static device scratch array of AMGE_STATIC_SCRATCH_BYTES per GPU (held from the
 * first call on a device until the process ends) instead of a context.  The call
 * allocates nothing.  r, z: device FP64, n_1 entries, caller-owned.  Asynchronous on
 * `stream`.  All calls on one GPU share its scratch, whose contents the next call
 * overwrites: calls that overlap in time on one GPU (other streams or threads) race.
 * Errors: AMGE_ERR_ARG if the hierarchy's single-column work vectors (sum over the
 * levels of 5 n_k + 4 m_k values of the V-cycle precision, each vector rounded up to
 * 256 bytes) exceed the scratch; AMGE_ERR_HIP. */
#define AMGE_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
amge_status amge_vcycle_static(const amge_hierarchy* h, const double* r, double* z, void* stream);

/* Inexact PCG (section 5.1) for A_1 x = b with x0 = 0 and one V-cycle per iteration.
 *   b, x     device FP64, n_1 x nrhs row-major; x is overwritten
 *   nrhs     1 <= nrhs <= the context's nrhs; every column follows its own recurrences and
 *            stopping test (nrhs > 1: batched kernels, a column that has stopped keeps
 *            its iterate while the others go on)
 *   rtol     stop when sqrt(r.z / r0.z0) <= rtol (stop_norm = 0, preconditioner norm) or
 *            ||r|| / ||b|| <= rtol (stop_norm = 1); rtol <= 0 runs exactly maxit iterations
 *   iters    host, nrhs entries: PCG steps per column (0 for a zero right-hand side)
 *   relres   host, nrhs entries: final relative residual in the chosen norm
 * The iterations run as replays of a HIP graph captured on the context's own stream
 * (ordered after `stream` and before later work on it by events); the call returns after
 * the solve.  Returns AMGE_NOT_CONVERGED if a column missed rtol within maxit,
 * AMGE_ERR_NONFINITE for a NaN/Inf right-hand side (nrhs > 1: in any column; the other
 * columns are still solved and written), AMGE_ERR_BREAKDOWN if p.q <= 0 or r.z <= 0
 * occurs. */
amge_status amge_pcg_solve(amge_ctx* c, const double* b, double* x, int32_t nrhs, double rtol,
                           int32_t maxit, int32_t stop_norm, int32_t* iters, double* relres, void* stream);

/* Single level operations, for testing each kernel of the path on its own.  Device FP64
 * in/out vectors (one column); precision 32 runs the FP32 kernel on rounded inputs
 * (temporary buffers; the first call in the precision other than the V-cycle's adds
 * that precision's level work set to the context).
 *   op  AMGE_OP_A       out = A_k in                 (sparse product)
 *       AMGE_OP_AHAT    out = (D^T A D)_k in          (auxiliary matrix)
 *       AMGE_OP_D       out = D_k in                  (incidence)
 *       AMGE_OP_DT      out = D_k^T in
 *       AMGE_OP_P       out = P_k in                  (prolongation, in has n_{k+1} rows)
 *       AMGE_OP_PT      out = P_k^T in                (restriction)
 *       AMGE_OP_SMOOTH  out = x + Mbar^{-1}(b - A x) with b = in, x = in2 (eq. (4.1))
 *       AMGE_OP_SMOOTHT out = x + Mbar^{-T}(b - A x) with b = in, x = in2 (reversed order)
 *       AMGE_OP_COARSE  out = A_L^{-1} in on the coarsest level (Cholesky apply)
 *       AMGE_OP_SWEEP   one sweep of the V-cycle's point smoother on A_k from x, b = in,
 *                       x = in2 (its sweep kernel): with the block Gauss-Seidel smoother
 *                       one symmetric block sweep, otherwise the l1-Jacobi sweep
 *                       out = x + d^{-1} (b - A x), d_i = sum_j |a_ij| (eq. (4.1))
 *       AMGE_OP_RESID   out = b - A x, b = in, x = in2 (the V-cycle's residual kernel,
 *                       Algorithm 4.1: with the block Gauss-Seidel smoother the kernel on
 *                       the smoother's layout of A; on the fine level at precision 32 with
 *                       resid_bits = 64 in use, FP64 values with FP64 sums)
 * On the fine level, SWEEP and RESID run exactly the launches the V-cycle times with
 * amge_timing_enable. */
enum {
    AMGE_OP_A = 0, AMGE_OP_AHAT = 1, AMGE_OP_D = 2, AMGE_OP_DT = 3, AMGE_OP_P = 4,
    AMGE_OP_PT = 5, AMGE_OP_SMOOTH = 6, AMGE_OP_SMOOTHT = 7, AMGE_OP_COARSE = 8,
    AMGE_OP_SWEEP = 9, AMGE_OP_RESID = 10
};
amge_status amge_level_apply(amge_ctx* c, int32_t level, int32_t op, int32_t precision,
                             const double* in, const double* in2, double* out, void* stream);

/* Event timing of the fine-level A_1 kernels of the V-cycle (the point smoother's sweeps
 * on A_1 and the residuals on level 1, the dominant kernel family of the path).  While enabled, every
 * such launch is bracketed by HIP events on its own stream.  amge_timing_read waits for
 * the recorded events and returns, since enabling or the previous read: the summed
 * kernel time in ms, the number of launches, and their algorithmic bytes (values and
 * column indices, row pointers, and each vector stream once).  Intended for measurement
 * runs; reading resets the counters. */
amge_status amge_timing_enable(amge_ctx* c, int32_t enable);
amge_status amge_timing_read(amge_ctx* c, double* ms, int64_t* launches, double* bytes);

/* Algorithmic bytes of one V-cycle on nrhs columns (1 <= nrhs <= opts.max_rhs) in the given
 * precision (32 or 64): every matrix of every level read once per use (values + column
 * indices + row pointers, incidences index-only; the batched path reads each matrix
 * once for all columns), every vector stream once per column, the l1 scalings once,
 * and the coarsest inverse. */
amge_status amge_vcycle_bytes(const amge_hierarchy* h, int32_t precision, int32_t nrhs, double* bytes);

/* Cancellation factor kappa = max over levels and rows e of (|D|^T |A| |D| 1)_e /
 * (|D^T A D| 1)_e (D^T A D keeps only the mass part of A, so products of A with vectors
 * near the range of D cancel up to this factor; their rounding error is ~ u * kappa
 * relative), the preconditioner precision in use (32 or 64) and, for an FP32 V-cycle,
 * the precision of its fine-level residual (32 or 64; 64 for an FP64 V-cycle).  Any
 * pointer may be NULL. */
amge_status amge_precision_info(const amge_hierarchy* h, double* kappa, int32_t* precond_bits,
                                int32_t* resid_bits);

/* Host sizes of a hierarchy: nlevels, and rows of A_k for k = 0..nlevels-1 (rows[] may be NULL). */
amge_status amge_hierarchy_info(const amge_hierarchy* h, int32_t* nlevels, int32_t* rows);

const char* amge_last_error(void);

/* ------------------------------------------------------------------------------------
 * Serving engine: many resident hierarchies and a stream of single right-hand-side
 * solve requests (inexact PCG of section 5.1 with one V-cycle per step, x0 = 0).
 * The hierarchies are reused across many right-hand sides, the regime where the setup
 * cost of the method pays off (section 5).
 *
 * Every hierarchy added to a server gets a context of the server's own (max_rhs columns)
 * and runs the batched PCG on its stream, one column per request (or, added with amge_server_add_grouped, together with the other members
 * of its ensemble in grouped launches).  Between chunks of iterations a request is
 * loaded into a free column of its hierarchy while the other columns stay in flight
 * (continuous batching), and the hierarchies advance concurrently on the device.  The
 * arithmetic of a column does not depend on the other columns, so a request's result is
 * the same alone and in a mix.
 *
 * Admission by device memory:
 *   hierarchy_budget  bytes; amge_server_add fails with AMGE_ERR_BUSY if the sum of the
 *                     footprints of the added hierarchies and of their server contexts
 *                     (amge_footprint with nrhs = max_rhs) would exceed it (0 = no limit)
 *   inflight_budget   bytes; a request is admitted only while the work footprint of all
 *                     admitted requests (amge_server_request_bytes each: its column of
 *                     the work blocks) stays within it (0 = no limit); requests are
 *                     admitted in submission order, a request that does not fit waits
 *                     and holds back those behind it, one whose hierarchy has no free
 *                     column does not
 *   chunk             at most this many PCG iterations per hierarchy between two looks at
 *                     its columns (fewer on large hierarchies: chunks are sized to about
 *                     2 ms of estimated GPU time, and chunks of different hierarchies are
 *                     started in turn while the estimated queued GPU time stays under 8 ms)
 *
 * Single-threaded: calls on one server must not overlap.  A hierarchy added to a
 * server needs max_rhs >= 2 (its max_rhs is the number of columns); it stays usable
 * through other contexts.  amge_server_destroy waits for the server's work and frees
 * its contexts; the hierarchies outlive the server and are destroyed by the caller.
 * ---------------------------------------------------------------------------------- */
typedef struct amge_server amge_server;

typedef struct {
    int64_t tag;         /* the caller's request id                                        */
    int32_t hierarchy;   /* id from amge_server_add                                         */
    int32_t status;      /* AMGE_OK, AMGE_NOT_CONVERGED, AMGE_CANCELLED, AMGE_ERR_BREAKDOWN,
                            AMGE_ERR_NONFINITE                                               */
    int32_t iters;       /* PCG steps                                                       */
    int32_t pad;
    double relres;       /* final relative residual in the chosen norm                      */
} amge_completion;

amge_status amge_server_create(size_t hierarchy_budget, size_t inflight_budget, int32_t chunk,
                               amge_server** out);
void amge_server_destroy(amge_server* s);
/* Makes h resident in the server; *id numbers the hierarchies 0, 1, ...
 * Errors: AMGE_ERR_ARG (max_rhs < 2, added twice), AMGE_ERR_BUSY (budget). */
amge_status amge_server_add(amge_server* s, amge_hierarchy* h, int32_t* id);
/* Like amge_server_add, but h joins ensemble number `ensemble` (0 <= ensemble < 16) of
 * the server: one PCG iteration of every hierarchy of an ensemble runs as a single
 * captured graph in which the same level operator of several hierarchies is one grouped
 * launch (each workgroup of a grouped launch works for one member, with that member's
 * operands), so hierarchies whose iterations are chains of short, latency-bound launches
 * (small problems) share their launches.  An ensemble advances all its members
 * together, on all their columns, on one stream of its own (different ensembles and
 * solo hierarchies advance concurrently); it is recaptured at its next chunk after a
 * member joins.  A request's result is bitwise the same as on a hierarchy added with
 * amge_server_add.  Errors as amge_server_add; AMGE_ERR_ARG for an ensemble number out
 * of range. */
amge_status amge_server_add_grouped(amge_server* s, amge_hierarchy* h, int32_t ensemble, int32_t* id);
/* The ensembles, summed: number of members, kernels in their captured iterations, and
 * kernels the members' iterations take when captured one by one (an ensemble counts 0
 * before its first chunk). */
amge_status amge_server_ensemble(const amge_server* s, int32_t* members, int32_t* launches,
                                 int32_t* solo_launches);
/* Work footprint of one request on hierarchy id, in bytes. */
amge_status amge_server_request_bytes(const amge_server* s, int32_t id, size_t* bytes);
/* Queues the solve A_1 x = b on hierarchy id.  b, x: device FP64, n_1 entries each,
 * caller-owned; b is read after the work already queued on `stream` (an event is
 * recorded there) and must stay valid, and x untouched, until the request's completion
 * is returned.  rtol, maxit, stop_norm as for amge_pcg_solve.  Errors: AMGE_ERR_ARG,
 * AMGE_ERR_BUSY (the request alone exceeds the in-flight budget). */
amge_status amge_server_submit(amge_server* s, int32_t id, const double* b, double* x, double rtol,
                               int32_t maxit, int32_t stop_norm, int64_t tag, void* stream);
/* Advances the server: looks at every hierarchy whose chunk has finished, copies
 * finished requests out, admits queued requests into free columns and starts the next
 * chunks.  With wait != 0 it returns once at least one request has completed or
 * nothing is left to do; with wait = 0 after one pass.  Up to cap completions are
 * written to out (*nout of them); x of a returned request is final. */
amge_status amge_server_progress(amge_server* s, int32_t wait, amge_completion* out, int32_t cap,
                                 int32_t* nout);
/* Cancels every request with this tag that has not finished: a queued one is removed,
 * an in-flight one leaves its column when the chunk of iterations it is in ends (at
 * once if none is running), and the column goes back to the pool.  Each cancelled
 * request is still returned by amge_server_progress, once, with status AMGE_CANCELLED
 * (iters / relres: its state at the last chunk boundary); its x is not written after the
 * call and b is no longer read once that completion is returned.  A request whose
 * solution is already being copied out is not cancelled (its completion is the real
 * one).  *count (may be NULL): the number of requests cancelled.  Errors: AMGE_ERR_ARG. */
amge_status amge_server_cancel(amge_server* s, int64_t tag, int32_t* count);
/* Queued and in-flight request counts, in-flight work bytes and resident hierarchy bytes
 * (any pointer may be NULL). */
amge_status amge_server_stats(const amge_server* s, int32_t* queued, int32_t* inflight,
                              size_t* inflight_bytes, size_t* resident_bytes);

/* ------------------------------------------------------------------------------------
 * Problem builder for the structured workloads: the unit cube split into n^3 hexes,
 * 6 Kuhn tetrahedra each; lowest-order Nedelec (kind AMGE_CURL) or Raviart-Thomas
 * (AMGE_DIV) discretisation of a(u,v) = (alpha Du, Dv) + (beta u, v) (eq. (2.2)), natural
 * boundary conditions; hierarchy by 2x2x2 agglomeration of the hexes on every level,
 * PV traces (eq. (3.5)) and minimum-mass extensions (eqs. (3.6), (3.8)), Galerkin
 * coarse matrices.  Dofs are numbered canonically: entities sorted lexicographically by
 * their sorted vertex indices, vertex (i,j,k) = i + (n+1)(j + (n+1)k).
 *   alpha_hex, beta_hex  host, n^3 values, hex (i,j,k) at i + n(j + n k)
 *   nlevels              >= 1; n must be divisible by 2^(nlevels-1)
 *   flags                0, or a combination of
 *       AMGE_BUILD_COEFFICIENT  coefficient-aware extensions (the remark closing section
 *                               3.3): the local minimum-mass problems weight the system
 *                               space's element masses by beta and the next space's (RT
 *                               for H(curl)) by alpha; face trace masses stay unweighted
 *       AMGE_BUILD_ESSENTIAL    homogeneous essential boundary conditions (section 5.1's
 *                               benchmark): every level keeps only the dofs off the boundary
 *                               of the cube (rows/columns of A, rows of D and P, columns
 *                               of P and of D restricted alike), renumbered in order
 *       AMGE_BUILD_DEVICE       set-up work on the current GPU (section 5.2.1: the local
 *                               extensions are embarrassingly parallel): the weighted local
 *                               problems of the first agglomeration step, one workgroup per
 *                               agglomerate whose hexes carry different weights (with
 *                               AMGE_BUILD_COEFFICIENT; unweighted agglomerates share the
 *                               reference solution on either path)
 * The returned problem owns host CSR arrays for every level (amge_level layout).
 * ---------------------------------------------------------------------------------- */
typedef struct amge_problem amge_problem;

enum { AMGE_BUILD_ESSENTIAL = 1, AMGE_BUILD_COEFFICIENT = 2, AMGE_BUILD_DEVICE = 4 };
amge_status amge_kuhn_build(int32_t kind, int32_t n, int32_t nlevels, const double* alpha_hex,
                            const double* beta_hex, int32_t flags, amge_problem** out);
int32_t amge_problem_nlevels(const amge_problem* p);
/* Fills levels[0..nlevels-1] with pointers into p (valid until amge_problem_free). */
amge_status amge_problem_levels(const amge_problem* p, amge_level* levels);
void amge_problem_free(amge_problem* p);

#ifdef __cplusplus
}
#endif

#endif /* AMGE_H */
