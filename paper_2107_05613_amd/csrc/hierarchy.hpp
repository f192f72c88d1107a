// Device-side data of a hierarchy (shared by the solver and the serving engine).
#pragma once

#include <cstdio>

#include <hip/hip_runtime.h>

#include <memory>
#include <vector>

#include "state.hpp"
#include "common.hpp"

namespace amge {

#define HIPCHECK(expr)                                                                        \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            fail(e_ == hipErrorOutOfMemory ? AMGE_ERR_OOM : AMGE_ERR_HIP,                     \
                 std::string(#expr) + ": " + hipGetErrorString(e_));                          \
    } while (0)

// Sliced ELL matrix (64-row slices, column-major inside a slice) on the device.
struct DSell {
    int nrows = 0, ncols = 0, nslices = 0;
    int K = 1;                // lanes per row
    int64_t nnz = 0;          // stored nonzeros of the CSR input
    int64_t stored = 0;       // entries including padding
    int* sptr = nullptr;      // nslices + 1 entry offsets
    int* srow = nullptr;      // slot -> row (-1: empty slot)
    int* ci = nullptr;        // value matrices: column indices (or, when every slice's
    uint16_t* c16 = nullptr;  //   columns span < 65536: 16-bit offsets from a per-slice
    int* cbase = nullptr;     //   base column, ci = nullptr)
    uint32_t* ent = nullptr;  // incidence matrices: column | sign << 31, padding 0xffffffff
    double* v64 = nullptr;
    float* v32 = nullptr;
    uint16_t* lead = nullptr; // split rows: leading entries per slot that read the first operand
    bool stream = false;      // FP32 matrix streams read with non-temporal loads
    bool deep = false;        // long rows per lane in a large matrix: 8 entries' loads in flight
    int fixedw = 0;           // incidence with fixedw entries in every row: fent (n x fixedw
    uint32_t* fent = nullptr; //   row-major words) replaces the sliced layout
};

template <class T>
struct Work {
    T *b = nullptr, *x = nullptr, *xt = nullptr, *r = nullptr, *g = nullptr, *y = nullptr, *yt = nullptr;
    T *bd = nullptr, *gd = nullptr;   // dinv * b, dhinv * g: first sweeps from zero
    T* dinv = nullptr;
    T* dhinv = nullptr;
};

// Event timing of the fine-level A kernels (the dominant kernel family of the V-cycle).
struct Probe {
    bool on = false;
    std::vector<hipEvent_t> ev;   // start/stop pairs, reused across reads
    size_t used = 0;              // pairs recorded since the last read
    double bytes = 0;             // algorithmic bytes of the recorded launches
    ~Probe() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
};

// Sliced ELL with one lane per row (K = 1) for the batched kernels: entry t of slot rr
// of a slice at sptr[slice] + t * 64 + rr, so every row keeps its CSR entry order.
struct DSellB {
    int nrows = 0, ncols = 0, nslices = 0;
    int64_t nnz = 0;
    int* sptr = nullptr;
    int* srow = nullptr;       // slot -> row (-1: empty slot)
    int* ci = nullptr;         // value matrices: column indices, or
    uint16_t* c16 = nullptr;   //   16-bit offsets from a per-slice base column
    int* cbase = nullptr;
    uint32_t* ent = nullptr;   // incidence matrices: column | sign << 31, padding 0xffffffff
    double* v64 = nullptr;
    float* v32 = nullptr;
    uint16_t* lead = nullptr;  // split rows, as in DSell
    int V = 1;                 // columns per lane, tuned
};

// Multicolour Gauss-Seidel data of one matrix: the rows of each colour as a sliced ELL
// of their own (srow: global rows), and 1 / a_ii.
struct GsColors {
    std::vector<DSell> col;
    double* dg64 = nullptr;
    float* dg32 = nullptr;
    template <class T> const T* dg() const;
};
template <> inline const double* GsColors::dg<double>() const { return dg64; }
template <> inline const float* GsColors::dg<float>() const { return dg32; }

// l1-scaled symmetric block Gauss-Seidel data of one matrix (kernels_bgs.hpp): blocks of
// 64 consecutive rows, one wave per block, the block's rows on the lanes sorted by
// length and its entries as jagged diagonals (slab t: entry t of the rows longer than t,
// contiguous); a row's entries inside its block first (code: the column's position in
// the block), then the others (code: column, or a 16-bit offset from blk.cbase when
// every block's outside columns span < 65536).
struct DBgs {
    int n = 0, nblk = 0;
    int nin = 0;              // register bound of inside entries per row (8 ... 64)
    int64_t nnz = 0;          // entries of A
    int64_t nnz_in = 0;       // entries inside blocks (read by sweeps from zero)
    dev::BgsBlock* blk = nullptr;
    uint32_t* meta = nullptr; // per lane: inside entries | colour << 8 | length << 16 | position << 24
    int* ci = nullptr;
    uint16_t* c16 = nullptr;
    double* v64 = nullptr;
    float* v32 = nullptr;
    double *dinv64 = nullptr, *mid64 = nullptr;   // 1 / (a_ii + l1 outside), a_ii + 2 l1 outside
    float *dinv32 = nullptr, *mid32 = nullptr;
    bool on() const { return nblk > 0; }
};

struct DLevel {
    int n = 0, m = 0;
    Probe* probe = nullptr;
    // FP32 V-cycle: the residual b - A x ahead of the restriction is formed with the FP64
    // values of A, summed in FP64 and rounded to FP32 once (opts.resid_bits = 64; fine
    // level only)
    bool resid64 = false;
    GsColors gsA, gsAh;       // symmetric Gauss-Seidel smoother (opts.smoother)
    DBgs bgA, bgAh;           // l1-scaled symmetric block Gauss-Seidel smoother
    DSell A, Ah, P, Pt;
    DSell Aux;                // [D^T | -D^T A]: auxiliary residual D^T b - (D^T A) x
    DSell PtA;                // [P^T | -P^T A] below the fine level: restricted residual
    DSell D, Dt;              // signed incidences
    Work<float> w32;
    Work<double> w64;
    // batched path (max_rhs > 1): one-lane-per-row copies and n x NC work buffers of the
    // preconditioner precision
    DSellB bA, bAh, bP, bPt, bAux, bD;
    Work<float> bw32;
    Work<double> bw64;
    template <class T> Work<T>& w();
    template <class T> Work<T>& bw();
};
template <> inline Work<float>& DLevel::w<float>() { return w32; }
template <> inline Work<double>& DLevel::w<double>() { return w64; }
template <> inline Work<float>& DLevel::bw<float>() { return bw32; }
template <> inline Work<double>& DLevel::bw<double>() { return bw64; }

}  // namespace amge

// A hierarchy (amge_setup_hierarchy) holds the read-only device operators of every
// level.  A context (amge_ctx_create) is an execution state: a copy of the hierarchy's
// operator descriptors (pointing at the hierarchy's device memory) plus work buffers,
// PCG state, stream, events and captured graphs of its own, so contexts of one
// hierarchy run concurrently.  Every launch routine works on an amge_hierarchy object:
// the hierarchy itself during set-up, a context's state afterwards.
struct amge_hierarchy {
    std::vector<amge::DLevel> lv;
    amge_opts opts{};
    const amge_hierarchy* parent = nullptr;   // context state: the hierarchy it runs
    int nrhs_cap = 0;            // context state: columns its work buffers hold
    int nc = 0;                  // coarsest size
    double kappa = 1.0;          // largest cancellation factor of the auxiliary matrices
    double* Ainv = nullptr;      // coarsest inverse from the Cholesky factor
    // single-column V-cycle: levels >= tail are applied as the dense FP64 operator
    // tail_op (tail_n x tail_n): the coarsest inverse, or a folded coarse tail
    int tail = 0, tail_n = 0;
    double* tail_op = nullptr;
    int tail_rpb = 4;            // rows per block of the batched dense tail product (tuned)
    // outer PCG buffers (FP64, level-1 length)
    double *r = nullptr, *p = nullptr, *q = nullptr, *z[2] = {nullptr, nullptr}, *x = nullptr;
    double *part_pq = nullptr, *part_dots[2] = {nullptr, nullptr};
    amge::dev::PcgStatus* st = nullptr;
    int* flags = nullptr;        // [0] done, [1] breakdown, [2..3] iteration count by buffer parity
    // batched PCG (NC = columns rounded up to a power of two, columns beyond nrhs are zero)
    int NC = 1, lgNC = 0;
    double *bX = nullptr, *bR = nullptr, *bP = nullptr, *bQ = nullptr, *bZ = nullptr, *bZv = nullptr;
    double* bpart = nullptr;
    int bnblk = 0;
    amge::dev::ColState* cs = nullptr;
    amge::dev::BatchStatus* bs = nullptr;
    int* zero_flag = nullptr;    // a device 0: the stop flag of launches outside PCG iterations
    hipStream_t gstream = nullptr;   // the state's stream for graph capture / replay
    hipGraphExec_t gexec[7][2] = {}; // captured batched PCG iteration per active width 2^i and parity
    int bpar = 0;                    // parity of the next batched iteration: z block bpar is the new z
    hipGraphExec_t pexec[2] = {};    // one captured single-column PCG iteration per buffer parity
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    // single-column PCG: host ring of iteration records (pinned, written by the device)
    // and one event per queued iteration
    static constexpr int NPEV = 8;
    amge::dev::PcgRecord* ring = nullptr;     // host address
    amge::dev::PcgRecord* ring_dev = nullptr; // its device address
    uint32_t epoch = 0;
    hipEvent_t pev[NPEV] = {};
    // device memory owned by this object: from the arena if one is set (no allocation
    // at all), else from the caller's allocator (opts.alloc) or hipMalloc.  dry: only
    // count the bytes (sizing), hand out placeholder addresses that are never used.
    std::vector<void*> allocs;
    size_t bytes = 0;
    bool dry = false;
    char* arena = nullptr;
    size_t arena_size = 0, arena_used = 0;
    amge::Probe probe;
    ~amge_hierarchy() {
        if (gstream) (void)hipStreamSynchronize(gstream);
        for (auto& gw : gexec)
            for (hipGraphExec_t g : gw)
                if (g) (void)hipGraphExecDestroy(g);
        for (hipGraphExec_t g : pexec)
            if (g) (void)hipGraphExecDestroy(g);
        for (hipEvent_t e : pev)
            if (e) (void)hipEventDestroy(e);
        if (ring) (void)hipHostFree(ring);
        if (ev_in) (void)hipEventDestroy(ev_in);
        if (ev_out) (void)hipEventDestroy(ev_out);
        if (gstream) (void)hipStreamDestroy(gstream);
        if (!allocs.empty()) {
            // the caller's allocator may hand the memory out again at once: no work queued
            // on any stream may still use it
            if (opts.dealloc) (void)hipDeviceSynchronize();
            for (void* a : allocs) {
                if (opts.dealloc) opts.dealloc(a, opts.alloc_user);
                else (void)hipFree(a);
            }
        }
    }
    template <class T>
    T* alloc(size_t n) {
        if (n == 0) n = 1;
        const size_t nb = (n * sizeof(T) + 255) & ~(size_t)255;
        if (arena) {
            if (arena_used + nb > arena_size) {
                char msg[160];
                snprintf(msg, sizeof(msg), "work buffers need more than the %zu bytes of the static scratch",
                         arena_size);
                amge::fail(AMGE_ERR_ARG, msg);
            }
            T* ptr = reinterpret_cast<T*>(arena + arena_used);
            arena_used += nb;
            return ptr;
        }
        bytes += n * sizeof(T);
        if (dry) return reinterpret_cast<T*>((uintptr_t)256);
        void* ptr = nullptr;
        if (opts.alloc) {
            ptr = opts.alloc(n * sizeof(T), opts.alloc_user);
            if (!ptr) {
                bytes -= n * sizeof(T);
                char msg[160];
                snprintf(msg, sizeof(msg), "the caller's allocator returned no memory for %zu bytes", n * sizeof(T));
                amge::fail(AMGE_ERR_OOM, msg);
            }
        } else {
            hipError_t e = hipMalloc(&ptr, n * sizeof(T));
            if (e != hipSuccess) {
                size_t fr = 0, tot = 0;
                (void)hipGetLastError();
                (void)hipMemGetInfo(&fr, &tot);
                char msg[160];
                snprintf(msg, sizeof(msg), "hipMalloc of %zu bytes failed (%s; device memory free %zu of %zu bytes)",
                         n * sizeof(T), hipGetErrorString(e), fr, tot);
                bytes -= n * sizeof(T);
                amge::fail(AMGE_ERR_OOM, msg);
            }
        }
        allocs.push_back(ptr);
        return (T*)ptr;
    }
};

// A context: execution state of one hierarchy (see above).
struct amge_ctx {
    amge_hierarchy st;
};

namespace amge {
// Execution state for nrhs columns of hierarchy P (nrhs <= P's max_rhs): operator
// descriptors copied from P, work buffers, PCG state, stream, events and the pinned
// iteration ring allocated here.  dry: only sizes it (amge_footprint).
std::unique_ptr<amge_ctx> make_ctx(const amge_hierarchy* P, int nrhs, bool dry = false);
}  // namespace amge

namespace amge {
// One batched PCG iteration of parity par (z block par receives the new z) on the
// first W columns (W a power of two <= NC) of a hierarchy, captured as a HIP graph on
// its own stream on first use.  Iterations must alternate parities (H->bpar).
hipGraphExec_t capture_iteration(amge_hierarchy* H, int W, int par);

// One batched PCG iteration of parity par of every hierarchy of hs (all NC columns of each), with the
// same level operator of several hierarchies run in one grouped launch, captured as one
// graph on stream s.  Every hierarchy computes exactly what its own captured iteration
// computes.  launches / solo_launches: kernels in the graph / in the separate graphs.
hipGraphExec_t capture_grouped_iteration(const std::vector<amge_hierarchy*>& hs, int par, hipStream_t s,
                                         int* launches, int* solo_launches);
}  // namespace amge
