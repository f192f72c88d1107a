// Set-up, V-cycle and PCG drivers, and the C ABI of the solve phase.
//
// Algorithm 4.1 (V-cycle) with the hybrid smoother of eq. (4.1) on every
// non-coarsest level and an exact FP64 Cholesky solve on the coarsest one; inexact
// PCG of section 5.1 around it.  The host only orchestrates launches; every vector
// operation of the path runs in the kernels of kernels.hpp.
#include <hip/hip_runtime.h>

#include <atomic>
#include <exception>
#include <chrono>
#include <cmath>
#include <cstring>
#include <cstdlib>
#include <memory>
#include <map>
#include <mutex>
#include <numeric>
#include <thread>
#include <tuple>
#include <type_traits>

#include "block_gs.hpp"
#include "common.hpp"
#include "hierarchy.hpp"
#include "kernels.hpp"
#include "kernels_batched.hpp"
#include "sell_layout.hpp"
#include "spgemm_device.hpp"


namespace amge {

using dev::BLOCK;
using dev::WAVES;

template <class T>
T* upload(amge_hierarchy* H, const T* src, size_t n, hipStream_t s) {
    T* d = H->alloc<T>(n);
    if (n) HIPCHECK(hipMemcpyAsync(d, src, n * sizeof(T), hipMemcpyHostToDevice, s));
    return d;
}

// A host CSR matrix copied to the device once, for the layout kernels of set-up (every
// candidate layout of the tuner and the final one are filled from it); the copy lives
// in its own allocation owner (the caller's allocator, if any) and goes with it.
struct Staged {
    amge_hierarchy mem;
    const Csr* A = nullptr;
    int32_t *rowptr = nullptr, *col = nullptr;
    double* val = nullptr;
    int* flag = nullptr;
};

std::unique_ptr<Staged> stage(const amge_opts& opts, const Csr& A, hipStream_t s) {
    auto st = std::make_unique<Staged>();
    st->mem.opts = opts;
    st->A = &A;
    st->rowptr = upload(&st->mem, A.rowptr.data(), A.rowptr.size(), s);
    st->col = upload(&st->mem, A.col.data(), A.col.size(), s);
    st->val = upload(&st->mem, A.val.data(), A.val.size(), s);
    st->flag = st->mem.alloc<int>(1);
    return st;
}

// Entry arrays of layout h (its row part) on the device from the staged matrix; srow
// is the layout's own slot -> row map (rows of st->A).  Value matrices: c16 + cbase when
// every slice spans < 65536 columns (and compact indices are on), else ci; v64 / v32 as
// requested.  Incidence matrices: ent.
struct DevEntries {
    int *ci = nullptr, *cbase = nullptr;
    uint16_t* c16 = nullptr;
    uint32_t* ent = nullptr;
    double* v64 = nullptr;
    float* v32 = nullptr;
};

DevEntries fill_entries(amge_hierarchy* H, const Staged& st, const HostSell& h, const int* d_sptr, bool incidence,
                        bool f32, bool f64, hipStream_t s) {
    DevEntries e;
    const size_t stored = h.sptr[h.nslices];
    const int ns = h.nslices;
    amge_hierarchy tmp;
    tmp.opts = H->opts;
    const int* srow = upload(&tmp, h.srow.data(), h.srow.size(), s);
    const unsigned grid = (unsigned)((ns + dev::WAVES - 1) / dev::WAVES);
    int flag = 0;
    HIPCHECK(hipMemsetAsync(st.flag, 0, sizeof(int), s));
    if (incidence) {
        e.ent = H->alloc<uint32_t>(stored);
        if (grid)
            dev::k_sell_fill<true><<<grid, dev::BLOCK, 0, s>>>(ns, h.K, d_sptr, srow, st.rowptr, st.col, st.val,
                                                                nullptr, nullptr, nullptr, nullptr, nullptr, e.ent,
                                                                st.flag);
        HIPCHECK(hipGetLastError());
        HIPCHECK(hipMemcpyAsync(&flag, st.flag, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHECK(hipStreamSynchronize(s));
        if (flag) fail(AMGE_ERR_ARG, "derivative matrix entries must be +-1");
        return e;
    }
    int* cb = tmp.alloc<int>(ns);
    if (grid)
        dev::k_slice_range<<<grid, dev::BLOCK, 0, s>>>(ns, h.K, srow, st.rowptr, st.col, cb, st.flag);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipMemcpyAsync(&flag, st.flag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    if (!flag && compact_indices()) {
        e.cbase = H->alloc<int>(ns);
        HIPCHECK(hipMemcpyAsync(e.cbase, cb, sizeof(int) * std::max(ns, 1), hipMemcpyDeviceToDevice, s));
        e.c16 = H->alloc<uint16_t>(stored);
    } else {
        e.ci = H->alloc<int>(stored);
    }
    if (f64) e.v64 = H->alloc<double>(stored);
    if (f32) e.v32 = H->alloc<float>(stored);
    if (grid)
        dev::k_sell_fill<false><<<grid, dev::BLOCK, 0, s>>>(ns, h.K, d_sptr, srow, st.rowptr, st.col, st.val, e.cbase,
                                                             e.ci, e.c16, e.v64, e.v32, nullptr, st.flag);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(s));   // tmp's buffers are freed on return
    return e;
}

// rowmap (optional): global row of each row of A (A holds a subset of a matrix's rows).
// st (optional): A staged on the device; staged here when absent.
DSell upload_sell(amge_hierarchy* H, const Csr& A, bool incidence, int K, hipStream_t s,
                  const std::vector<int>* lead = nullptr, const std::vector<int>* rowmap = nullptr,
                  const Staged* st = nullptr) {
    const bool on_dev = device_layouts();
    HostSell h = on_dev ? sell_rows(A, K, lead) : make_sell(A, incidence, K, lead);
    const std::vector<int> local_srow = rowmap && on_dev ? h.srow : std::vector<int>();
    if (rowmap)
        for (int& r : h.srow)
            if (r >= 0) r = (*rowmap)[r];
    DSell d;
    d.nrows = A.nrows;
    d.ncols = A.ncols;
    d.nnz = A.nnz();
    d.K = K;
    d.nslices = h.nslices;
    d.stored = h.sptr[h.nslices];
    // long rows for their lanes (>= 12 entries per lane) in a large matrix (>= 2^23
    // entries): eight entries' loads in flight per lane.  Measured on the 64^3 H(curl)
    // hierarchy: fine A_k (one lane per row) FP32 sweep 40.8 -> 38.4 us, FP64 83.5 -> 77.9
    // us; adding the level-1 auxiliary and restriction matrices (4 and 8 lanes per row)
    // FP32 solve 12.53 -> 12.38 ms.  Four stay better for short rows and small levels.
    d.deep = !incidence && K <= 8 && A.nnz() >= (1 << 23) && A.nnz() >= 12 * (int64_t)K * A.nrows;
    d.sptr = upload(H, h.sptr.data(), h.sptr.size(), s);
    d.srow = upload(H, h.srow.data(), h.srow.size(), s);
    if (!incidence && lead) d.lead = upload(H, h.lead.data(), h.lead.size(), s);
    if (on_dev) {
        std::unique_ptr<Staged> own;
        if (!st) {
            own = stage(H->opts, A, s);
            st = own.get();
        }
        HostSell rows;   // the fill kernels read rows of A: the unmapped slot map
        rows.K = K;
        rows.nslices = h.nslices;
        rows.sptr = std::move(h.sptr);
        rows.srow = rowmap ? local_srow : std::move(h.srow);
        const DevEntries e = fill_entries(H, *st, rows, d.sptr, incidence, true, true, s);
        d.ent = e.ent;
        d.ci = e.ci;
        d.c16 = e.c16;
        d.cbase = e.cbase;
        d.v64 = e.v64;
        d.v32 = e.v32;
        return d;
    }
    if (incidence) {
        d.ent = upload(H, h.ent.data(), h.ent.size(), s);
    } else {
        if (h.compact && compact_indices()) {
            d.c16 = upload(H, h.c16.data(), h.c16.size(), s);
            d.cbase = upload(H, h.cbase.data(), h.cbase.size(), s);
        } else {
            d.ci = upload(H, h.ci.data(), h.ci.size(), s);
        }
        d.v64 = upload(H, h.val.data(), h.val.size(), s);
        std::vector<float> v32(h.val.begin(), h.val.end());   // round to nearest
        d.v32 = upload(H, v32.data(), v32.size(), s);
    }
    HIPCHECK(hipStreamSynchronize(s));
    return d;
}

// ------------------------------------------------------------------ launches
inline unsigned grid_for(int64_t threads) { return (unsigned)((threads + BLOCK - 1) / BLOCK); }
inline unsigned grid_slices(int ns) { return (unsigned)((ns + WAVES - 1) / WAVES); }

template <class T> const T* vals(const DSell& M);
template <> const float* vals<float>(const DSell& M) { return M.v32; }
template <> const double* vals<double>(const DSell& M) { return M.v64; }

template <class T, int K, int UNR>
void sell_ku(const DSell& M, int mode, const T* x, const T* b, const T* dinv, T* y, T* yd, hipStream_t s,
             const int* stop) {
    unsigned g = grid_slices(M.nslices);
    if (g == 0) return;
    const T* v = vals<T>(M);
#define AMGE_SELL(MODE, C16, NT)                                                                         \
    dev::k_sell<T, K, MODE, C16, NT, UNR><<<g, BLOCK, 0, s>>>(M.nslices, M.sptr, M.srow, M.ci, M.c16, M.cbase, v, \
                                                              x, b, dinv, y, yd, M.lead, stop)
#define AMGE_SELL_MODES(C16, NT)                                    \
    switch (mode) {                                                 \
        case dev::SPMV: AMGE_SELL(dev::SPMV, C16, NT); break;       \
        case dev::SPMV_ADD: AMGE_SELL(dev::SPMV_ADD, C16, NT); break; \
        case dev::RESID: AMGE_SELL(dev::RESID, C16, NT); break;     \
        case dev::JAC: AMGE_SELL(dev::JAC, C16, NT); break;         \
        default: AMGE_SELL(dev::SPLIT, C16, NT); break;             \
    }
    if (M.c16) {
        if (M.stream) AMGE_SELL_MODES(true, true) else AMGE_SELL_MODES(true, false)
    } else {
        if (M.stream) AMGE_SELL_MODES(false, true) else AMGE_SELL_MODES(false, false)
    }
#undef AMGE_SELL_MODES
#undef AMGE_SELL
}

template <class T, int K>
void sell_k(const DSell& M, int mode, const T* x, const T* b, const T* dinv, T* y, T* yd, hipStream_t s,
            const int* stop) {
    if constexpr (K <= 8) {
        if (M.deep) {
            sell_ku<T, K, 8>(M, mode, x, b, dinv, y, yd, s, stop);
            return;
        }
    }
    sell_ku<T, K, 4>(M, mode, x, b, dinv, y, yd, s, stop);
}

// mode as in dev::Mode (SPLIT needs a matrix with split rows); yd (SPMV, SPLIT) receives
// dinv * y when non-null.  stop: device flag, the launch does nothing while it is set
// (PCG iterations after convergence).
template <class T>
void sell(const DSell& M, int mode, const T* x, const T* b, const T* dinv, T* y, hipStream_t s, const int* stop,
          T* yd = nullptr) {
    if (mode == dev::SPLIT && !M.lead) fail(AMGE_ERR_ARG, "split product on a matrix without split rows");
    switch (M.K) {
        case 1: sell_k<T, 1>(M, mode, x, b, dinv, y, yd, s, stop); break;
        case 2: sell_k<T, 2>(M, mode, x, b, dinv, y, yd, s, stop); break;
        case 4: sell_k<T, 4>(M, mode, x, b, dinv, y, yd, s, stop); break;
        case 8: sell_k<T, 8>(M, mode, x, b, dinv, y, yd, s, stop); break;
        case 16: sell_k<T, 16>(M, mode, x, b, dinv, y, yd, s, stop); break;
        case 32: sell_k<T, 32>(M, mode, x, b, dinv, y, yd, s, stop); break;
        default: sell_k<T, 64>(M, mode, x, b, dinv, y, yd, s, stop); break;
    }
}

template <class T, int K>
void sell_inc_k(const DSell& M, int add, const T* x, T* y, hipStream_t s, const int* stop) {
    unsigned g = grid_slices(M.nslices);
    if (g == 0) return;
    if (add) dev::k_sell_inc<T, K, 1><<<g, BLOCK, 0, s>>>(M.nslices, M.sptr, M.srow, M.ent, x, y, stop);
    else dev::k_sell_inc<T, K, 0><<<g, BLOCK, 0, s>>>(M.nslices, M.sptr, M.srow, M.ent, x, y, stop);
}

template <class T, int W>
void inc_fixed_w(const DSell& M, int add, const T* x, T* y, hipStream_t s, const int* stop) {
    const unsigned g = grid_for((M.nrows + dev::INC_ROWS - 1) / dev::INC_ROWS);
    if (add) dev::k_inc_fixed<T, W, 1><<<g, BLOCK, 0, s>>>(M.nrows, M.fent, x, y, stop);
    else dev::k_inc_fixed<T, W, 0><<<g, BLOCK, 0, s>>>(M.nrows, M.fent, x, y, stop);
}

template <class T>
void sell_inc(const DSell& M, int add, const T* x, T* y, hipStream_t s, const int* stop) {
    if (M.nrows == 0) return;
    switch (M.fixedw) {
        case 0: break;
        case 1: inc_fixed_w<T, 1>(M, add, x, y, s, stop); return;
        case 2: inc_fixed_w<T, 2>(M, add, x, y, s, stop); return;
        case 3: inc_fixed_w<T, 3>(M, add, x, y, s, stop); return;
        default: inc_fixed_w<T, 4>(M, add, x, y, s, stop); return;
    }
    switch (M.K) {
        case 1: sell_inc_k<T, 1>(M, add, x, y, s, stop); break;
        case 2: sell_inc_k<T, 2>(M, add, x, y, s, stop); break;
        case 4: sell_inc_k<T, 4>(M, add, x, y, s, stop); break;
        case 8: sell_inc_k<T, 8>(M, add, x, y, s, stop); break;
        case 16: sell_inc_k<T, 16>(M, add, x, y, s, stop); break;
        case 32: sell_inc_k<T, 32>(M, add, x, y, s, stop); break;
        default: sell_inc_k<T, 64>(M, add, x, y, s, stop); break;
    }
}

// ------------------------------------------------------------------ multicolour Gauss-Seidel
template <class T, int K, int UNR>
void gs_ku(const DSell& M, const T* b, const T* dg, T* x, hipStream_t s, const int* stop) {
    unsigned g = grid_slices(M.nslices);
    if (g == 0) return;
    const T* v = vals<T>(M);
    if (M.c16)
        dev::k_sell_gs<T, K, true, false, UNR><<<g, BLOCK, 0, s>>>(M.nslices, M.sptr, M.srow, M.ci, M.c16, M.cbase,
                                                                   v, b, dg, x, stop);
    else
        dev::k_sell_gs<T, K, false, false, UNR><<<g, BLOCK, 0, s>>>(M.nslices, M.sptr, M.srow, M.ci, M.c16,
                                                                    M.cbase, v, b, dg, x, stop);
}

// One colour's relaxation x_i += dg_i (b - A x)_i over the colour's rows.
template <class T>
void gs_color(const DSell& M, const T* b, const T* dg, T* x, hipStream_t s, const int* stop) {
    switch (M.K) {
        case 1: gs_ku<T, 1, 4>(M, b, dg, x, s, stop); break;
        case 2: gs_ku<T, 2, 4>(M, b, dg, x, s, stop); break;
        case 4: gs_ku<T, 4, 4>(M, b, dg, x, s, stop); break;
        case 8: gs_ku<T, 8, 4>(M, b, dg, x, s, stop); break;
        case 16: gs_ku<T, 16, 4>(M, b, dg, x, s, stop); break;
        case 32: gs_ku<T, 32, 4>(M, b, dg, x, s, stop); break;
        default: gs_ku<T, 64, 4>(M, b, dg, x, s, stop); break;
    }
}

// nu symmetric sweeps (colours increasing, then decreasing) on x in place.  The colour
// that ends one half-sweep would start the next with a zero residual on its rows, so it
// is not relaxed twice: nu sweeps of C colours launch 2 nu (C - 1) + 1 colours.
template <class T>
void gs_sweeps(const GsColors& g, const T* b, T* x, int nu, hipStream_t s, const int* stop) {
    const int C = (int)g.col.size();
    if (nu <= 0 || C == 0) return;
    const T* dg = g.dg<T>();
    gs_color<T>(g.col[0], b, dg, x, s, stop);
    for (int k = 0; k < nu; ++k) {
        for (int c = 1; c < C; ++c) gs_color<T>(g.col[c], b, dg, x, s, stop);
        for (int c = C - 2; c >= 0; --c) gs_color<T>(g.col[c], b, dg, x, s, stop);
    }
}

// ------------------------------------------------------------------ autotuning
// Lanes per row K for one matrix: every candidate layout is built and its FP32 product
// timed with HIP events; the fastest is kept.  Results are cached per matrix shape for
// the process lifetime.
struct TuneKey {
    int nrows, ncols;
    int64_t nnz;
    bool inc;
    bool operator<(const TuneKey& o) const {
        return std::tie(nrows, ncols, nnz, inc) < std::tie(o.nrows, o.ncols, o.nnz, o.inc);
    }
};

static bool verbose() {
    static int v = -1;
    if (v < 0) {
        const char* e = getenv("AMGE_VERBOSE");
        v = (e && *e && *e != '0') ? 1 : 0;
    }
    return v == 1;
}

static std::mutex g_tune_mu;
static std::map<TuneKey, int> g_tune;

int tune_lanes(const Csr& A, bool incidence, const amge_opts& opts, hipStream_t s, const Staged* st = nullptr) {
    TuneKey key{A.nrows, A.ncols, A.nnz(), incidence};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) return it->second;
    }
    const double avg = A.nrows ? (double)A.nnz() / A.nrows : 0;
    // starting point: long loops per lane on large matrices (bandwidth), more lanes per
    // row on small ones (latency); then the neighbours K/2, 2K are timed against it
    auto p2 = [](double v) { return 1 << std::min(5, std::max(0, (int)std::lround(std::log2(std::max(1.0, v))))); };
    const int k0 = p2(A.nrows >= 65536 ? avg / 16.0 : avg / 6.0);
    std::vector<int> cands = {k0};
    for (int K : {k0 / 2, k0 * 2})
        if (K >= 1 && K <= 32 && avg >= 2.0 * K) cands.push_back(K);
    int best = cands[0];
    if (cands.size() > 1) {
        std::unique_ptr<Staged> own;
        if (!st && device_layouts()) {
            own = stage(opts, A, s);
            st = own.get();
        }
        amge_hierarchy tmp;   // owns the trial buffers
        tmp.opts = opts;
        float* x = tmp.alloc<float>(A.ncols);
        float* y = tmp.alloc<float>(A.nrows);
        int* zero = tmp.alloc<int>(1);
        HIPCHECK(hipMemsetAsync(x, 0, sizeof(float) * A.ncols, s));
        HIPCHECK(hipMemsetAsync(zero, 0, sizeof(int), s));
        hipEvent_t e0, e1;
        HIPCHECK(hipEventCreate(&e0));
        HIPCHECK(hipEventCreate(&e1));
        float best_ms = 1e30f;
        for (int K : cands) {
            amge_hierarchy t2;
            t2.opts = opts;
            DSell M = upload_sell(&t2, A, incidence, K, s, nullptr, nullptr, st);
            auto run = [&]() {
                if (incidence) sell_inc<float>(M, 0, x, y, s, zero);
                else sell<float>(M, dev::SPMV, x, nullptr, nullptr, y, s, zero);
            };
            for (int i = 0; i < 2; ++i) run();
            float ms = 1e30f;
            for (int rep = 0; rep < 3; ++rep) {   // best of three rounds of five launches
                HIPCHECK(hipEventRecord(e0, s));
                for (int i = 0; i < 5; ++i) run();
                HIPCHECK(hipEventRecord(e1, s));
                HIPCHECK(hipEventSynchronize(e1));
                float t = 0;
                HIPCHECK(hipEventElapsedTime(&t, e0, e1));
                ms = std::min(ms, t);
            }
            HIPCHECK(hipGetLastError());
            if (verbose())
                fprintf(stderr, "[amge tune] rows %d nnz %lld avg %.1f K=%d: %.2f us\n", A.nrows, (long long)A.nnz(),
                        avg, K, 1e3 * ms / 5);
            if (ms < best_ms * 0.9f) {    // keep the starting point unless clearly faster
                best_ms = ms;
                best = K;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = best;
    return best;
}

DSell upload_tuned(amge_hierarchy* H, const Csr& A, bool incidence, hipStream_t s,
                   const std::vector<int>* lead = nullptr) {
    std::unique_ptr<Staged> st;
    if (device_layouts()) st = stage(H->opts, A, s);
    return upload_sell(H, A, incidence, tune_lanes(A, incidence, H->opts, s, st.get()), s, lead, nullptr, st.get());
}

// A signed incidence (entries +-1): rows of one common length W <= 4 (the fine-level
// derivatives) are stored row-major as n x W words for k_inc_fixed; others in the
// tuned sliced layout.
DSell upload_incidence(amge_hierarchy* H, const Csr& D, hipStream_t s) {
    int W = D.nrows ? D.rowptr[1] - D.rowptr[0] : 0;
    for (int i = 0; i < D.nrows && W; ++i)
        if (D.rowptr[i + 1] - D.rowptr[i] != W) W = 0;
    if (W < 1 || W > 4) return upload_tuned(H, D, true, s);
    std::vector<uint32_t> w((size_t)D.nrows * W);
    for (size_t q = 0; q < w.size(); ++q) {
        const double v = D.val[q];
        if (v != 1.0 && v != -1.0) fail(AMGE_ERR_ARG, "derivative matrix entries must be +-1");
        w[q] = (uint32_t)D.col[q] | (v < 0 ? 0x80000000u : 0u);
    }
    DSell d;
    d.nrows = D.nrows;
    d.ncols = D.ncols;
    d.nnz = D.nnz();
    d.stored = D.nnz();
    d.fixedw = W;
    d.fent = upload(H, w.data(), w.size(), s);
    HIPCHECK(hipStreamSynchronize(s));
    return d;
}

// Launch of an A_k kernel; on a probed level the launch is bracketed by events and its
// algorithmic bytes are counted: values + column indices, one row index per row, and
// the vector streams of the mode (x gathered once, b, dinv, y).
// y = b - A x with FP32 vectors and the FP64 values of A, summed in FP64 (the
// fine-level residual of an FP32 V-cycle with opts.resid_bits = 64).
template <int K, int UNR>
void sell_resid64_ku(const DSell& M, const float* x, const float* b, float* y, hipStream_t s, const int* stop) {
    const unsigned g = grid_slices(M.nslices);
    if (g == 0) return;
    if (M.c16)
        dev::k_sell<float, K, dev::RESID, true, true, UNR, double><<<g, BLOCK, 0, s>>>(
            M.nslices, M.sptr, M.srow, M.ci, M.c16, M.cbase, M.v64, x, b, nullptr, y, nullptr, M.lead, stop);
    else
        dev::k_sell<float, K, dev::RESID, false, true, UNR, double><<<g, BLOCK, 0, s>>>(
            M.nslices, M.sptr, M.srow, M.ci, M.c16, M.cbase, M.v64, x, b, nullptr, y, nullptr, M.lead, stop);
}

template <int K>
void sell_resid64_k(const DSell& M, const float* x, const float* b, float* y, hipStream_t s, const int* stop) {
    if constexpr (K <= 8) {
        if (M.deep) {
            sell_resid64_ku<K, 8>(M, x, b, y, s, stop);
            return;
        }
    }
    sell_resid64_ku<K, 4>(M, x, b, y, s, stop);
}

void sell_resid64(const DSell& M, const float* x, const float* b, float* y, hipStream_t s, const int* stop) {
    if (!M.v64) fail(AMGE_ERR_ARG, "FP64 residual on a matrix without FP64 values");
    switch (M.K) {
        case 1: sell_resid64_k<1>(M, x, b, y, s, stop); break;
        case 2: sell_resid64_k<2>(M, x, b, y, s, stop); break;
        case 4: sell_resid64_k<4>(M, x, b, y, s, stop); break;
        case 8: sell_resid64_k<8>(M, x, b, y, s, stop); break;
        case 16: sell_resid64_k<16>(M, x, b, y, s, stop); break;
        case 32: sell_resid64_k<32>(M, x, b, y, s, stop); break;
        default: sell_resid64_k<64>(M, x, b, y, s, stop); break;
    }
}

// A launch on A_k (probed on the fine level when timing is on); the residual of an FP32
// level with resid64 takes the FP64 values.
template <class T>
void asell_launch(DLevel& L, int mode, const T* x, const T* b, const T* dinv, T* y, hipStream_t s, const int* stop) {
    if constexpr (std::is_same<T, float>::value) {
        if (L.resid64 && mode == dev::RESID) {
            sell_resid64(L.A, x, b, y, s, stop);
            return;
        }
    }
    sell<T>(L.A, mode, x, b, dinv, y, s, stop);
}

template <class T>
void asell(DLevel& L, int mode, const T* x, const T* b, const T* dinv, T* y, hipStream_t s, const int* stop) {
    Probe* pr = L.probe;
    if (!pr || !pr->on) {
        asell_launch<T>(L, mode, x, b, dinv, y, s, stop);
        return;
    }
    if (pr->ev.size() < 2 * (pr->used + 1)) {
        hipEvent_t a, c;
        HIPCHECK(hipEventCreate(&a));
        HIPCHECK(hipEventCreate(&c));
        pr->ev.push_back(a);
        pr->ev.push_back(c);
    }
    HIPCHECK(hipEventRecord(pr->ev[2 * pr->used], s));
    asell_launch<T>(L, mode, x, b, dinv, y, s, stop);
    HIPCHECK(hipEventRecord(pr->ev[2 * pr->used + 1], s));
    pr->used++;
    const double nv = mode == dev::JAC ? 4 : 3;   // JAC: x, b, dinv, y; others: three streams
    const double vs = (std::is_same<T, float>::value && L.resid64 && mode == dev::RESID) ? 8 : sizeof(T);
    pr->bytes += (double)L.A.nnz * (vs + (L.A.c16 ? 2 : 4)) + 4.0 * L.n + nv * sizeof(T) * L.n;
}

template <class T>
void scale(int n, const T* dinv, const T* x, T* y, hipStream_t s) {
    if (n) dev::k_scale<T><<<grid_for(n), BLOCK, 0, s>>>(n, dinv, x, y);
}

// x = M b for a dense FP64 n x n operator (k_coarse)
template <class T>
void dense_apply(int n, const double* M, const T* b, T* x, hipStream_t s, const int* stop) {
    if (n) dev::k_coarse<T><<<(unsigned)((n + WAVES - 1) / WAVES), BLOCK, 0, s>>>(n, M, b, x, stop);
}

// The coarsest solve with the inverse from the Cholesky factor
template <class T>
void coarse_solve(amge_hierarchy* H, const T* b, T* x, hipStream_t s, const int* stop) {
    dense_apply<T>(H->nc, H->Ainv, b, x, s, stop);
}

template <class T>
void copy_vec(int64_t n, const T* a, T* b, hipStream_t s, const int* stop) {
    if (n) launch<dev::Copy<T>>((unsigned)std::min<int64_t>(grid_for(n), 4096), s, n, a, b, stop);
}

template <class T>
void fill_zero(int64_t n, T* x, hipStream_t s, const int* stop) {
    if (n) launch<dev::Fill<T>>((unsigned)std::min<int64_t>(grid_for(n), 4096), s, n, x, stop);
}

template <class S, class D>
void convert(int64_t n, const S* a, D* b, hipStream_t s) {
    if (n) dev::k_convert<S, D><<<(unsigned)std::min<int64_t>(grid_for(n), 4096), BLOCK, 0, s>>>(n, a, b);
}

// ------------------------------------------------------------------ smoother and V-cycle
// Primary l1-Jacobi sweeps on A: x <- x + dinv (b - A x), nu times.  From zero, the
// first sweep is x = dinv b, which the producer of b has already written to bd, so the
// first launched sweep starts from bd.  x and xt are swapped by the ping-pong; the
// caller tracks where the result is.
// One block Gauss-Seidel sweep on A_k or D^T A D (probed on the fine level like asell).
template <class T>
void bgs(DLevel& L, const DBgs& g, bool zero, const T* x, const T* b, T* y, hipStream_t s, const int* stop) {
    Probe* pr = &g == &L.bgA ? L.probe : nullptr;
    if (!pr || !pr->on) {
        bgs_launch<T>(g, zero, x, b, y, s, stop);
        return;
    }
    if (pr->ev.size() < 2 * (pr->used + 1)) {
        hipEvent_t a, c;
        HIPCHECK(hipEventCreate(&a));
        HIPCHECK(hipEventCreate(&c));
        pr->ev.push_back(a);
        pr->ev.push_back(c);
    }
    HIPCHECK(hipEventRecord(pr->ev[2 * pr->used], s));
    bgs_launch<T>(g, zero, x, b, y, s, stop);
    HIPCHECK(hipEventRecord(pr->ev[2 * pr->used + 1], s));
    pr->used++;
    pr->bytes += bgs_bytes(g, zero, (int)sizeof(T));
}

// r = b - A x ahead of the restriction.  With the block Gauss-Seidel smoother it reads
// the smoother's copy of A_k (one copy of A_k stays cache-resident through the V-cycle);
// probed on the fine level like the sweeps.
template <class T>
void aresid(DLevel& L, const T* x, const T* b, T* r, hipStream_t s, const int* stop) {
    if (!L.bgA.on()) {
        asell<T>(L, dev::RESID, x, b, nullptr, r, s, stop);
        return;
    }
    const bool v64 = std::is_same<T, float>::value && L.resid64;
    Probe* pr = L.probe;
    if (!pr || !pr->on) {
        bgs_resid_launch<T>(L.bgA, v64, x, b, r, s, stop);
        return;
    }
    if (pr->ev.size() < 2 * (pr->used + 1)) {
        hipEvent_t a, c;
        HIPCHECK(hipEventCreate(&a));
        HIPCHECK(hipEventCreate(&c));
        pr->ev.push_back(a);
        pr->ev.push_back(c);
    }
    HIPCHECK(hipEventRecord(pr->ev[2 * pr->used], s));
    bgs_resid_launch<T>(L.bgA, v64, x, b, r, s, stop);
    HIPCHECK(hipEventRecord(pr->ev[2 * pr->used + 1], s));
    pr->used++;
    pr->bytes += bgs_resid_bytes(L.bgA, v64 ? 8 : (int)sizeof(T), (int)sizeof(T));
}

// nu block Gauss-Seidel sweeps through the ping-pong pair x / xt (the result ends in x).
template <class T>
void bgs_sweeps(DLevel& L, const DBgs& g, const T* b, T*& x, T*& xt, bool from_zero, int nu, hipStream_t s,
                const int* stop) {
    int k = 0;
    if (from_zero) {
        if (nu <= 0) {
            fill_zero<T>(g.n, x, s, stop);
            return;
        }
        // start in the other buffer: a V-cycle level then makes 2 nu - 1 swaps in all
        // and ends in the buffer it started with (no copy)
        std::swap(x, xt);
        bgs<T>(L, g, true, nullptr, b, x, s, stop);
        k = 1;
    }
    for (; k < nu; ++k) {
        bgs<T>(L, g, false, x, b, xt, s, stop);
        std::swap(x, xt);
    }
}

template <class T>
void primary(DLevel& L, const T* b, const T* bd, T*& x, T*& xt, bool from_zero, int nu, hipStream_t s,
             const int* stop) {
    if (L.bgA.on()) {   // l1-scaled symmetric block Gauss-Seidel
        bgs_sweeps<T>(L, L.bgA, b, x, xt, from_zero, nu, s, stop);
        return;
    }
    if (!L.gsA.col.empty()) {   // symmetric Gauss-Seidel: in place, from zero if asked
        if (from_zero) fill_zero<T>(L.n, x, s, stop);
        gs_sweeps<T>(L.gsA, b, x, nu, s, stop);
        return;
    }
    Work<T>& w = L.w<T>();
    int k = 0;
    if (from_zero) {
        if (nu >= 2) {
            asell<T>(L, dev::JAC, bd, b, w.dinv, x, s, stop);
            k = 2;
        } else if (nu == 1) {
            copy_vec<T>(L.n, bd, x, s, stop);
            k = 1;
        } else {
            fill_zero<T>(L.n, x, s, stop);
        }
    }
    for (; k < nu; ++k) {
        asell<T>(L, dev::JAC, x, b, w.dinv, xt, s, stop);
        std::swap(x, xt);
    }
}

// Auxiliary correction of eq. (4.1): x <- x + D Mhat^{-1} D^T (b - A x), Mhat^{-1} being
// nu l1-Jacobi sweeps on D^T A D from zero.  The residual kernel also writes the first
// sweep gd = dhinv g.
template <class T>
void auxiliary(DLevel& L, const T* b, T* x, int nu, hipStream_t s, const int* stop) {
    if (nu <= 0 || L.m == 0) return;
    Work<T>& w = L.w<T>();
    if (L.bgAh.on()) {   // block Gauss-Seidel sweeps on D^T A D from zero
        sell<T>(L.Aux, dev::SPLIT, x, b, nullptr, w.g, s, stop);
        T* y = w.y;
        T* yt = w.yt;
        bgs_sweeps<T>(L, L.bgAh, w.g, y, yt, true, nu, s, stop);
        sell_inc<T>(L.D, 1, y, x, s, stop);
        return;
    }
    if (!L.gsAh.col.empty()) {   // symmetric Gauss-Seidel sweeps on D^T A D from zero
        sell<T>(L.Aux, dev::SPLIT, x, b, nullptr, w.g, s, stop);
        fill_zero<T>(L.m, w.y, s, stop);
        gs_sweeps<T>(L.gsAh, w.g, w.y, nu, s, stop);
        sell_inc<T>(L.D, 1, w.y, x, s, stop);
        return;
    }
    sell<T>(L.Aux, dev::SPLIT, x, b, w.dhinv, w.g, s, stop, w.gd);
    const T* y = w.gd;
    T* ya = w.y;
    T* yb = w.yt;
    for (int k = 1; k < nu; ++k) {
        sell<T>(L.Ah, dev::JAC, y, w.g, w.dhinv, ya, s, stop);
        y = ya;
        std::swap(ya, yb);
    }
    sell_inc<T>(L.D, 1, y, x, s, stop);
}

// One V-cycle (Algorithm 4.1, x0 = 0) from level l down: b and bd = dinv b are the
// level's right-hand side and first sweep, the result goes to xout.
template <class T>
void vcycle_level(amge_hierarchy* H, int l, const T* b, const T* bd, T* xout, hipStream_t s, const int* stop) {
    if (l == H->tail) {   // the coarsest solve, or the folded coarse tail
        dense_apply<T>(H->tail_n, H->tail_op, b, xout, s, stop);
        return;
    }
    DLevel& L = H->lv[l];
    DLevel& C = H->lv[l + 1];
    Work<T>& w = L.w<T>();
    Work<T>& wc = C.w<T>();
    T* x = xout;
    T* xt = w.xt;
    const int nup = H->opts.nu_primary, nua = H->opts.nu_aux;
    // the coarse level's first l1-Jacobi sweep from zero, written with its right-hand
    // side (not needed by the coarsest level or the Gauss-Seidel smoothers)
    const bool next_coarsest = l + 1 == H->tail || C.bgA.on() || !C.gsA.col.empty();
    // pre-smoothing with Mbar (eq. (4.1)): primary, then auxiliary
    primary<T>(L, b, bd, x, xt, true, nup, s, stop);
    auxiliary<T>(L, b, x, nua, s, stop);
    // restriction of the residual (and the coarse first sweep), coarse correction,
    // prolongation
    if (L.PtA.nrows) {   // P^T b - (P^T A) x in one launch
        sell<T>(L.PtA, dev::SPLIT, x, b, next_coarsest ? nullptr : wc.dinv, wc.b, s, stop,
                next_coarsest ? nullptr : wc.bd);
    } else {
        aresid<T>(L, x, b, w.r, s, stop);
        sell<T>(L.Pt, dev::SPMV, w.r, nullptr, next_coarsest ? nullptr : wc.dinv, wc.b, s, stop,
                next_coarsest ? nullptr : wc.bd);
    }
    vcycle_level<T>(H, l + 1, wc.b, wc.bd, wc.x, s, stop);
    sell<T>(L.P, dev::SPMV_ADD, wc.x, nullptr, nullptr, x, s, stop);
    // post-smoothing with Mbar^T: auxiliary first, then primary
    auxiliary<T>(L, b, x, nua, s, stop);
    primary<T>(L, b, nullptr, x, xt, false, nup, s, stop);
    if (x != xout) copy_vec<T>(L.n, x, xout, s, stop);
}

// z = B r on level-1 vectors in FP64; the FP32 path rounds r, runs the V-cycle in FP32
// and widens the result.
void precondition(amge_hierarchy* H, const double* r, double* z, hipStream_t s) {
    DLevel& L = H->lv[0];
    if (H->opts.precond_bits == 32) {
        convert<double, float>(L.n, r, L.w32.b, s);
        scale<float>(L.n, L.w32.dinv, L.w32.b, L.w32.bd, s);
        vcycle_level<float>(H, 0, L.w32.b, L.w32.bd, L.w32.x, s, H->zero_flag);
        convert<float, double>(L.n, L.w32.x, z, s);
    } else {
        scale<double>(L.n, L.w64.dinv, r, L.w64.bd, s);
        vcycle_level<double>(H, 0, r, L.w64.bd, z, s, H->zero_flag);
    }
}

// ------------------------------------------------------------------ batched path
// Several right-hand sides at once (n x NC row-major blocks, NC a power of two): every
// level operator is one SpMM launch over the one-lane-per-row sliced ELL, whose lanes
// own V consecutive columns of a row.  V is tuned per matrix at set-up.
constexpr int BPCG_BLOCKS = 2048;  // blocks of the per-column dot products
constexpr int BPCG_CHUNK = 4;      // graph replays between status polls
template <class T> const T* bvals(const DSellB& M);
template <> const float* bvals<float>(const DSellB& M) { return M.v32; }
template <> const double* bvals<double>(const DSellB& M) { return M.v64; }

DSellB upload_sell_b(amge_hierarchy* H, const Csr& A, bool incidence, bool f32, bool f64, hipStream_t s,
                     const std::vector<int>* lead = nullptr) {
    const bool on_dev = device_layouts();
    HostSell h = on_dev ? sell_rows(A, 1, lead) : make_sell(A, incidence, 1, lead);
    DSellB M;
    M.nrows = A.nrows;
    M.ncols = A.ncols;
    M.nnz = A.nnz();
    M.nslices = h.nslices;
    M.sptr = upload(H, h.sptr.data(), h.sptr.size(), s);
    M.srow = upload(H, h.srow.data(), h.srow.size(), s);
    if (!incidence && lead) M.lead = upload(H, h.lead.data(), h.lead.size(), s);
    if (on_dev) {
        const std::unique_ptr<Staged> st = stage(H->opts, A, s);
        const DevEntries e = fill_entries(H, *st, h, M.sptr, incidence, f32, f64, s);
        M.ent = e.ent;
        M.ci = e.ci;
        M.c16 = e.c16;
        M.cbase = e.cbase;
        M.v64 = e.v64;
        M.v32 = e.v32;
        return M;
    }
    if (incidence) {
        M.ent = upload(H, h.ent.data(), h.ent.size(), s);
    } else {
        if (h.compact && compact_indices()) {
            M.c16 = upload(H, h.c16.data(), h.c16.size(), s);
            M.cbase = upload(H, h.cbase.data(), h.cbase.size(), s);
        } else {
            M.ci = upload(H, h.ci.data(), h.ci.size(), s);
        }
        if (f64) M.v64 = upload(H, h.val.data(), h.val.size(), s);
        if (f32) {
            std::vector<float> v(h.val.begin(), h.val.end());
            M.v32 = upload(H, v.data(), v.size(), s);
        }
    }
    HIPCHECK(hipStreamSynchronize(s));
    return M;
}

template <class T, int V, int MODE>
void bmm_v(const DSellB& M, int W, int NC, const T* X, const T* B, const T* dinv, T* Y, T* YD,
           const int* stop, hipStream_t s) {
    const int L = W / V;
    const unsigned grid = (unsigned)(((int64_t)M.nslices * L + WAVES - 1) / WAVES);
    if (!grid) return;
    if (M.c16)
        launch<dev::SellMM<T, V, MODE, true>>(grid, s, M.nslices, L, NC, M.sptr, M.srow, M.ci, M.c16, M.cbase,
                                              bvals<T>(M), X, B, dinv, Y, YD, M.lead, stop);
    else
        launch<dev::SellMM<T, V, MODE, false>>(grid, s, M.nslices, L, NC, M.sptr, M.srow, M.ci, M.c16, M.cbase,
                                               bvals<T>(M), X, B, dinv, Y, YD, M.lead, stop);
}

template <class T, int V>
void bmm_m(const DSellB& M, int mode, int W, int NC, const T* X, const T* B, const T* dinv, T* Y, T* YD,
           const int* stop, hipStream_t s) {
    switch (mode) {
        case dev::SPMV: bmm_v<T, V, dev::SPMV>(M, W, NC, X, B, dinv, Y, YD, stop, s); break;
        case dev::SPMV_ADD: bmm_v<T, V, dev::SPMV_ADD>(M, W, NC, X, B, dinv, Y, YD, stop, s); break;
        case dev::RESID: bmm_v<T, V, dev::RESID>(M, W, NC, X, B, dinv, Y, YD, stop, s); break;
        case dev::JAC: bmm_v<T, V, dev::JAC>(M, W, NC, X, B, dinv, Y, YD, stop, s); break;
        case dev::JAC0: bmm_v<T, V, dev::JAC0>(M, W, NC, X, B, dinv, Y, YD, stop, s); break;
        case dev::SPLIT:
            if (!M.lead) fail(AMGE_ERR_ARG, "split product on a matrix without split rows");
            bmm_v<T, V, dev::SPLIT>(M, W, NC, X, B, dinv, Y, YD, stop, s);
            break;
        default: fail(AMGE_ERR_ARG, "bad SpMM mode");
    }
}

// Columns per lane actually used: the tuned V, at most the active width W.
inline int lane_cols(int V, int W) { return std::min(V, W); }

// Y = B - A X on FP32 blocks with the FP64 values of A, summed in FP64 (the fine-level
// residual of an FP32 batched V-cycle with opts.resid_bits = 64).
template <int V>
void bmm_resid64_v(const DSellB& M, int W, int NC, const float* X, const float* B, float* Y, const int* stop,
                   hipStream_t s) {
    const int L = W / V;
    const unsigned grid = (unsigned)(((int64_t)M.nslices * L + WAVES - 1) / WAVES);
    if (!grid) return;
    if (M.c16)
        launch<dev::SellMM<float, V, dev::RESID, true, double>>(grid, s, M.nslices, L, NC, M.sptr, M.srow, M.ci,
                                                                M.c16, M.cbase, (const double*)M.v64, X, B,
                                                                (const float*)nullptr, Y, (float*)nullptr, M.lead,
                                                                stop);
    else
        launch<dev::SellMM<float, V, dev::RESID, false, double>>(grid, s, M.nslices, L, NC, M.sptr, M.srow, M.ci,
                                                                 M.c16, M.cbase, (const double*)M.v64, X, B,
                                                                 (const float*)nullptr, Y, (float*)nullptr, M.lead,
                                                                 stop);
}

void bmm_resid64(const DSellB& M, int W, int NC, const float* X, const float* B, float* Y, const int* stop,
                 hipStream_t s) {
    if (!M.v64) fail(AMGE_ERR_ARG, "FP64 residual on a matrix without FP64 values");
    switch (lane_cols(M.V, W)) {
        case 1: bmm_resid64_v<1>(M, W, NC, X, B, Y, stop, s); break;
        case 2: bmm_resid64_v<2>(M, W, NC, X, B, Y, stop, s); break;
        case 4: bmm_resid64_v<4>(M, W, NC, X, B, Y, stop, s); break;
        case 8: bmm_resid64_v<8>(M, W, NC, X, B, Y, stop, s); break;
        default: bmm_resid64_v<16>(M, W, NC, X, B, Y, stop, s); break;
    }
}

// Block product on the first W (active) of the NC stored columns.
template <class T>
void bmm(const DSellB& M, int mode, int W, int NC, const T* X, const T* B, const T* dinv, T* Y, const int* stop,
         hipStream_t s, T* YD = nullptr) {
    switch (lane_cols(M.V, W)) {
        case 1: bmm_m<T, 1>(M, mode, W, NC, X, B, dinv, Y, YD, stop, s); break;
        case 2: bmm_m<T, 2>(M, mode, W, NC, X, B, dinv, Y, YD, stop, s); break;
        case 4: bmm_m<T, 4>(M, mode, W, NC, X, B, dinv, Y, YD, stop, s); break;
        case 8: bmm_m<T, 8>(M, mode, W, NC, X, B, dinv, Y, YD, stop, s); break;
        default: bmm_m<T, 16>(M, mode, W, NC, X, B, dinv, Y, YD, stop, s); break;
    }
}

template <class T, int V>
void inc_mm_v(const DSellB& M, int W, int NC, const T* X, T* Y, const int* stop, hipStream_t s) {
    const int L = W / V;
    const unsigned grid = (unsigned)(((int64_t)M.nslices * L + WAVES - 1) / WAVES);
    launch<dev::IncMMAdd<T, V>>(grid, s, M.nslices, L, NC, M.sptr, M.srow, M.ent, X, Y, stop);
}

template <class T>
void inc_mm_add(const DSellB& M, int W, int NC, const T* X, T* Y, const int* stop, hipStream_t s) {
    switch (lane_cols(M.V, W)) {
        case 1: inc_mm_v<T, 1>(M, W, NC, X, Y, stop, s); break;
        case 2: inc_mm_v<T, 2>(M, W, NC, X, Y, stop, s); break;
        case 4: inc_mm_v<T, 4>(M, W, NC, X, Y, stop, s); break;
        case 8: inc_mm_v<T, 8>(M, W, NC, X, Y, stop, s); break;
        default: inc_mm_v<T, 16>(M, W, NC, X, Y, stop, s); break;
    }
}

inline unsigned grid_stride(int64_t threads) { return (unsigned)std::min<int64_t>(grid_for(threads), 4096); }

template <class T>
void bfill(int64_t n, T* x, const int* stop, hipStream_t s) {
    if (n) launch<dev::Fill<T>>(grid_stride(n), s, n, x, stop);
}

template <class T>
void bcopy(int64_t n, const T* a, T* b, const int* stop, hipStream_t s) {
    if (n) launch<dev::Copy<T>>(grid_stride(n), s, n, a, b, stop);
}

// Columns per lane V for one matrix and block width NC: the default (16-byte lane
// loads) is timed against the other widths with HIP events and replaced only by a
// clearly faster one.  Cached per matrix shape, width and precision.
struct BTuneKey {
    int nrows, ncols;
    int64_t nnz;
    int inc, NC, bits;
    bool operator<(const BTuneKey& o) const {
        return std::tie(nrows, ncols, nnz, inc, NC, bits) < std::tie(o.nrows, o.ncols, o.nnz, o.inc, o.NC, o.bits);
    }
};
static std::map<BTuneKey, int> g_btune;

template <class T>
int tune_cols(DSellB& M, bool incidence, int NC, T* X, T* Y, const int* stop, hipStream_t s) {
    BTuneKey key{M.nrows, M.ncols, M.nnz, incidence ? 1 : 0, NC, (int)(8 * sizeof(T))};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_btune.find(key);
        if (it != g_btune.end()) return it->second;
    }
    const int v0 = std::min(NC, (int)(16 / sizeof(T)));
    std::vector<int> cands = {v0};
    for (int V : {1, 2, 4, 8, 16})
        if (V != v0 && V <= NC && V * sizeof(T) <= 64) cands.push_back(V);
    hipEvent_t e0, e1;
    HIPCHECK(hipEventCreate(&e0));
    HIPCHECK(hipEventCreate(&e1));
    int best = v0;
    float best_ms = 1e30f;
    for (int V : cands) {
        M.V = V;
        auto run = [&]() {
            if (incidence) inc_mm_add<T>(M, NC, NC, X, Y, stop, s);
            else bmm<T>(M, dev::SPMV, NC, NC, X, nullptr, nullptr, Y, stop, s);
        };
        run();
        float ms = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            HIPCHECK(hipEventRecord(e0, s));
            for (int i = 0; i < 3; ++i) run();
            HIPCHECK(hipEventRecord(e1, s));
            HIPCHECK(hipEventSynchronize(e1));
            float t = 0;
            HIPCHECK(hipEventElapsedTime(&t, e0, e1));
            ms = std::min(ms, t);
        }
        HIPCHECK(hipGetLastError());
        if (verbose())
            fprintf(stderr, "[amge tune-mm] rows %d nnz %lld NC %d fp%d V=%d: %.2f us\n", M.nrows, (long long)M.nnz, NC,
                    (int)(8 * sizeof(T)), V, 1e3 * ms / 3);
        if (V == v0 || ms < best_ms * 0.95f) {   // keep the default unless clearly faster
            best_ms = ms;
            best = V;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    M.V = best;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_btune[key] = best;
    return best;
}

// ---- batched smoother and V-cycle: the single-column steps on n x NC blocks, of which
// the first W columns are computed (the others are idle); every kernel returns at once
// when *stop is set (all columns of a PCG batch converged).
template <class T>
void bprimary(amge_hierarchy* H, DLevel& L, const T* b, const T* bd, T*& x, T*& xt, bool from_zero, int nu, int W,
              const int* stop, hipStream_t s) {
    Work<T>& w = L.bw<T>();
    const int NC = H->NC;
    int k = 0;
    if (L.bgA.on()) {   // block Gauss-Seidel sweeps, arranged as in bgs_sweeps (no final copy)
        if (from_zero) {
            if (nu <= 0) {
                bfill<T>((int64_t)L.n * NC, x, stop, s);
                return;
            }
            std::swap(x, xt);
            bgs_mm_launch<T>(L.bgA, true, W, NC, nullptr, b, x, stop, s);
            k = 1;
        }
        for (; k < nu; ++k) {
            bgs_mm_launch<T>(L.bgA, false, W, NC, x, b, xt, stop, s);
            std::swap(x, xt);
        }
        return;
    }
    if (from_zero) {
        if (nu >= 2) {
            // bd = dinv b from the producer of b, or (bd null) formed by the sweep itself
            if (bd) bmm<T>(L.bA, dev::JAC, W, NC, bd, b, w.dinv, x, stop, s);
            else bmm<T>(L.bA, dev::JAC0, W, NC, nullptr, b, w.dinv, x, stop, s);
            k = 2;
        } else if (nu == 1) {
            if (!bd) fail(AMGE_ERR_ARG, "one sweep from zero needs dinv b");
            bcopy<T>((int64_t)L.n * NC, bd, x, stop, s);
            k = 1;
        } else {
            bfill<T>((int64_t)L.n * NC, x, stop, s);
        }
    }
    for (; k < nu; ++k) {
        bmm<T>(L.bA, dev::JAC, W, NC, x, b, w.dinv, xt, stop, s);
        std::swap(x, xt);
    }
}

template <class T>
void bauxiliary(amge_hierarchy* H, DLevel& L, const T* b, T* x, int nu, int W, const int* stop, hipStream_t s) {
    if (nu <= 0 || L.m == 0) return;
    Work<T>& w = L.bw<T>();
    const int NC = H->NC;
    if (L.bgAh.on()) {   // block Gauss-Seidel sweeps on D^T A D from zero
        bmm<T>(L.bAux, dev::SPLIT, W, NC, x, b, nullptr, w.g, stop, s);
        T* y = w.y;
        T* yt = w.yt;
        bgs_mm_launch<T>(L.bgAh, true, W, NC, nullptr, w.g, yt, stop, s);
        y = yt;
        yt = w.y;
        for (int k = 1; k < nu; ++k) {
            bgs_mm_launch<T>(L.bgAh, false, W, NC, y, w.g, yt, stop, s);
            std::swap(y, yt);
        }
        inc_mm_add<T>(L.bD, W, NC, y, x, stop, s);
        return;
    }
    bmm<T>(L.bAux, dev::SPLIT, W, NC, x, b, w.dhinv, w.g, stop, s, w.gd);
    const T* y = w.gd;
    T* ya = w.y;
    T* yb = w.yt;
    for (int k = 1; k < nu; ++k) {
        bmm<T>(L.bAh, dev::JAC, W, NC, y, w.g, w.dhinv, ya, stop, s);
        y = ya;
        std::swap(ya, yb);
    }
    inc_mm_add<T>(L.bD, W, NC, y, x, stop, s);
}

inline int log2i(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

// X = tail_op B on the first W columns (the batched coarsest solve or folded tail).
template <class T, int CPT>
void bcoarse_c(const amge_hierarchy* H, int W, const T* b, T* x, const int* stop, hipStream_t s) {
    const int R = H->tail_rpb, n = H->tail_n, lgW = log2i(W);
    const unsigned grid = (unsigned)((n + R - 1) / R);
    switch (R) {
        case 1: launch<dev::CoarseMM<T, CPT, 1>>(grid, s, n, lgW, H->lgNC, H->tail_op, b, x, stop); break;
        case 2: launch<dev::CoarseMM<T, CPT, 2>>(grid, s, n, lgW, H->lgNC, H->tail_op, b, x, stop); break;
        default: launch<dev::CoarseMM<T, CPT, 4>>(grid, s, n, lgW, H->lgNC, H->tail_op, b, x, stop);
    }
}

template <class T>
void bcoarse(const amge_hierarchy* H, int W, const T* b, T* x, const int* stop, hipStream_t s) {
    switch (std::min(H->NC, 8)) {   // columns per thread
        case 1: bcoarse_c<T, 1>(H, W, b, x, stop, s); break;
        case 2: bcoarse_c<T, 2>(H, W, b, x, stop, s); break;
        case 4: bcoarse_c<T, 4>(H, W, b, x, stop, s); break;
        default: bcoarse_c<T, 8>(H, W, b, x, stop, s);
    }
}

// Rows per block of the batched dense tail: 4, 2 and 1 timed on the full width (a
// row's sums do not depend on it), a smaller count kept only if clearly faster (few
// rows leave too few blocks to fill the device).
template <class T>
void tune_tail(amge_hierarchy* H, hipStream_t s) {
    if (!H->tail_n || H->NC < 2) return;
    const size_t m = (size_t)H->tail_n * H->NC;
    amge_hierarchy tmp;   // owns the trial buffers
    tmp.opts = H->opts;
    T* B = tmp.alloc<T>(m);
    T* X = tmp.alloc<T>(m);
    HIPCHECK(hipMemsetAsync(B, 0, sizeof(T) * m, s));
    hipEvent_t e0, e1;
    HIPCHECK(hipEventCreate(&e0));
    HIPCHECK(hipEventCreate(&e1));
    int best = 4;
    float best_ms = 1e30f;
    for (int R : {4, 2, 1}) {
        H->tail_rpb = R;
        bcoarse<T>(H, H->NC, B, X, H->zero_flag, s);
        float ms = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            HIPCHECK(hipEventRecord(e0, s));
            for (int i = 0; i < 3; ++i) bcoarse<T>(H, H->NC, B, X, H->zero_flag, s);
            HIPCHECK(hipEventRecord(e1, s));
            HIPCHECK(hipEventSynchronize(e1));
            float t = 0;
            HIPCHECK(hipEventElapsedTime(&t, e0, e1));
            ms = std::min(ms, t);
        }
        HIPCHECK(hipGetLastError());
        if (verbose())
            fprintf(stderr, "[amge tune-tail] n %d NC %d rows/block %d: %.2f us\n", H->tail_n, H->NC, R, 1e3 * ms / 3);
        if (R == 4 || ms < best_ms * 0.95f) {
            best_ms = ms;
            best = R;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    H->tail_rpb = best;
}

template <class T>
void bvcycle_level(amge_hierarchy* H, int l, const T* b, const T* bd, T* xout, int W, const int* stop,
                   hipStream_t s) {
    const int NC = H->NC;
    if (l == H->tail) {   // the coarsest solve, or the folded coarse tail
        if (H->tail_n) bcoarse<T>(H, W, b, xout, stop, s);
        return;
    }
    DLevel& L = H->lv[l];
    DLevel& C = H->lv[l + 1];
    Work<T>& w = L.bw<T>();
    Work<T>& wc = C.bw<T>();
    T* x = xout;
    T* xt = w.xt;
    const int nup = H->opts.nu_primary, nua = H->opts.nu_aux;
    // the coarse level's first l1-Jacobi sweep from zero, written with its right-hand side
    // (not needed by the coarsest level or the block Gauss-Seidel smoother)
    const bool next_coarsest = l + 1 == H->tail || C.bgA.on();
    bprimary<T>(H, L, b, bd, x, xt, true, nup, W, stop, s);
    bauxiliary<T>(H, L, b, x, nua, W, stop, s);
    if (L.bgA.on()) {
        bgs_resid_mm_launch<T>(L.bgA, std::is_same<T, float>::value && L.resid64, W, NC, x, b, w.r, stop, s);
    } else if constexpr (std::is_same<T, float>::value) {
        if (L.resid64) bmm_resid64(L.bA, W, NC, x, b, w.r, stop, s);
        else bmm<T>(L.bA, dev::RESID, W, NC, x, b, nullptr, w.r, stop, s);
    } else {
        bmm<T>(L.bA, dev::RESID, W, NC, x, b, nullptr, w.r, stop, s);
    }
    bmm<T>(L.bPt, dev::SPMV, W, NC, w.r, nullptr, next_coarsest ? nullptr : wc.dinv, wc.b, stop, s,
              next_coarsest ? nullptr : wc.bd);
    bvcycle_level<T>(H, l + 1, wc.b, wc.bd, wc.x, W, stop, s);
    bmm<T>(L.bP, dev::SPMV_ADD, W, NC, wc.x, nullptr, nullptr, x, stop, s);
    bauxiliary<T>(H, L, b, x, nua, W, stop, s);
    bprimary<T>(H, L, b, nullptr, x, xt, false, nup, W, stop, s);
    if (x != xout) bcopy<T>((int64_t)L.n * NC, x, xout, stop, s);
}

// Active width for nrhs columns: the power of two >= nrhs (at most NC).
inline int active_width(const amge_hierarchy* H, int nrhs) {
    int W = 1;
    while (W < nrhs) W *= 2;
    return std::min(W, H->NC);
}

// Batched V-cycle on the caller's n x nrhs FP64 block.
template <class T>
void bprecondition(amge_hierarchy* H, const double* r, double* z, int nrhs, hipStream_t s) {
    DLevel& L = H->lv[0];
    Work<T>& w = L.bw<T>();
    const int64_t n = L.n;
    const bool ml = H->lv.size() > 1;
    dev::k_pack<T><<<grid_stride(n * H->NC), BLOCK, 0, s>>>(n, nrhs, H->lgNC, r, ml ? w.dinv : nullptr, w.b,
                                                           ml ? w.bd : nullptr);
    bvcycle_level<T>(H, 0, w.b, w.bd, w.x, active_width(H, nrhs), H->zero_flag, s);
    dev::k_unpack<T><<<grid_stride(n * nrhs), BLOCK, 0, s>>>(n, nrhs, H->lgNC, w.x, z);
}

// ------------------------------------------------------------------ set-up
// Dense FP64 Cholesky factor of the coarsest matrix and the inverse it gives; the host
// copy of the inverse goes to ainv.
void build_coarse(amge_hierarchy* H, const Csr& A, hipStream_t s, std::vector<double>& ainv) {
    int n = A.nrows;
    if (n > 8192) fail(AMGE_ERR_ARG, "coarsest level larger than 8192 rows");
    std::vector<double> L((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) L[(size_t)i * n + A.col[k]] = A.val[k];
    double amax = 0;
    for (double v : L) amax = std::max(amax, std::fabs(v));
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j)
            if (std::fabs(L[(size_t)i * n + j] - L[(size_t)j * n + i]) > 1e-12 * amax)
                fail(AMGE_ERR_NOT_SPD, "coarsest matrix is not symmetric");
    // Cholesky A = L L^T (lower, in place)
    for (int j = 0; j < n; ++j) {
        double d = L[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) d -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
        if (!(d > 0)) fail(AMGE_ERR_NOT_SPD, "coarsest matrix is not positive definite");
        d = std::sqrt(d);
        L[(size_t)j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            double v = L[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) v -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
            L[(size_t)i * n + j] = v / d;
        }
    }
    // W = L^{-1} (lower triangular), by forward substitution on the identity
    std::vector<double> W((size_t)n * n, 0.0);
    for (int c = 0; c < n; ++c)
        for (int i = c; i < n; ++i) {
            double v = (i == c) ? 1.0 : 0.0;
            for (int k = c; k < i; ++k) v -= L[(size_t)i * n + k] * W[(size_t)k * n + c];
            W[(size_t)i * n + c] = v / L[(size_t)i * n + i];
        }
    // A^{-1} = W^T W (symmetric), applied on the device as one dense product
    std::vector<double> Ainv((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j <= i; ++j) {
            double v = 0;
            for (int k = i; k < n; ++k) v += W[(size_t)k * n + i] * W[(size_t)k * n + j];
            Ainv[(size_t)i * n + j] = v;
            Ainv[(size_t)j * n + i] = v;
        }
    H->nc = n;
    H->Ainv = upload(H, Ainv.data(), Ainv.size(), s);
    HIPCHECK(hipStreamSynchronize(s));
    ainv.swap(Ainv);
}

// l1 scalings of a level (read-only, in the hierarchy): dinv = 1 / d, dhinv = 1 / dhat.
template <class T>
void upload_scalings(amge_hierarchy* H, Work<T>& w, const std::vector<double>& dinv,
                     const std::vector<double>& dhinv, hipStream_t s) {
    std::vector<T> a(dinv.begin(), dinv.end()), c(dhinv.begin(), dhinv.end());
    w.dinv = upload(H, a.data(), a.size(), s);
    w.dhinv = upload(H, c.data(), c.size(), s);
    HIPCHECK(hipStreamSynchronize(s));
}

// Single-column work vectors of one level (context state); the scalings stay shared.
template <class T>
void alloc_work(amge_hierarchy* C, DLevel& L, Work<T>& w) {
    size_t nr = (size_t)L.n, mr = (size_t)L.m;
    w.b = C->alloc<T>(nr);
    w.x = C->alloc<T>(nr);
    w.xt = C->alloc<T>(nr);
    w.r = C->alloc<T>(nr);
    w.g = C->alloc<T>(mr);
    w.y = C->alloc<T>(mr);
    w.yt = C->alloc<T>(mr);
    w.bd = C->alloc<T>(nr);
    w.gd = C->alloc<T>(mr);
}

// Batched work block of one level (n x NC, m x NC) in the preconditioner precision;
// the l1 scalings are shared with the single-column buffers.
template <class T>
void alloc_bwork(amge_hierarchy* H, DLevel& L, const Work<T>& w1, Work<T>& w) {
    const size_t nr = (size_t)L.n * H->NC, mr = (size_t)L.m * H->NC;
    w.b = H->alloc<T>(nr);
    w.x = H->alloc<T>(nr);
    w.xt = H->alloc<T>(nr);
    w.r = H->alloc<T>(nr);
    w.bd = H->alloc<T>(nr);
    if (mr) {
        w.g = H->alloc<T>(mr);
        w.y = H->alloc<T>(mr);
        w.yt = H->alloc<T>(mr);
        w.gd = H->alloc<T>(mr);
    }
    w.dinv = w1.dinv;
    w.dhinv = w1.dhinv;
}

// Level matrices kept on the host during set-up for the batched uploads.
struct HostLevel {
    Csr A, Ah, P, Pt, Aux, D;
    std::vector<int> aux_lead;   // split rows of Aux: entries of D^T per row
};

template <class T>
void tune_batched(amge_hierarchy* H, hipStream_t s) {
    size_t mx = 0, my = 0;
    for (DLevel& L : H->lv)
        for (DSellB* M : {&L.bA, &L.bAh, &L.bP, &L.bPt, &L.bAux, &L.bD})
            if (M->nrows) {
                mx = std::max(mx, (size_t)M->ncols * H->NC);
                my = std::max(my, (size_t)M->nrows * H->NC);
            }
    if (!mx) return;
    amge_hierarchy tmp;   // owns the trial buffers
    tmp.opts = H->opts;
    T* X = tmp.alloc<T>(mx);
    T* Y = tmp.alloc<T>(my);
    HIPCHECK(hipMemsetAsync(X, 0, sizeof(T) * mx, s));
    HIPCHECK(hipMemsetAsync(Y, 0, sizeof(T) * my, s));
    for (DLevel& L : H->lv) {
        for (DSellB* M : {&L.bA, &L.bAh, &L.bP, &L.bPt, &L.bAux})
            if (M->nrows) tune_cols<T>(*M, false, H->NC, X, Y, H->zero_flag, s);
        if (L.bD.nrows) tune_cols<T>(L.bD, true, H->NC, X, Y, H->zero_flag, s);
    }
    HIPCHECK(hipStreamSynchronize(s));
}

void setup_batched(amge_hierarchy* H, const std::vector<HostLevel>& hl, hipStream_t s) {
    int NC = 2, lg = 1;
    while (NC < H->opts.max_rhs) {
        NC *= 2;
        ++lg;
    }
    H->NC = NC;
    H->lgNC = lg;
    const bool f32 = H->opts.precond_bits == 32;
    const int nl = (int)H->lv.size();
    for (int k = 0; k < nl; ++k) {
        DLevel& L = H->lv[k];
        const HostLevel& h = hl[k];
        if (k < nl - 1 || nl == 1) {
            // A_1 is also the outer PCG operator (FP64)
            L.bA = upload_sell_b(H, h.A, false, f32, !f32 || k == 0, s);
        }
        if (k < nl - 1) {
            L.bAh = upload_sell_b(H, h.Ah, false, f32, !f32, s);
            L.bP = upload_sell_b(H, h.P, false, f32, !f32, s);
            L.bPt = upload_sell_b(H, h.Pt, false, f32, !f32, s);
            L.bAux = upload_sell_b(H, h.Aux, false, f32, !f32, s, &h.aux_lead);
            L.bD = upload_sell_b(H, h.D, true, false, false, s);
        }
    }
    if (f32 && nl > 1) tune_batched<float>(H, s);
    else tune_batched<double>(H, s);
}

// Cancellation factor of the auxiliary matrix on one level:
//   max_e (|D|^T |A| |D| 1)_e / (|D^T A D| 1)_e.
// D^T A D only keeps the mass part of A (the derivative part vanishes on the range of
// D), so applying A to a vector near that range cancels terms up to this factor larger
// than the result.  Evaluated in a precision with unit roundoff u, such products carry
// relative errors up to u * kappa in exactly the components the auxiliary space of the
// smoother and the coarse levels must resolve.
double cancellation_factor(const Csr& A, const Csr& D, const Csr& Dt, const std::vector<double>& dh) {
    const std::vector<double> v = l1_row_sums(D);
    std::vector<double> w(A.nrows, 0.0);
    for (int i = 0; i < A.nrows; ++i)
        for (int k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) w[i] += std::fabs(A.val[k]) * v[A.col[k]];
    double kap = 1.0;
    for (int e = 0; e < Dt.nrows; ++e) {
        double num = 0;
        for (int k = Dt.rowptr[e]; k < Dt.rowptr[e + 1]; ++k) num += std::fabs(Dt.val[k]) * w[Dt.col[k]];
        if (dh[e] > 0) kap = std::max(kap, num / dh[e]);
    }
    return kap;
}

amge_status pcg(amge_hierarchy* H, const double* b, double* x, double rtol, int maxit, int stop_l2, int* iters,
                double* relres, hipStream_t s);

// Automatic V-cycle precision (opts.precond_bits = 0): trial PCG solves on a fixed
// pseudo-random right-hand side (uniform in [-1, 1), splitmix64 of the row index), to
// rtol 1e-8 in the preconditioner norm.  An FP32 V-cycle is kept when it converges within
// AUTO_FP32_EXTRA iterations of the FP64 one: first with the FP32 fine-level residual,
// then with the FP64 one.  Neither the cancellation factor nor the FP32 cycle's deviation
// on one vector predicts this: on the jump workloads the all-FP32 cycle costs nothing on
// every H(div) hierarchy up to n = 32 (kappa 5.5e7) but 60 % more iterations on an
// H(curl) one with n = 24 (kappa 2.5e7), and stalls at n >= 48; with the fine-level
// residual in FP64 it takes the FP64 iteration count on those too.
constexpr int AUTO_FP32_EXTRA = 3;
constexpr double AUTO_TRIAL_RTOL = 1e-8;
constexpr int AUTO_TRIAL_MAXIT = 1000;

// Returns {precond_bits, resid_bits}.
std::pair<int, int> trial_precision(amge_hierarchy* H, hipStream_t s) {
    if (H->lv.size() < 2) return {64, 64};   // no V-cycle: the preconditioner is the FP64 coarse solve
    const int n = H->lv[0].n;
    std::vector<double> b(n);
    for (int i = 0; i < n; ++i) {
        uint64_t z = (uint64_t)i * 0x9e3779b97f4a7c15ull + 0x632be59bd9b4e019ull;
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        z ^= z >> 31;
        b[i] = (double)(z >> 11) * 0x1.0p-52 - 1.0;
    }
    amge_hierarchy tmp;   // the trial vectors, through the caller's allocator
    tmp.opts = H->opts;
    double* db = tmp.alloc<double>(n);
    double* dx = tmp.alloc<double>(n);
    HIPCHECK(hipMemcpyAsync(db, b.data(), sizeof(double) * n, hipMemcpyHostToDevice, s));
    // candidates in order: FP64; FP32 with the FP32 fine-level residual; FP32 with the
    // FP64 one.  The first FP32 candidate within AUTO_FP32_EXTRA iterations of FP64 wins.
    const int bits[3] = {64, 32, 32}, resid[3] = {64, 32, 64};
    int it64 = -1;
    for (int p = 0; p < 3; ++p) {
        H->opts.precond_bits = bits[p];
        H->lv[0].resid64 = resid[p] == 64 && bits[p] == 32;
        const int maxit = p ? it64 + AUTO_FP32_EXTRA : AUTO_TRIAL_MAXIT;
        int it = 0;
        double rr = 0;
        amge_status st = AMGE_ERR_BREAKDOWN;
        try {
            auto C = make_ctx(H, 1);
            st = pcg(&C->st, db, dx, AUTO_TRIAL_RTOL, maxit, 0, &it, &rr, s);
        } catch (const Error& e) {
            if (e.code == AMGE_ERR_OOM || e.code == AMGE_ERR_HIP) throw;
        }
        const int its = st == AMGE_OK ? it : -1;
        if (verbose())
            fprintf(stderr, "[amge precision] FP%d trial (fine residual FP%d): %d iterations (status %d)\n", bits[p],
                    resid[p], it, (int)st);
        H->lv[0].resid64 = false;
        H->opts.precond_bits = 0;
        if (p == 0) {
            if (its < 0) return {64, 64};   // FP64 itself did not converge: keep FP64
            it64 = its;
        } else if (its >= 0 && its <= it64 + AUTO_FP32_EXTRA) {
            return {32, resid[p]};
        }
    }
    return {64, 64};
}

// ------------------------------------------------------------------ coarse-tail folding
// With a zero initial guess the V-cycle from level l down is a fixed linear map B_l of
// the level's right-hand side.  While the level above the current tail (first the
// coarsest level, B = A^{-1}) is not the fine level and has at most opts.tail_rows rows,
// B_l is formed at set-up, one unit vector at a time, by an FP64 host evaluation of the
// V-cycle at level l (the steps of vcycle_level) around the dense B of the level below;
// the single-column V-cycle then applies it as one dense FP64 product (k_coarse), the
// same operator in one launch instead of every launch of those levels.

std::vector<int> greedy_colors(const Csr& A);

// Host copy of a level that may be folded.
struct TailLevel {
    Csr A, D, Dt, DtA, Ah, P, Pt;
    std::vector<double> dinv, dhinv;
    // symmetric Gauss-Seidel smoother: rows of every colour, 1 / a_ii (A and D^T A D)
    bool gs = false;
    std::vector<std::vector<int>> clsA, clsAh;
    std::vector<double> dgA, dgAh;
    // l1-scaled symmetric block Gauss-Seidel smoother (A and D^T A D)
    bool bgs = false;
    BgsHost bgA, bgAh;
};

// Rows of every colour, and 1 / a_ii, of a matrix (host Gauss-Seidel of the folded tail).
void host_gs_data(const Csr& A, std::vector<std::vector<int>>& cls, std::vector<double>& dg) {
    const std::vector<int> color = greedy_colors(A);
    int C = 0;
    for (int c : color) C = std::max(C, c + 1);
    cls.assign(C, {});
    for (int i = 0; i < A.nrows; ++i) cls[color[i]].push_back(i);
    dg.assign(A.nrows, 0.0);
    for (int i = 0; i < A.nrows; ++i)
        for (int q = A.rowptr[i]; q < A.rowptr[i + 1]; ++q)
            if (A.col[q] == i) dg[i] = 1.0 / A.val[q];
}

namespace {

void host_spmv(const Csr& M, const double* x, double* y) {
    for (int i = 0; i < M.nrows; ++i) {
        double a = 0;
        for (int q = M.rowptr[i]; q < M.rowptr[i + 1]; ++q) a += M.val[q] * x[M.col[q]];
        y[i] = a;
    }
}

struct TailScratch {
    std::vector<double> ax, g, y, ay, r, bc, xc;
    TailScratch(int n, int m, int nc) : ax(n), g(m), y(m), ay(m), r(n), bc(nc), xc(nc) {}
};

// nu symmetric Gauss-Seidel sweeps in colour order on x, with the colour sequence of
// gs_sweeps (the colour that ends a half-sweep is not relaxed again).
void host_gs(const Csr& A, const std::vector<std::vector<int>>& cls, const std::vector<double>& dg, int nu,
             const double* b, double* x) {
    const int C = (int)cls.size();
    if (nu <= 0 || C == 0) return;
    auto relax = [&](int c) {
        for (int i : cls[c]) {
            double a = 0;
            for (int q = A.rowptr[i]; q < A.rowptr[i + 1]; ++q) a += A.val[q] * x[A.col[q]];
            x[i] += dg[i] * (b[i] - a);
        }
    };
    relax(0);
    for (int k = 0; k < nu; ++k) {
        for (int c = 1; c < C; ++c) relax(c);
        for (int c = C - 2; c >= 0; --c) relax(c);
    }
}

// nu l1-Jacobi sweeps x <- x + dinv (b - A x)
void host_sweeps(const TailLevel& L, int nu, const double* b, double* x, TailScratch& w) {
    const int n = L.A.nrows;
    for (int k = 0; k < nu; ++k) {
        host_spmv(L.A, x, w.ax.data());
        for (int i = 0; i < n; ++i) x[i] += L.dinv[i] * (b[i] - w.ax[i]);
    }
}

// x <- x + D Mhat^{-1} (D^T b - (D^T A) x), Mhat^{-1}: nua sweeps on D^T A D from zero
void host_aux(const TailLevel& L, int nua, const double* b, double* x, TailScratch& w) {
    const int n = L.A.nrows, m = L.D.ncols;
    if (nua <= 0 || m == 0) return;
    host_spmv(L.Dt, b, w.g.data());
    host_spmv(L.DtA, x, w.ay.data());
    for (int i = 0; i < m; ++i) w.g[i] -= w.ay[i];
    if (L.gs) {
        std::fill(w.y.begin(), w.y.end(), 0.0);
        host_gs(L.Ah, L.clsAh, L.dgAh, nua, w.g.data(), w.y.data());
    } else if (L.bgs) {
        std::fill(w.y.begin(), w.y.end(), 0.0);
        for (int k = 0; k < nua; ++k) host_bgs_sweep(L.bgAh, w.g.data(), w.y.data(), w.ay);
    } else {
        for (int i = 0; i < m; ++i) w.y[i] = L.dhinv[i] * w.g[i];
        for (int k = 1; k < nua; ++k) {
            host_spmv(L.Ah, w.y.data(), w.ay.data());
            for (int i = 0; i < m; ++i) w.y[i] += L.dhinv[i] * (w.g[i] - w.ay[i]);
        }
    }
    host_spmv(L.D, w.y.data(), w.ax.data());
    for (int i = 0; i < n; ++i) x[i] += w.ax[i];
}

// x = V-cycle at level L applied to b, with the dense operator Bc (nc x nc) below
void host_tail_vcycle(const TailLevel& L, int nu, int nua, const std::vector<double>& Bc, int nc,
                      const double* b, double* x, TailScratch& w) {
    const int n = L.A.nrows;
    if (L.gs) {
        std::fill(x, x + n, 0.0);
        host_gs(L.A, L.clsA, L.dgA, nu, b, x);
    } else if (L.bgs) {
        std::fill(x, x + n, 0.0);
        for (int k = 0; k < nu; ++k) host_bgs_sweep(L.bgA, b, x, w.r);
    } else if (nu >= 1) {   // the first sweep from zero is dinv b
        for (int i = 0; i < n; ++i) x[i] = L.dinv[i] * b[i];
        host_sweeps(L, nu - 1, b, x, w);
    } else {
        std::fill(x, x + n, 0.0);
    }
    host_aux(L, nua, b, x, w);
    host_spmv(L.A, x, w.ax.data());
    for (int i = 0; i < n; ++i) w.r[i] = b[i] - w.ax[i];
    host_spmv(L.Pt, w.r.data(), w.bc.data());
    for (int i = 0; i < nc; ++i) {
        double a = 0;
        for (int j = 0; j < nc; ++j) a += Bc[(size_t)i * nc + j] * w.bc[j];
        w.xc[i] = a;
    }
    host_spmv(L.P, w.xc.data(), w.ax.data());
    for (int i = 0; i < n; ++i) x[i] += w.ax[i];
    host_aux(L, nua, b, x, w);
    if (L.gs) host_gs(L.A, L.clsA, L.dgA, nu, b, x);
    else if (L.bgs)
        for (int k = 0; k < nu; ++k) host_bgs_sweep(L.bgA, b, x, w.r);
    else host_sweeps(L, nu, b, x, w);
}

}  // namespace

// tl: host copies of the levels that may be folded; ainv: the coarsest inverse (row-major)
void fold_tail(amge_hierarchy* H, const std::vector<TailLevel>& tl, const std::vector<double>& ainv,
               hipStream_t s) {
    const int lim = H->opts.tail_rows, nl = (int)H->lv.size();
    const int nu = H->opts.nu_primary, nua = H->opts.nu_aux;
    int t = nl - 1, nb = H->nc;
    std::vector<double> B = ainv;
    while (lim > 0 && t >= 2 && H->lv[t - 1].n <= lim) {
        const TailLevel& L = tl[t - 1];
        const int n = L.A.nrows, m = L.D.ncols;
        std::vector<double> Bl((size_t)n * n);
        const int nthr = std::max(1, std::min(16, (int)std::thread::hardware_concurrency()));
        std::vector<std::thread> pool;
        std::vector<std::exception_ptr> err(nthr);   // carried to this thread, rethrown after the join
        for (int id = 0; id < nthr; ++id)
            pool.emplace_back([&, id]() {
                try {
                    TailScratch w(n, m, nb);
                    std::vector<double> e(n, 0.0), x(n);
                    for (int i = id; i < n; i += nthr) {   // column i = B_l e_i
                        e[i] = 1.0;
                        host_tail_vcycle(L, nu, nua, B, nb, e.data(), x.data(), w);
                        e[i] = 0.0;
                        for (int j = 0; j < n; ++j) Bl[(size_t)j * n + i] = x[j];
                    }
                } catch (...) {
                    err[id] = std::current_exception();
                }
            });
        for (std::thread& th : pool) th.join();
        for (auto& e : err)
            if (e) std::rethrow_exception(e);
        B.swap(Bl);
        nb = n;
        t -= 1;
    }
    if (t == nl - 1) return;
    for (double v : B)
        if (!std::isfinite(v)) fail(AMGE_ERR_NONFINITE, "non-finite folded coarse tail");
    H->tail = t;
    H->tail_n = nb;
    H->tail_op = upload(H, B.data(), B.size(), s);
    HIPCHECK(hipStreamSynchronize(s));
}

// Greedy colouring: row i takes the smallest colour not held by an earlier row j < i
// with a_ij != 0.
std::vector<int> greedy_colors(const Csr& A) {
    std::vector<int> color(A.nrows, -1), mark;
    for (int i = 0; i < A.nrows; ++i) {
        for (int q = A.rowptr[i]; q < A.rowptr[i + 1]; ++q) {
            const int j = A.col[q];
            if (j >= i || A.val[q] == 0.0) continue;
            if (color[j] >= (int)mark.size()) mark.resize(color[j] + 1, -1);
            mark[color[j]] = i;
        }
        int c = 0;
        while (c < (int)mark.size() && mark[c] == i) ++c;
        color[i] = c;
    }
    return color;
}

// Multicolour Gauss-Seidel data of A: the rows of every colour as their own sliced ELL
// (lanes per row tuned per colour) and 1 / a_ii in both precisions.
void build_gs(amge_hierarchy* H, const Csr& A, GsColors& g, hipStream_t s) {
    const std::vector<int> color = greedy_colors(A);
    int C = 0;
    for (int c : color) C = std::max(C, c + 1);
    std::vector<std::vector<int>> rows(C);
    for (int i = 0; i < A.nrows; ++i) rows[color[i]].push_back(i);
    std::vector<double> dg(A.nrows, 0.0);
    for (int i = 0; i < A.nrows; ++i) {
        for (int q = A.rowptr[i]; q < A.rowptr[i + 1]; ++q)
            if (A.col[q] == i) dg[i] = A.val[q];
        if (!(dg[i] > 0)) fail(AMGE_ERR_NOT_SPD, "Gauss-Seidel needs a positive diagonal");
        dg[i] = 1.0 / dg[i];
    }
    for (int c = 0; c < C; ++c) {
        Csr S;
        S.nrows = (int32_t)rows[c].size();
        S.ncols = A.ncols;
        for (int i : rows[c]) {
            for (int q = A.rowptr[i]; q < A.rowptr[i + 1]; ++q) {
                S.col.push_back(A.col[q]);
                S.val.push_back(A.val[q]);
            }
            S.rowptr.push_back((int32_t)S.col.size());
        }
        g.col.push_back(upload_sell(H, S, false, tune_lanes(S, false, H->opts, s), s, nullptr, &rows[c]));
    }
    std::vector<float> dg32(dg.begin(), dg.end());
    g.dg64 = upload(H, dg.data(), dg.size(), s);
    g.dg32 = upload(H, dg32.data(), dg32.size(), s);
    HIPCHECK(hipStreamSynchronize(s));
}

// Wall-clock phases of set-up, printed with AMGE_VERBOSE.
struct PhaseClock {
    std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
    std::map<std::string, double> ms;
    void lap(const char* name) {
        auto now = std::chrono::steady_clock::now();
        ms[name] += std::chrono::duration<double, std::milli>(now - t).count();
        t = now;
    }
    ~PhaseClock() {
        if (!verbose()) return;
        for (auto& kv : ms) fprintf(stderr, "[amge setup] %-28s %9.1f ms\n", kv.first.c_str(), kv.second);
    }
};

void setup(amge_hierarchy* H, const amge_level* levels, int nl, hipStream_t s) {
    if (!levels || nl < 1) fail(AMGE_ERR_ARG, "need at least one level");
    PhaseClock clk;
    std::vector<Csr> A(nl), D(nl), P(nl);
    for (int k = 0; k < nl; ++k) {
        A[k] = csr_from_view(levels[k].A);
        if (A[k].nrows != A[k].ncols || A[k].nrows == 0) fail(AMGE_ERR_SHAPE, "A_k must be square and non-empty");
        if (k > 0 && A[k].nrows != P[k - 1].ncols) fail(AMGE_ERR_SHAPE, "P_{k-1} columns != rows of A_k");
        if (k < nl - 1) {
            D[k] = csr_from_view(levels[k].D);
            if (D[k].nrows != A[k].nrows) fail(AMGE_ERR_SHAPE, "D_k rows != rows of A_k");
            P[k] = csr_from_view(levels[k].P);
            if (P[k].nrows != A[k].nrows) fail(AMGE_ERR_SHAPE, "P_k rows != rows of A_k");
        }
    }
    H->lv.resize(nl);
    H->zero_flag = H->alloc<int>(1);
    HIPCHECK(hipMemsetAsync(H->zero_flag, 0, sizeof(int), s));
    const bool batched = H->opts.max_rhs > 1;
    std::vector<HostLevel> hl(batched ? nl : 0);
    std::vector<TailLevel> tl(nl);   // host copies of the levels that may be folded
    std::vector<double> ainv;
    for (int k = 0; k < nl; ++k) {
        DLevel& L = H->lv[k];
        L.n = A[k].nrows;
        if (batched) hl[k].A = A[k];
        if (k == nl - 1) {
            build_coarse(H, A[k], s, ainv);
            continue;
        }
        L.m = D[k].ncols;
        clk.lap("other per-level work");
        Csr Dt = transpose(D[k]);
        // D^T A (for the auxiliary residual) and the auxiliary matrix D^T A D (eq. (4.1))
        auto [DtA, Ah] = chain_on_device(Dt, A[k], D[k], s, &H->opts);
        std::vector<double> d = l1_row_sums(A[k]), dh = l1_row_sums(Ah);
        H->kappa = std::max(H->kappa, cancellation_factor(A[k], D[k], Dt, dh));
        std::vector<double> dinv(d.size()), dhinv(dh.size());
        for (size_t i = 0; i < d.size(); ++i) {
            if (!(d[i] > 0)) fail(AMGE_ERR_NOT_SPD, "zero row in A_k");
            dinv[i] = 1.0 / d[i];
        }
        for (size_t i = 0; i < dh.size(); ++i) dhinv[i] = dh[i] > 0 ? 1.0 / dh[i] : 0.0;
        if (k >= 1 && A[k].nrows <= H->opts.tail_rows) {
            TailLevel& T = tl[k];
            T.A = A[k];
            T.D = D[k];
            T.Dt = Dt;
            T.DtA = DtA;
            T.Ah = Ah;
            T.P = P[k];
            T.Pt = transpose(P[k]);
            T.dinv = dinv;
            T.dhinv = dhinv;
            if (H->opts.smoother == AMGE_SMOOTHER_SYM_GS) {
                T.gs = true;
                host_gs_data(A[k], T.clsA, T.dgA);
                host_gs_data(Ah, T.clsAh, T.dgAh);
            } else if (H->opts.smoother == AMGE_SMOOTHER_BLOCK_GS) {
                T.bgs = true;
                T.bgA = bgs_layout(A[k]);
                T.bgAh = bgs_layout(Ah);
            }
        }
        clk.lap("host products D^T A, D^T A D");
        L.A = upload_tuned(H, A[k], false, s);
        L.Ah = upload_tuned(H, Ah, false, s);
        clk.lap("layouts+tuning A, D^T A D");
        if (H->opts.smoother == AMGE_SMOOTHER_SYM_GS) {
            build_gs(H, A[k], L.gsA, s);
            build_gs(H, Ah, L.gsAh, s);
        } else if (H->opts.smoother == AMGE_SMOOTHER_BLOCK_GS) {
            build_bgs(H, A[k], L.bgA, s);
            build_bgs(H, Ah, L.bgAh, s);
            clk.lap("block Gauss-Seidel layouts");
        }
        L.P = upload_tuned(H, P[k], false, s);
        L.Pt = upload_tuned(H, transpose(P[k]), false, s);
        clk.lap("layouts+tuning P, P^T");
        // every operator but A_k streamed past the caches (A_k is used four times)
        L.Ah.stream = L.P.stream = L.Pt.stream = true;
        L.D = upload_incidence(H, D[k], s);
        L.Dt = upload_tuned(H, Dt, true, s);
        {
            // [D^T | -D^T A] acting on [b; x]: split rows, the D^T entries of a row first
            // (they read b), then those of -D^T A (they read x); both index 0..n-1, so the
            // 16-bit column offsets apply as for A_k
            Csr X;
            X.nrows = L.m;
            X.ncols = L.n;
            X.rowptr.assign(L.m + 1, 0);
            std::vector<int> lead(L.m);
            for (int i = 0; i < L.m; ++i) {
                for (int q = Dt.rowptr[i]; q < Dt.rowptr[i + 1]; ++q) {
                    X.col.push_back(Dt.col[q]);
                    X.val.push_back(Dt.val[q]);
                }
                lead[i] = Dt.rowptr[i + 1] - Dt.rowptr[i];
                for (int q = DtA.rowptr[i]; q < DtA.rowptr[i + 1]; ++q) {
                    X.col.push_back(DtA.col[q]);
                    X.val.push_back(-DtA.val[q]);
                }
                X.rowptr[i + 1] = (int32_t)X.col.size();
            }
            clk.lap("other per-level work");
            L.Aux = upload_tuned(H, X, false, s, &lead);
            L.Aux.stream = true;
            clk.lap("layouts+tuning aux residual");
            if (k >= 1) {
                // [P^T | -P^T A] on [b; x] below the fine level: the restricted residual
                // P^T (b - A x) in one (latency-bound) launch instead of a residual and a
                // restriction.  On the fine level the residual reads the cache-resident
                // A_k and stays separate.
                const Csr Pt = transpose(P[k]);
                const Csr PtA = spgemm_on_device(Pt, A[k], s, &H->opts);
                Csr R;
                R.nrows = Pt.nrows;
                R.ncols = L.n;
                R.rowptr.assign(Pt.nrows + 1, 0);
                std::vector<int> rlead(Pt.nrows);
                for (int i = 0; i < Pt.nrows; ++i) {
                    for (int q = Pt.rowptr[i]; q < Pt.rowptr[i + 1]; ++q) {
                        R.col.push_back(Pt.col[q]);
                        R.val.push_back(Pt.val[q]);
                    }
                    rlead[i] = Pt.rowptr[i + 1] - Pt.rowptr[i];
                    for (int q = PtA.rowptr[i]; q < PtA.rowptr[i + 1]; ++q) {
                        R.col.push_back(PtA.col[q]);
                        R.val.push_back(-PtA.val[q]);
                    }
                    R.rowptr[i + 1] = (int32_t)R.col.size();
                }
                clk.lap("host products P^T A");
                L.PtA = upload_tuned(H, R, false, s, &rlead);
                L.PtA.stream = true;
                clk.lap("layouts+tuning restriction");
            }
            if (batched) {
                hl[k].Ah = Ah;
                hl[k].P = P[k];
                hl[k].Pt = transpose(P[k]);
                hl[k].Aux = std::move(X);
                hl[k].aux_lead = std::move(lead);
                hl[k].D = D[k];
            }
        }
        upload_scalings<float>(H, L.w32, dinv, dhinv, s);
        upload_scalings<double>(H, L.w64, dinv, dhinv, s);
    }
    if (nl == 1) {
        // the fine matrix itself is needed by the outer PCG even on one level
        H->lv[0].A = upload_tuned(H, A[0], false, s);
    }
    H->tail = nl - 1;
    H->tail_n = H->nc;
    H->tail_op = H->Ainv;
    clk.lap("other per-level work");
    fold_tail(H, tl, ainv, s);
    clk.lap("folded coarse tail");
    if (H->opts.precond_bits == 0) {
        const std::pair<int, int> pr = trial_precision(H, s);
        H->opts.precond_bits = pr.first;
        H->opts.resid_bits = pr.second;
    }
    if (H->opts.resid_bits == 0) H->opts.resid_bits = 32;
    H->lv[0].resid64 = H->opts.precond_bits == 32 && H->opts.resid_bits == 64 && H->lv.size() > 1;
    clk.lap("precision trial");
    if (batched) setup_batched(H, hl, s);
    clk.lap("batched layouts, tuning");
    if (batched) {
        if (H->opts.precond_bits == 32 && H->lv.size() > 1) tune_tail<float>(H, s);
        else tune_tail<double>(H, s);
    }
    HIPCHECK(hipStreamSynchronize(s));
}

// ------------------------------------------------------------------ contexts
// Execution state S of hierarchy P for nrhs columns: P's operator descriptors and
// scalings (P's device memory; P holds no work buffers, so every work pointer copied
// here is null), then the single-column level work in the V-cycle precision from S's
// own allocator (an arena, the caller's allocator or hipMalloc).
void init_state(amge_hierarchy* S, const amge_hierarchy* P, int nrhs) {
    S->opts = P->opts;
    S->parent = P;
    S->nrhs_cap = nrhs;
    S->lv = P->lv;
    for (DLevel& L : S->lv) L.probe = nullptr;
    S->nc = P->nc;
    S->kappa = P->kappa;
    S->Ainv = P->Ainv;
    S->tail = P->tail;
    S->tail_n = P->tail_n;
    S->tail_op = P->tail_op;
    S->tail_rpb = P->tail_rpb;
    S->zero_flag = P->zero_flag;
    const bool f32 = S->opts.precond_bits == 32 && S->lv.size() > 1;
    for (DLevel& L : S->lv) {
        if (f32) alloc_work<float>(S, L, L.w32);
        else alloc_work<double>(S, L, L.w64);
    }
}

std::unique_ptr<amge_ctx> make_ctx(const amge_hierarchy* P, int nrhs, bool dry) {
    if (!P || P->parent) fail(AMGE_ERR_ARG, "not a hierarchy");
    if (nrhs < 1 || nrhs > P->opts.max_rhs) fail(AMGE_ERR_ARG, "a context needs 1 <= nrhs <= max_rhs of its hierarchy");
    auto C = std::make_unique<amge_ctx>();
    amge_hierarchy* S = &C->st;
    S->dry = dry;
    init_state(S, P, nrhs);
    const bool f32 = S->opts.precond_bits == 32 && S->lv.size() > 1;
    // outer PCG (FP64, level-1 length) and its partial sums
    const size_t n1 = (size_t)S->lv[0].n;
    S->r = S->alloc<double>(n1);
    S->p = S->alloc<double>(n1);
    S->q = S->alloc<double>(n1);
    S->z[0] = S->alloc<double>(n1);
    S->z[1] = S->alloc<double>(n1);
    S->x = S->alloc<double>(n1);
    S->part_pq = S->alloc<double>(dev::NRED);
    S->part_dots[0] = S->alloc<double>(3 * dev::NRED);
    S->part_dots[1] = S->alloc<double>(3 * dev::NRED);
    S->st = S->alloc<dev::PcgStatus>(1);
    S->flags = S->alloc<int>(4);
    if (nrhs > 1) {
        int NC = 2, lg = 1;
        while (NC < nrhs) {
            NC *= 2;
            ++lg;
        }
        S->NC = NC;
        S->lgNC = lg;
        for (DLevel& L : S->lv) {
            if (f32) alloc_bwork<float>(S, L, L.w32, L.bw32);
            else alloc_bwork<double>(S, L, L.w64, L.bw64);
        }
        const size_t nn = n1 * NC;
        S->bX = S->alloc<double>(nn);
        S->bR = S->alloc<double>(nn);
        S->bP = S->alloc<double>(nn);
        S->bQ = S->alloc<double>(nn);
        // the two z blocks (new and old, alternating with the iteration parity): FP64
        // blocks bZ and bZv, or, for an FP32 V-cycle, the two halves of bZ
        S->bZ = S->alloc<double>(nn);
        S->bZv = S->alloc<double>(nn);
        S->bpart = S->alloc<double>((size_t)3 * NC * BPCG_BLOCKS);
        S->cs = S->alloc<dev::ColState>(NC);
        S->bs = S->alloc<dev::BatchStatus>(1);
    } else {
        S->NC = 1;
        S->lgNC = 0;
    }
    if (!dry) {
        HIPCHECK(hipStreamCreateWithFlags(&S->gstream, hipStreamNonBlocking));
        HIPCHECK(hipEventCreateWithFlags(&S->ev_in, hipEventDisableTiming));
        HIPCHECK(hipEventCreateWithFlags(&S->ev_out, hipEventDisableTiming));
        for (hipEvent_t& e : S->pev) HIPCHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        HIPCHECK(hipHostMalloc((void**)&S->ring, sizeof(dev::PcgRecord) * dev::PCG_RING,
                               hipHostMallocMapped | hipHostMallocCoherent));
        memset((void*)S->ring, 0, sizeof(dev::PcgRecord) * dev::PCG_RING);
        HIPCHECK(hipHostGetDevicePointer((void**)&S->ring_dev, S->ring, 0));
    }
    return C;
}

// ------------------------------------------------------------------ PCG
template <int K, int UNR>
void pcg_ap_ku(amge_hierarchy* H, hipStream_t s) {
    const DSell& A = H->lv[0].A;
    if (A.c16)
        dev::k_pcg_ap<K, true, UNR><<<dev::NRED, BLOCK, 0, s>>>(A.nslices, A.sptr, A.srow, A.ci, A.c16, A.cbase,
                                                                A.v64, H->p, H->q, H->part_pq, H->flags);
    else
        dev::k_pcg_ap<K, false, UNR><<<dev::NRED, BLOCK, 0, s>>>(A.nslices, A.sptr, A.srow, A.ci, A.c16, A.cbase,
                                                                 A.v64, H->p, H->q, H->part_pq, H->flags);
}

template <int K>
void pcg_ap_k(amge_hierarchy* H, hipStream_t s) {
    if constexpr (K == 1) {
        if (H->lv[0].A.deep) {
            pcg_ap_ku<1, 8>(H, s);
            return;
        }
    }
    pcg_ap_ku<K, 4>(H, s);
}

void launch_pcg_ap(amge_hierarchy* H, hipStream_t s) {
    switch (H->lv[0].A.K) {
        case 1: pcg_ap_k<1>(H, s); break;
        case 2: pcg_ap_k<2>(H, s); break;
        case 4: pcg_ap_k<4>(H, s); break;
        case 8: pcg_ap_k<8>(H, s); break;
        case 16: pcg_ap_k<16>(H, s); break;
        case 32: pcg_ap_k<32>(H, s); break;
        default: pcg_ap_k<64>(H, s); break;
    }
}

// One PCG iteration with buffer parity `par` (z and the dot partials alternate between
// iterations): q = A p and p.q; x, r update with the preconditioner input; z = B r;
// dots; beta, p update and the stopping test.  Every launch returns at once after
// convergence (device flag), so iterations can be queued ahead of the test.
void pcg_iteration(amge_hierarchy* H, int par, hipStream_t s) {
    const int n = H->lv[0].n;
    const bool f32 = H->opts.precond_bits == 32;
    const bool multilevel = H->lv.size() > 1;
    DLevel& L1 = H->lv[0];
    float* r32 = f32 && multilevel ? L1.w32.b : nullptr;
    float* rd32 = f32 && multilevel ? L1.w32.bd : nullptr;
    double* rd64 = !f32 && multilevel ? L1.w64.bd : nullptr;
    const int* done = H->flags;
    double* znew = H->z[par];
    double* zold = H->z[par ^ 1];
    double* dnew = H->part_dots[par];
    double* dold = H->part_dots[par ^ 1];
    launch_pcg_ap(H, s);
    dev::k_pcg_xr<<<dev::NRED, BLOCK, 0, s>>>(n, H->part_pq, dold, H->p, H->q, H->x, H->r, r32, rd32,
                                              f32 ? L1.w32.dinv : nullptr, rd64, f32 ? nullptr : L1.w64.dinv,
                                              H->flags, H->flags + 1);
    if (f32 && multilevel) {
        // FP32 V-cycle: z stays FP32, in the first half of the z buffer of its parity
        float* z32 = reinterpret_cast<float*>(znew);
        vcycle_level<float>(H, 0, r32, rd32, z32, s, done);
        dev::k_pcg_dots<float><<<dev::NRED, BLOCK, 0, s>>>(n, z32, reinterpret_cast<const float*>(zold), H->r, dnew,
                                                           H->flags);
        dev::k_pcg_p<float><<<dev::NRED, BLOCK, 0, s>>>(n, dnew, dold, z32, H->p, H->st, H->flags, H->flags + 1,
                                                        H->flags + 2 + par, H->flags + 2 + (par ^ 1), H->ring_dev);
    } else {
        if (!multilevel) coarse_solve<double>(H, H->r, znew, s, done);
        else vcycle_level<double>(H, 0, H->r, rd64, znew, s, done);
        dev::k_pcg_dots<double><<<dev::NRED, BLOCK, 0, s>>>(n, znew, zold, H->r, dnew, H->flags);
        dev::k_pcg_p<double><<<dev::NRED, BLOCK, 0, s>>>(n, dnew, dold, znew, H->p, H->st, H->flags, H->flags + 1,
                                                         H->flags + 2 + par, H->flags + 2 + (par ^ 1), H->ring_dev);
    }
}

// One iteration of each buffer parity captured once as a HIP graph on the hierarchy's
// stream.
void capture_pcg(amge_hierarchy* H) {
    for (int par = 0; par < 2; ++par) {
        if (H->pexec[par]) continue;
        hipGraph_t graph = nullptr;
        HIPCHECK(hipStreamBeginCapture(H->gstream, hipStreamCaptureModeThreadLocal));
        pcg_iteration(H, par, H->gstream);
        hipError_t e = hipStreamEndCapture(H->gstream, &graph);
        if (e != hipSuccess || !graph) fail(AMGE_ERR_HIP, "graph capture of the PCG iteration failed");
        e = hipGraphInstantiate(&H->pexec[par], graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            H->pexec[par] = nullptr;
            fail(AMGE_ERR_HIP, "graph instantiation failed");
        }
    }
}

// Iterations the host may queue beyond the last one it has seen.  Iterations run after
// convergence do nothing but still cost their launches (~0.2 ms for a five-level
// hierarchy), and an empty queue costs a host round trip (~40 us), so the queue is kept
// at most as long as the iterations still needed, predicted from the mean contraction
// of the stopping quantity over the last (up to) four iterations.  rel[k] is that
// quantity after iteration k (rel[0] = 1).
int pcg_lookahead(const std::vector<double>& rel, double rtol) {
    constexpr int MAXQ = 4;
    if (rtol <= 0) return MAXQ;   // a fixed number of iterations
    const int k = (int)rel.size() - 1;
    if (k == 0) return 2;
    const int m = std::min(k, 4);
    const double cur = rel[k], prev = rel[k - m];
    if (!(cur > 0) || !(prev > cur) || !std::isfinite(prev)) return 2;   // no contraction seen
    const double need = std::log(rtol / cur) / (std::log(cur / prev) / m);
    if (!(need >= 1)) return 1;
    return (int)std::min<double>(MAXQ, std::floor(need));
}

amge_status pcg(amge_hierarchy* H, const double* b, double* x, double rtol, int maxit, int stop_l2,
                int* iters, double* relres, hipStream_t s) {
    const int n = H->lv[0].n;
    const bool f32 = H->opts.precond_bits == 32;
    const bool multilevel = H->lv.size() > 1;
    DLevel& L1 = H->lv[0];
    // the iteration kernels use the hierarchy's x buffer; the caller's x is written at the end
    const bool timed = L1.probe && L1.probe->on;   // probed launches are recorded eagerly
    hipStream_t gs = timed ? s : H->gstream;
    if (!timed) {
        capture_pcg(H);
        HIPCHECK(hipEventRecord(H->ev_in, s));
        HIPCHECK(hipStreamWaitEvent(gs, H->ev_in, 0));
    }
    copy_vec<double>(n, b, H->r, gs, H->zero_flag);
    fill_zero<double>(n, H->x, gs, H->zero_flag);
    fill_zero<int>(4, H->flags, gs, H->zero_flag);
    if (f32 && multilevel) {
        convert<double, float>(n, H->r, L1.w32.b, gs);
        scale<float>(n, L1.w32.dinv, L1.w32.b, L1.w32.bd, gs);
    }
    if (!f32 && multilevel) scale<double>(n, L1.w64.dinv, H->r, L1.w64.bd, gs);
    // z_0 = B r_0 into z[1] (the "old" z of the first iteration; FP32 in its first half
    // for an FP32 V-cycle), delta_0 = r_0 . z_0
    float* z32 = f32 && multilevel ? reinterpret_cast<float*>(H->z[1]) : nullptr;
    if (z32) {
        vcycle_level<float>(H, 0, L1.w32.b, L1.w32.bd, z32, gs, H->zero_flag);
        dev::k_pcg_dots<float><<<dev::NRED, BLOCK, 0, gs>>>(n, z32, nullptr, H->r, H->part_dots[1], H->zero_flag);
    } else {
        if (!multilevel) coarse_solve<double>(H, H->r, H->z[1], gs, H->zero_flag);
        else vcycle_level<double>(H, 0, H->r, L1.w64.bd, H->z[1], gs, H->zero_flag);
        dev::k_pcg_dots<double><<<dev::NRED, BLOCK, 0, gs>>>(n, H->z[1], nullptr, H->r, H->part_dots[1],
                                                             H->zero_flag);
    }
    const uint32_t epoch = ++H->epoch == 0 ? ++H->epoch : H->epoch;   // never 0 (the ring's initial tags)
    dev::k_pcg_init<<<1, BLOCK, 0, gs>>>(H->part_dots[1], H->st, rtol, maxit, stop_l2, epoch);
    dev::PcgStatus hs;
    HIPCHECK(hipMemcpyAsync(&hs, H->st, sizeof(hs), hipMemcpyDeviceToHost, gs));
    HIPCHECK(hipStreamSynchronize(gs));
    auto finish = [&]() {
        if (!timed) {
            HIPCHECK(hipEventRecord(H->ev_out, gs));
            HIPCHECK(hipStreamWaitEvent(s, H->ev_out, 0));
        }
    };
    if (!std::isfinite(hs.bnorm) || !std::isfinite(hs.delta0)) {
        finish();
        fail(AMGE_ERR_NONFINITE, "non-finite right-hand side");
    }
    if (hs.bnorm == 0) {
        copy_vec<double>(n, H->x, x, gs, H->zero_flag);
        finish();
        *iters = 0;
        *relres = 0;
        return AMGE_OK;
    }
    if (!(hs.delta0 > 0)) {
        finish();
        fail(AMGE_ERR_BREAKDOWN, "preconditioner not positive on the right-hand side");
    }
    if (z32) convert<float, double>(n, z32, H->p, gs);
    else copy_vec<double>(n, H->z[1], H->p, gs, H->zero_flag);
    // Iterations are queued ahead (graph replays, or direct launches when timing is on)
    // while the host follows the records they leave in the pinned ring: iteration k's
    // record is read once the event queued after it has completed.  Iterations queued
    // past convergence do nothing; the queue length comes from pcg_lookahead.
    std::vector<double> rel(1, 1.0);
    int launched = 0, seen = 0;
    while (!hs.done) {
        // timed runs launch the iterations directly, two at a time, and wait for each pair
        int upto = launched;
        if (!timed) upto = std::min(maxit, seen + pcg_lookahead(rel, rtol));
        else if (launched == seen) upto = std::min(maxit, seen + 2);
        for (; launched < upto; ++launched) {
            if (timed) pcg_iteration(H, launched & 1, gs);
            else HIPCHECK(hipGraphLaunch(H->pexec[launched & 1], gs));
            HIPCHECK(hipEventRecord(H->pev[launched % amge_hierarchy::NPEV], gs));
        }
        if (launched == seen) {
            finish();
            fail(AMGE_ERR_HIP, "PCG did not terminate");
        }
        HIPCHECK(hipEventSynchronize(H->pev[seen % amge_hierarchy::NPEV]));
        ++seen;
        const volatile dev::PcgRecord* rec = H->ring + seen % dev::PCG_RING;
        if (rec->tag != (((uint64_t)epoch << 32) | (uint32_t)seen)) {
            finish();
            fail(AMGE_ERR_HIP, "PCG iteration record missing");
        }
        std::atomic_thread_fence(std::memory_order_acquire);
        memcpy(&hs, (const void*)&rec->st, sizeof(hs));
        rel.push_back(hs.relres);
    }
    if (verbose()) fprintf(stderr, "[amge pcg] %d iterations, %d queued\n", hs.iters, launched);
    copy_vec<double>(n, H->x, x, gs, H->zero_flag);
    HIPCHECK(hipGetLastError());
    finish();
    *iters = hs.iters;
    *relres = hs.relres;
    if (hs.breakdown) fail(AMGE_ERR_BREAKDOWN, "PCG breakdown (p.q <= 0)");
    if (!std::isfinite(hs.delta)) fail(AMGE_ERR_NONFINITE, "non-finite PCG iterate");
    if (rtol > 0 && !(hs.relres <= rtol)) return AMGE_NOT_CONVERGED;
    return AMGE_OK;
}

// ---- batched inexact PCG: the single-column recurrences per column, with the
// stopping test per column on the device (a finished column takes alpha = 0 and keeps
// its iterate).  Columns are loaded as "fresh": their first pass through an iteration
// computes z0 = B b and the initial quantities instead of a step, so columns loaded at
// different times share every launch (the serving engine inserts requests into free
// columns between chunks).  One iteration per active width W (the first W of the NC
// columns) is captured as a HIP graph on the hierarchy's own stream and replayed in
// chunks; the host polls the batch status between chunks.  Sums over rows run in the
// same order whatever W is, so a column's result does not depend on the width.

template <int V, bool C16>
void bpcg_ap_v(amge_hierarchy* H, int W, hipStream_t s) {
    const DSellB& A = H->lv[0].bA;
    launch<dev::BpcgAp<V, C16>>(BPCG_BLOCKS, s, A.nslices, W, H->NC, A.sptr, A.srow, A.ci, A.c16, A.cbase, A.v64,
                                H->bP, H->bQ, H->bpart, H->bs);
}

void bpcg_ap(amge_hierarchy* H, int W, hipStream_t s) {
    const bool c16 = H->lv[0].bA.c16 != nullptr;
    if (H->NC >= 2) {   // 16-byte lane loads
        if (c16) bpcg_ap_v<2, true>(H, W, s);
        else bpcg_ap_v<2, false>(H, W, s);
    } else {
        if (c16) bpcg_ap_v<1, true>(H, W, s);
        else bpcg_ap_v<1, false>(H, W, s);
    }
}

// The FP32 V-cycle reads its input from the level-1 FP32 block; a one-level hierarchy
// (coarse solve only) always works in FP64, like the single-column path.
bool bz32(const amge_hierarchy* H) { return H->opts.precond_bits == 32 && H->lv.size() > 1; }

// z = B r on the residual block in the preconditioner precision; writes zv.
// With two or more primary sweeps the fine level's first launched sweep forms dinv r
// itself (JAC0), so the PCG update does not store it.
bool bpcg_fused_bd(const amge_hierarchy* H) { return H->lv.size() > 1 && H->opts.nu_primary >= 2; }

// z block of parity par in the preconditioner precision.
float* bz_f32(const amge_hierarchy* H, int par) {
    return reinterpret_cast<float*>(H->bZ) + (par ? (int64_t)H->lv[0].n * H->NC : 0);
}
double* bz_f64(const amge_hierarchy* H, int par) { return par ? H->bZv : H->bZ; }

void bpcg_precond(amge_hierarchy* H, int W, int par, const int* stop, hipStream_t s) {
    DLevel& L = H->lv[0];
    const bool fused = bpcg_fused_bd(H);
    if (bz32(H)) bvcycle_level<float>(H, 0, L.bw32.b, fused ? nullptr : L.bw32.bd, bz_f32(H, par), W, stop, s);
    else bvcycle_level<double>(H, 0, H->bR, fused ? nullptr : L.bw64.bd, bz_f64(H, par), W, stop, s);
}

void bpcg_dots(amge_hierarchy* H, int W, int par, hipStream_t s) {
    const int n = H->lv[0].n;
    if (bz32(H))
        launch<dev::BpcgDots<float>>(BPCG_BLOCKS, s, n, W, H->NC, bz_f32(H, par), bz_f32(H, par ^ 1), H->bR,
                                     H->bpart, H->bs);
    else
        launch<dev::BpcgDots<double>>(BPCG_BLOCKS, s, n, W, H->NC, bz_f64(H, par), bz_f64(H, par ^ 1), H->bR,
                                      H->bpart, H->bs);
}

// One PCG iteration on the first W columns (the captured body): q = A p, alpha, x/r
// update with the next preconditioner input, z = B r, dots, stopping test and beta,
// p update.
void bpcg_iteration(amge_hierarchy* H, int W, int par, hipStream_t s) {
    DLevel& L = H->lv[0];
    const int lgW = log2i(W);
    const int64_t nn = (int64_t)L.n * W;
    const bool f32 = bz32(H);
    const bool ml = H->lv.size() > 1;
    const unsigned g = grid_stride(nn);
    bpcg_ap(H, W, s);
    launch<dev::BpcgAlpha>(1, s, W, H->NC, H->bpart, BPCG_BLOCKS, H->cs, H->bs);
    const bool fused = bpcg_fused_bd(H);
    launch<dev::BpcgXr>(g, s, nn, lgW, H->lgNC, H->cs, H->bQ, H->bR, f32 ? L.bw32.b : nullptr,
                        f32 && !fused ? L.bw32.bd : nullptr, f32 ? L.bw32.dinv : nullptr,
                        !f32 && ml && !fused ? L.bw64.bd : nullptr, !f32 && ml ? L.bw64.dinv : nullptr, H->bs);
    bpcg_precond(H, W, par, &H->bs->all_done, s);
    bpcg_dots(H, W, par, s);
    launch<dev::BpcgUpdate>(1, s, W, H->NC, H->bpart, BPCG_BLOCKS, H->cs, H->bs);
    if (f32) launch<dev::BpcgP<float>>(g, s, nn, lgW, H->lgNC, H->cs, bz_f32(H, par), H->bP, H->bX, H->bs);
    else launch<dev::BpcgP<double>>(g, s, nn, lgW, H->lgNC, H->cs, bz_f64(H, par), H->bP, H->bX, H->bs);
    launch<dev::BpcgFinish>(1, s, H->bs);
}

hipGraphExec_t capture_iteration(amge_hierarchy* H, int W, int par) {
    if (H->NC < 2 || !H->gstream) fail(AMGE_ERR_ARG, "hierarchy has no batched path (max_rhs = 1)");
    if (W < 1 || W > H->NC || (W & (W - 1))) fail(AMGE_ERR_ARG, "active width must be a power of two <= NC");
    hipGraphExec_t& ex = H->gexec[log2i(W)][par & 1];
    if (ex) return ex;
    hipGraph_t graph = nullptr;
    HIPCHECK(hipStreamBeginCapture(H->gstream, hipStreamCaptureModeThreadLocal));
    bpcg_iteration(H, W, par & 1, H->gstream);
    hipError_t e = hipStreamEndCapture(H->gstream, &graph);
    if (e != hipSuccess || !graph) fail(AMGE_ERR_HIP, "graph capture of the batched PCG iteration failed");
    e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        ex = nullptr;
        fail(AMGE_ERR_HIP, "graph instantiation failed");
    }
    return ex;
}

LaunchRecorder*& launch_recorder() {
    static thread_local LaunchRecorder* r = nullptr;
    return r;
}

int group_launches(const std::vector<LaunchRecorder>& mem, hipStream_t s) {
    const int M = (int)mem.size();
    std::vector<size_t> next(M, 0);
    std::vector<const LaunchRec*> ops;
    int launches = 0;
    for (;;) {
        const void* best = nullptr;
        int best_count = 0;
        size_t best_left = 0;
        for (int m = 0; m < M; ++m) {
            if (next[m] >= mem[m].ops.size()) continue;
            const void* k = mem[m].ops[next[m]].key;
            int count = 0;
            size_t left = 0;
            for (int q = 0; q < M; ++q)
                if (next[q] < mem[q].ops.size() && mem[q].ops[next[q]].key == k) {
                    ++count;
                    left = std::max(left, mem[q].ops.size() - next[q]);
                }
            if (count > best_count || (count == best_count && left > best_left)) {
                best = k;
                best_count = count;
                best_left = left;
            }
        }
        if (!best) break;
        ops.clear();
        for (int m = 0; m < M; ++m)
            if (next[m] < mem[m].ops.size() && mem[m].ops[next[m]].key == best) ops.push_back(&mem[m].ops[next[m]++]);
        launches += ops[0]->emit(ops.data(), (int)ops.size(), s);
    }
    return launches;
}

hipGraphExec_t capture_grouped_iteration(const std::vector<amge_hierarchy*>& hs, int par, hipStream_t s,
                                         int* launches, int* solo_launches) {
    std::vector<LaunchRecorder> rec(hs.size());
    int solo = 0;
    for (size_t i = 0; i < hs.size(); ++i) {
        amge_hierarchy* H = hs[i];
        if (H->NC < 2 || !H->gstream) fail(AMGE_ERR_ARG, "hierarchy has no batched path (max_rhs = 1)");
        RecordLaunches scope(&rec[i]);
        bpcg_iteration(H, H->NC, par & 1, s);
        solo += (int)rec[i].ops.size();
    }
    hipGraph_t graph = nullptr;
    HIPCHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    const int n = group_launches(rec, s);
    hipError_t e = hipStreamEndCapture(s, &graph);
    if (e != hipSuccess || !graph) fail(AMGE_ERR_HIP, "graph capture of the grouped PCG iteration failed");
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) fail(AMGE_ERR_HIP, "graph instantiation failed");
    if (launches) *launches = n;
    if (solo_launches) *solo_launches = solo;
    return ex;
}

amge_status bpcg(amge_hierarchy* H, const double* b, double* x, int nrhs, double rtol, int maxit, int stop_l2,
                 int* iters, double* relres, hipStream_t s) {
    DLevel& L = H->lv[0];
    const int64_t n = L.n;
    const int NC = H->NC;
    hipStream_t gs = H->gstream;
    const int W = active_width(H, nrhs);
    hipGraphExec_t ex[2] = {capture_iteration(H, W, 0), capture_iteration(H, W, 1)};
    // order the internal stream after the caller's work
    HIPCHECK(hipEventRecord(H->ev_in, s));
    HIPCHECK(hipStreamWaitEvent(gs, H->ev_in, 0));
    dev::k_bpcg_load<<<grid_stride(n * NC), BLOCK, 0, gs>>>(n, nrhs, H->lgNC, b, H->bR, H->bX, H->bP, H->cs, H->bs,
                                                            rtol, maxit, stop_l2);
    HIPCHECK(hipGetLastError());
    dev::BatchStatus st{};
    // every column finishes within maxit steps after its initial pass
    for (int launched = 0;;) {
        if (launched > maxit + 1) fail(AMGE_ERR_HIP, "batched PCG did not terminate");
        for (int i = 0; i < BPCG_CHUNK; ++i) {
            HIPCHECK(hipGraphLaunch(ex[H->bpar], gs));
            H->bpar ^= 1;
        }
        launched += BPCG_CHUNK;
        HIPCHECK(hipMemcpyAsync(&st, H->bs, sizeof(st), hipMemcpyDeviceToHost, gs));
        HIPCHECK(hipStreamSynchronize(gs));
        if (st.all_done) break;
    }
    std::vector<dev::ColState> cs(NC);
    HIPCHECK(hipMemcpyAsync(cs.data(), H->cs, sizeof(dev::ColState) * NC, hipMemcpyDeviceToHost, gs));
    dev::k_unpack<double><<<grid_stride(n * nrhs), BLOCK, 0, gs>>>(n, nrhs, H->lgNC, H->bX, x);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(gs));
    HIPCHECK(hipEventRecord(H->ev_out, gs));
    HIPCHECK(hipStreamWaitEvent(s, H->ev_out, 0));
    bool brk = false, nonfin = false, unconv = false;
    for (int c = 0; c < nrhs; ++c) {
        iters[c] = cs[c].iters;
        relres[c] = cs[c].relres;
        brk |= cs[c].breakdown != 0;
        nonfin |= cs[c].nonfinite != 0;
        unconv |= rtol > 0 && !(cs[c].relres <= rtol);
    }
    if (nonfin) fail(AMGE_ERR_NONFINITE, "non-finite right-hand side or PCG iterate in a column");
    if (brk) fail(AMGE_ERR_BREAKDOWN, "PCG breakdown (p.q <= 0 or preconditioner not positive) in a column");
    if (unconv) return AMGE_NOT_CONVERGED;
    return AMGE_OK;
}

template <class F>
amge_status guard(F&& f) {
    try {
        return f();
    } catch (const Error& e) {
        set_last_error(e.what());
        return e.code;
    } catch (const std::bad_alloc&) {
        set_last_error("host allocation failed");
        return AMGE_ERR_OOM;
    } catch (const std::exception& e) {
        set_last_error(e.what());
        return AMGE_ERR_ARG;
    }
}

}  // namespace amge

using namespace amge;

extern "C" void amge_default_opts(amge_opts* o) {
    if (!o) return;
    o->nu_primary = 2;
    o->nu_aux = 2;
    o->precond_bits = 32;
    o->max_rhs = 1;
    o->tail_rows = 2048;
    o->smoother = AMGE_SMOOTHER_L1_JACOBI;
    o->resid_bits = 0;
    o->alloc = nullptr;
    o->dealloc = nullptr;
    o->alloc_user = nullptr;
}

extern "C" amge_status amge_setup_hierarchy(const amge_level* levels, int32_t nlevels, const amge_opts* opts,
                                            void* stream, amge_hierarchy** out) {
    return guard([&]() -> amge_status {
        if (!out) fail(AMGE_ERR_ARG, "null output pointer");
        *out = nullptr;
        auto H = std::make_unique<amge_hierarchy>();
        if (opts) H->opts = *opts;
        else amge_default_opts(&H->opts);
        if (H->opts.nu_primary < 0 || H->opts.nu_aux < 0 || H->opts.max_rhs < 1 || H->opts.max_rhs > 64 ||
            H->opts.tail_rows < 0 || H->opts.tail_rows > 8192 ||
            (H->opts.precond_bits != 0 && H->opts.precond_bits != 32 && H->opts.precond_bits != 64) ||
            (H->opts.resid_bits != 0 && H->opts.resid_bits != 32 && H->opts.resid_bits != 64))
            fail(AMGE_ERR_ARG, "invalid options");
        if ((H->opts.alloc == nullptr) != (H->opts.dealloc == nullptr))
            fail(AMGE_ERR_ARG, "give both alloc and dealloc, or neither");
        if (H->opts.smoother != AMGE_SMOOTHER_L1_JACOBI && H->opts.smoother != AMGE_SMOOTHER_SYM_GS &&
            H->opts.smoother != AMGE_SMOOTHER_BLOCK_GS)
            fail(AMGE_ERR_ARG, "unknown smoother");
        if (H->opts.smoother == AMGE_SMOOTHER_SYM_GS && H->opts.max_rhs > 1)
            fail(AMGE_ERR_ARG, "the colour-order Gauss-Seidel smoother runs single-column contexts only (max_rhs = 1)");
        setup(H.get(), levels, nlevels, (hipStream_t)stream);
        *out = H.release();
        return AMGE_OK;
    });
}

extern "C" void amge_destroy(amge_hierarchy* h) { delete h; }

extern "C" amge_status amge_ctx_create(const amge_hierarchy* h, int32_t nrhs, amge_ctx** out) {
    return guard([&]() -> amge_status {
        if (!h || !out) fail(AMGE_ERR_ARG, "null argument");
        *out = nullptr;
        *out = make_ctx(h, nrhs).release();
        return AMGE_OK;
    });
}

extern "C" void amge_ctx_destroy(amge_ctx* c) { delete c; }

extern "C" amge_status amge_footprint(const amge_hierarchy* h, int32_t nrhs, size_t* hier_bytes,
                                      size_t* ctx_bytes) {
    return guard([&]() -> amge_status {
        if (!h || h->parent) fail(AMGE_ERR_ARG, "not a hierarchy");
        if (hier_bytes) *hier_bytes = h->bytes;
        if (ctx_bytes) *ctx_bytes = make_ctx(h, nrhs, true)->st.bytes;
        return AMGE_OK;
    });
}

extern "C" amge_status amge_precision_info(const amge_hierarchy* h, double* kappa, int32_t* precond_bits,
                                           int32_t* resid_bits) {
    if (!h) {
        set_last_error("null argument");
        return AMGE_ERR_ARG;
    }
    if (kappa) *kappa = h->kappa;
    if (precond_bits) *precond_bits = h->opts.precond_bits;
    if (resid_bits) *resid_bits = (h->opts.precond_bits == 32 && !h->lv.empty() && !h->lv[0].resid64) ? 32 : 64;
    return AMGE_OK;
}

extern "C" amge_status amge_hierarchy_info(const amge_hierarchy* h, int32_t* nlevels, int32_t* rows) {
    if (!h || !nlevels) {
        set_last_error("null argument");
        return AMGE_ERR_ARG;
    }
    *nlevels = (int32_t)h->lv.size();
    if (rows)
        for (size_t k = 0; k < h->lv.size(); ++k) rows[k] = h->lv[k].n;
    return AMGE_OK;
}

extern "C" amge_status amge_vcycle(amge_ctx* c, const double* r, double* z, int32_t nrhs, void* stream) {
    return guard([&]() -> amge_status {
        if (!c || !r || !z) fail(AMGE_ERR_ARG, "null argument");
        amge_hierarchy* h = &c->st;
        if (nrhs < 1 || nrhs > h->nrhs_cap) fail(AMGE_ERR_ARG, "amge_vcycle: need 1 <= nrhs <= the context's nrhs");
        hipStream_t s = (hipStream_t)stream;
        if (nrhs > 1) {
            if (h->opts.precond_bits == 32 && h->lv.size() > 1) bprecondition<float>(h, r, z, nrhs, s);
            else bprecondition<double>(h, r, z, nrhs, s);
        } else if (h->lv.size() == 1) {
            coarse_solve<double>(h, r, z, s, h->zero_flag);
        } else {
            precondition(h, r, z, s);
        }
        HIPCHECK(hipGetLastError());
        return AMGE_OK;
    });
}

// ------------------------------------------------------------------ no-allocation V-cycle
// amge_vcycle_static: the single-column V-cycle with its level work vectors carved out
// of `scratch`, a file-scope device array (one per GPU, held until the process ends),
// instead of a context's buffers.  Host code never passes `scratch` itself to a kernel
// (in host code the name is a stand-in, not a device address): its device address is
// looked up once per device with hipGetSymbolAddress and only that address is used.
constexpr size_t STATIC_SCRATCH_BYTES = AMGE_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[STATIC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
std::map<int, char*> g_scratch_ptr;   // device -> address of its scratch

// Address of the current device's scratch, looked up on the first call on that device.
char* scratch_address() {
    int d = 0;
    HIPCHECK(hipGetDevice(&d));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(d);
    if (it != g_scratch_ptr.end()) return it->second;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        fail(AMGE_ERR_HIP, std::string("hipGetSymbolAddress of the static scratch failed: ") + hipGetErrorString(e));
    g_scratch_ptr[d] = (char*)ptr;
    return (char*)ptr;
}
}  // namespace

extern "C" amge_status amge_vcycle_static(const amge_hierarchy* h, const double* r, double* z, void* stream) {
    return guard([&]() -> amge_status {
        if (!h || !r || !z) fail(AMGE_ERR_ARG, "null argument");
        if (h->parent) fail(AMGE_ERR_ARG, "not a hierarchy");
        amge_hierarchy S;   // execution state whose work vectors live in the scratch
        S.arena = scratch_address();
        S.arena_size = STATIC_SCRATCH_BYTES;
        init_state(&S, h, 1);   // fails before any launch if the work does not fit
        hipStream_t s = (hipStream_t)stream;
        if (S.lv.size() == 1) coarse_solve<double>(&S, r, z, s, S.zero_flag);
        else precondition(&S, r, z, s);
        HIPCHECK(hipGetLastError());
        return AMGE_OK;
    });
}

extern "C" amge_status amge_pcg_solve(amge_ctx* c, const double* b, double* x, int32_t nrhs, double rtol,
                                      int32_t maxit, int32_t stop_norm, int32_t* iters, double* relres,
                                      void* stream) {
    return guard([&]() -> amge_status {
        if (!c || !b || !x || !iters || !relres) fail(AMGE_ERR_ARG, "null argument");
        amge_hierarchy* h = &c->st;
        if (nrhs < 1 || nrhs > h->nrhs_cap)
            fail(AMGE_ERR_ARG, "amge_pcg_solve: need 1 <= nrhs <= the context's nrhs");
        if (maxit < 1) fail(AMGE_ERR_ARG, "maxit must be >= 1");
        if (nrhs > 1) return bpcg(h, b, x, nrhs, rtol, maxit, stop_norm, iters, relres, (hipStream_t)stream);
        int it = 0;
        double rr = 0;
        amge_status st = pcg(h, b, x, rtol, maxit, stop_norm, &it, &rr, (hipStream_t)stream);
        iters[0] = it;
        relres[0] = rr;
        return st;
    });
}

extern "C" amge_status amge_level_apply(amge_ctx* c, int32_t level, int32_t op, int32_t precision,
                                        const double* in, const double* in2, double* out, void* stream) {
    return guard([&]() -> amge_status {
        if (!c || !in || !out) fail(AMGE_ERR_ARG, "null argument");
        amge_hierarchy* h = &c->st;
        const int nl = (int)h->lv.size();
        if (level < 0 || level >= nl) fail(AMGE_ERR_ARG, "level out of range");
        if (precision != 32 && precision != 64) fail(AMGE_ERR_ARG, "precision must be 32 or 64");
        hipStream_t s = (hipStream_t)stream;
        DLevel& L = h->lv[level];
        const bool last = level == nl - 1;
        if (op == AMGE_OP_COARSE) {
            if (!last) fail(AMGE_ERR_ARG, "coarse solve only on the coarsest level");
            coarse_solve<double>(h, in, out, s, h->zero_flag);
            HIPCHECK(hipGetLastError());
            return AMGE_OK;
        }
        if (last) fail(AMGE_ERR_ARG, "operator not stored on the coarsest level");
        if ((op == AMGE_OP_SMOOTH || op == AMGE_OP_SMOOTHT || op == AMGE_OP_SWEEP || op == AMGE_OP_RESID) && !in2)
            fail(AMGE_ERR_ARG, "this operation needs x (in2)");
        // in / out lengths
        int nin = L.n, nout = L.n;
        switch (op) {
            case AMGE_OP_A: break;
            case AMGE_OP_AHAT: nin = nout = L.m; break;
            case AMGE_OP_D: nin = L.m; break;
            case AMGE_OP_DT: nout = L.m; break;
            case AMGE_OP_P: nin = h->lv[level + 1].n; break;
            case AMGE_OP_PT: nout = h->lv[level + 1].n; break;
            case AMGE_OP_SMOOTH: case AMGE_OP_SMOOTHT: case AMGE_OP_SWEEP: case AMGE_OP_RESID: break;
            default: fail(AMGE_ERR_ARG, "unknown op");
        }
        const int* z0 = h->zero_flag;
        auto run = [&](auto tag, const auto* vin, const auto* vin2, auto* vout) {
            using T = decltype(tag);
            // the level work of this precision, if the context does not hold it yet
            if (!L.w<T>().x) alloc_work<T>(h, L, L.w<T>());
            switch (op) {
                case AMGE_OP_A: sell<T>(L.A, dev::SPMV, vin, nullptr, nullptr, vout, s, z0); break;
                case AMGE_OP_AHAT: sell<T>(L.Ah, dev::SPMV, vin, nullptr, nullptr, vout, s, z0); break;
                case AMGE_OP_D: sell_inc<T>(L.D, 0, vin, vout, s, z0); break;
                case AMGE_OP_DT: sell_inc<T>(L.Dt, 0, vin, vout, s, z0); break;
                case AMGE_OP_P: sell<T>(L.P, dev::SPMV, vin, nullptr, nullptr, vout, s, z0); break;
                case AMGE_OP_PT: sell<T>(L.Pt, dev::SPMV, vin, nullptr, nullptr, vout, s, z0); break;
                // the V-cycle's own A_k launches (timed by amge_timing_* on the fine level)
                case AMGE_OP_SWEEP:
                    if (L.bgA.on()) bgs<T>(L, L.bgA, false, vin2, vin, vout, s, z0);
                    else asell<T>(L, dev::JAC, vin2, vin, L.w<T>().dinv, vout, s, z0);
                    break;
                case AMGE_OP_RESID: aresid<T>(L, vin2, vin, vout, s, z0); break;
                default: {
                    Work<T>& w = L.w<T>();
                    // x lives in w.x (copied in), result copied out
                    HIPCHECK(hipMemcpyAsync(w.x, vin2, sizeof(T) * L.n, hipMemcpyDeviceToDevice, s));
                    T* x = w.x;
                    T* xt = w.xt;
                    if (op == AMGE_OP_SMOOTH) {
                        primary<T>(L, vin, nullptr, x, xt, false, h->opts.nu_primary, s, z0);
                        auxiliary<T>(L, vin, x, h->opts.nu_aux, s, z0);
                    } else {
                        auxiliary<T>(L, vin, x, h->opts.nu_aux, s, z0);
                        primary<T>(L, vin, nullptr, x, xt, false, h->opts.nu_primary, s, z0);
                    }
                    HIPCHECK(hipMemcpyAsync(vout, x, sizeof(T) * L.n, hipMemcpyDeviceToDevice, s));
                }
            }
        };
        if (precision == 64) {
            run(double{}, in, in2, out);
        } else {
            // FP32 kernels on rounded copies held in temporary buffers
            size_t nmax = (size_t)std::max(std::max(nin, nout), L.n);
            amge_hierarchy tmp;   // owns the temporaries (the context's allocator)
            tmp.opts = h->opts;
            float* fin = tmp.alloc<float>(nmax);
            float* fin2 = tmp.alloc<float>(nmax);
            float* fout = tmp.alloc<float>(nmax);
            convert<double, float>(nin, in, fin, s);
            if (in2) convert<double, float>(L.n, in2, fin2, s);
            run(float{}, (const float*)fin, (const float*)fin2, fout);
            convert<float, double>(nout, fout, out, s);
            HIPCHECK(hipStreamSynchronize(s));
        }
        HIPCHECK(hipGetLastError());
        return AMGE_OK;
    });
}

extern "C" amge_status amge_timing_enable(amge_ctx* c, int32_t enable) {
    return guard([&]() -> amge_status {
        if (!c) fail(AMGE_ERR_ARG, "null argument");
        amge_hierarchy* h = &c->st;
        h->probe.on = enable != 0;
        h->probe.used = 0;
        h->probe.bytes = 0;
        h->lv[0].probe = h->lv.size() > 1 ? &h->probe : nullptr;
        return AMGE_OK;
    });
}

extern "C" amge_status amge_timing_read(amge_ctx* c, double* ms, int64_t* launches, double* bytes) {
    return guard([&]() -> amge_status {
        if (!c || !ms || !launches || !bytes) fail(AMGE_ERR_ARG, "null argument");
        amge_hierarchy* h = &c->st;
        double tot = 0;
        for (size_t i = 0; i < h->probe.used; ++i) {
            HIPCHECK(hipEventSynchronize(h->probe.ev[2 * i + 1]));
            float t = 0;
            HIPCHECK(hipEventElapsedTime(&t, h->probe.ev[2 * i], h->probe.ev[2 * i + 1]));
            tot += t;
        }
        *ms = tot;
        *launches = (int64_t)h->probe.used;
        *bytes = h->probe.bytes;
        h->probe.used = 0;
        h->probe.bytes = 0;
        return AMGE_OK;
    });
}

extern "C" amge_status amge_vcycle_bytes(const amge_hierarchy* h, int32_t precision, int32_t nrhs, double* bytes) {
    return guard([&]() -> amge_status {
        if (!h || !bytes) fail(AMGE_ERR_ARG, "null argument");
        if (precision != 32 && precision != 64) fail(AMGE_ERR_ARG, "precision must be 32 or 64");
        if (nrhs < 1 || nrhs > h->opts.max_rhs) fail(AMGE_ERR_ARG, "need 1 <= nrhs <= max_rhs");
        if (h->parent) fail(AMGE_ERR_ARG, "not a hierarchy");
        const bool batched = nrhs > 1;
        const double sv = precision == 32 ? 4.0 : 8.0;   // value size
        const double sx = sv * nrhs;                       // one row of a vector block
        const int nup = h->opts.nu_primary, nua = h->opts.nu_aux;
        double tot = 0;
        // levels run by their kernels: those above the dense tail (the coarsest inverse or
        // the folded coarse tail)
        const size_t last = (size_t)h->tail;
        for (size_t k = 0; k < last; ++k) {
            const DLevel& L = h->lv[k];
            const double n = L.n, m = L.m, nc = h->lv[k + 1].n;
            // matrix streams: values + column indices + one row pointer (sliced ELL: one
            // row index) per row; incidences are index-only
            auto mat = [&](const DSell& M, const DSellB& B) {
                return batched ? (double)B.nnz * (sv + (B.c16 ? 2.0 : 4.0)) + 4.0 * B.nrows
                               : (double)M.nnz * (sv + (M.c16 ? 2.0 : 4.0)) + 4.0 * M.nrows;
            };
            auto incb = [&](const DSell& M, const DSellB& B) {
                return batched ? (double)B.nnz * 4.0 + 4.0 * B.nrows
                               : (double)M.nnz * 4.0 + (M.fixedw ? 0.0 : 4.0 * M.nrows);
            };
            // Gauss-Seidel colour launches: the colour's rows (values, indices, row index,
            // b, 1/a_ii, x read and written) and the gathered x once
            auto gsb = [&](const GsColors& g, double ncols, int nu) {
                const int C = (int)g.col.size();
                if (nu <= 0 || C == 0) return 0.0;
                auto one = [&](int c) {
                    const DSell& M = g.col[c];
                    return (double)M.nnz * (sv + (M.c16 ? 2.0 : 4.0)) + 4.0 * M.nrows + 4 * sv * M.nrows + sv * ncols;
                };
                double t = one(0);
                for (int k = 0; k < nu; ++k) {
                    for (int c = 1; c < C; ++c) t += one(c);
                    for (int c = C - 2; c >= 0; --c) t += one(c);
                }
                return t;
            };
            const bool gs = !L.gsA.col.empty();
            const bool bg = L.bgA.on();
            // block Gauss-Seidel: nu sweeps, the first of a smoothing from zero a pre-smoothing
            auto bgb = [&](const DBgs& g, int nu, bool zero) {
                if (nu <= 0) return zero ? sx * g.n : 0.0;
                return bgs_bytes(g, zero, (int)sv, nrhs) + (nu - 1) * bgs_bytes(g, false, (int)sv, nrhs);
            };
            if (bg) {
                tot += bgb(L.bgA, nup, true) + bgb(L.bgA, nup, false);
            } else if (gs) {
                // pre-smoother from zero (x filled with zeros), post-smoother from x
                tot += sx * n + 2 * gsb(L.gsA, n, nup);
            } else {
                // primary sweeps: the first one from zero is the producer's bd = dinv b (two
                // extra streams there), every launched sweep reads x, b and writes y (+ dinv)
                const int launched = std::max(0, nup - 1) + nup;
                tot += launched * (mat(L.A, L.bA) + 3 * sx * n + sv * n) + 2 * sx * n;
            }
            // auxiliary step, pre and post: residual [D^T | -D^T A][b; x] (+ gd), sweeps, D add
            if (nua > 0 && bg) {
                // [D^T | -D^T A] (g only), block sweeps on D^T A D from zero, D add
                double aux = mat(L.Aux, L.bAux) + 2.0 * m + sx * (2 * n + m);
                aux += bgb(L.bgAh, nua, true);
                aux += incb(L.D, L.bD) + sx * (m + 2 * n);
                tot += 2 * aux;
            } else if (nua > 0 && gs) {
                // [D^T | -D^T A] (g only), y filled with zeros, Gauss-Seidel on D^T A D, D add
                double aux = mat(L.Aux, L.bAux) + 2.0 * m + sx * (2 * n + m) + sx * m;
                aux += gsb(L.gsAh, m, nua);
                aux += incb(L.D, L.bD) + sx * (m + 2 * n);
                tot += 2 * aux;
            } else if (nua > 0) {
                // [D^T | -D^T A] with its split counts (2 bytes a row); b, x; g, gd; dhinv
                double aux = mat(L.Aux, L.bAux) + 2.0 * m + sx * (2 * n + m) + sx * m + sv * m;
                aux += (nua - 1) * (mat(L.Ah, L.bAh) + 3 * sx * m + sv * m);
                aux += incb(L.D, L.bD) + sx * (m + 2 * n);
                tot += 2 * aux;
            }
            // restriction: residual then P^T, or (single column below the fine level)
            // [P^T | -P^T A][b; x] with its split counts; then the P add
            if (!batched && L.PtA.nrows) {
                tot += mat(L.PtA, L.bPt) + 2.0 * nc + sx * (2 * n) + 2 * sx * nc;
            } else {
                // an FP32 cycle's fine-level residual with resid64 reads the FP64 values
                const double extra = (precision == 32 && L.resid64)
                                         ? (double)(batched ? L.bA.nnz : L.A.nnz) * (8.0 - sv) : 0.0;
                if (bg)
                    tot += bgs_resid_bytes(L.bgA, (precision == 32 && L.resid64) ? 8 : (int)sv, (int)sv, nrhs);
                else
                    tot += mat(L.A, L.bA) + extra + 3 * sx * n;
                tot += mat(L.Pt, L.bPt) + sx * (n + nc);
            }
            tot += mat(L.P, L.bP) + sx * (nc + 2 * n);
        }
        // the dense operator read once, the right-hand side and solution blocks
        const double nd = h->tail_n;
        tot += 8.0 * nd * nd + 2 * sx * nd;
        *bytes = tot;
        return AMGE_OK;
    });
}
