// l1-scaled symmetric block Gauss-Seidel sweep (the point smoother of section 4.1, last
// paragraph, with the two sweeps of section 5.1), one wave per block of 64 consecutive
// rows.
//
// The cited smoother relaxes the rows of each processor in turn (Gauss-Seidel) while
// couplings to other processors' rows read the values from the start of the sweep, and
// adds their absolute values to the diagonal.  Here a 64-row block plays the processor:
// one wave holds its rows, one row per lane, so the in-block order has to expose
// parallelism.  Rows are coloured over the couplings inside the block and relaxed colour
// by colour; rows of one colour are not coupled, so each colour's relaxation is exact
// Gauss-Seidel in (colour, row) order.  With r = b - A x0 at the start of the sweep, the
// forward pass solves (D_l1 + L) u = r and the backward pass (D_l1 + U) w = (D + 2 D_l1) u,
// x = x0 + w (D: a_ii, D_l1: the outside l1 sums, L / U: the inside couplings to earlier
// / later colours); this is the forward-then-backward row relaxation with the outside
// couplings frozen.
//
// Layout per block: an ELL of width w (entry t of lane q at base + t * 64 + q), each
// row's entries inside the block first (code: position in the block), then the others
// (code: column, or a 16-bit offset from the block's base column); padding: value 0 and
// code 0.  The first NIN entries of a row (NIN >= every block's inside width, so they hold
// the inside entries) are loaded together, then gathered together; the rest follow in
// uniform loops, and the colour passes read LDS without per-lane branches.  The inside
// couplings stay in registers, u and w in LDS; the passes synchronise the wave only.  A
// sweep from x0 = 0 reads the first wi entries of every row only (wi: the block's most
// inside entries of a row).
//
// Bytes: a full sweep reads every stored entry once (value + 2- or 4-byte code) plus b,
// x, the row data and writes y, like an l1-Jacobi sweep.
#pragma once

#include <type_traits>

#include "grouped.hpp"
#include "kernels_base.hpp"
#include "state.hpp"

namespace amge {
namespace dev {

// Orders the LDS accesses of one wave: every lane's earlier LDS writes are visible to
// the wave's later LDS reads.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Column of entry t of a row with nin inside entries.
template <bool C16>
__device__ __forceinline__ int bgs_col(int t, int nin, int code, int row0, int cb) {
    return t < nin ? row0 + code : (C16 ? cb + code : code);
}

template <bool C16>
__device__ __forceinline__ int bgs_code(const int* __restrict__ ci, const uint16_t* __restrict__ c16, int e) {
    return C16 ? (int)c16[e] : ci[e];
}

// y = x + w (ZERO: x = 0, y = w) for every block; NIN >= every block's inside width.
template <typename T, bool C16, bool ZERO, int NIN>
__global__ void __launch_bounds__(BLOCK)
k_bgs(int nblk, int n, const BgsBlock* __restrict__ blocks, const uint16_t* __restrict__ meta,
      const int* __restrict__ ci, const uint16_t* __restrict__ c16, const T* __restrict__ av,
      const T* __restrict__ dinv, const T* __restrict__ mid, const T* __restrict__ x,
      const T* __restrict__ b, T* __restrict__ y, const int* __restrict__ stop) {
    __shared__ T su[WAVES][64], sw[WAVES][64];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int blk = xcd_block(blockIdx.x, gridDim.x) * WAVES + wv;   // uniform: scalar block record
    const int bl = min(blk, nblk - 1);
    const int stopped = *stop;
    const BgsBlock B = blocks[bl];
    if (stopped | (blk >= nblk)) return;   // whole waves only
    const int row0 = bl * 64;
    const int i = row0 + lane;
    const bool live = i < n;
    const int ir = live ? i : row0;
    const int mt = meta[ir];
    const int nin = live ? (mt & 0xff) : 0;
    const int colour = live ? (mt >> 8) : -1;
    const T br = b[ir], di = dinv[ir], mi = mid[ir];
    const T xr = ZERO ? T(0) : x[ir];
    su[wv][lane] = T(0);
    sw[wv][lane] = T(0);
    const int ncol = B.info >> 8;
    const int e0 = B.base + lane;
    const int cb = B.cbase;
    // the first NIN entries of every row (they hold every inside entry): all loads first,
    // then all gathers, so a row's loads are in flight together; the arrays are padded
    // past their end, and entries at t >= width are masked
    const int W = B.width;
    T a[NIN];
    int id[NIN];
#pragma unroll
    for (int t = 0; t < NIN; ++t) {
        a[t] = T(0);
        id[t] = lane;
        // a sweep from zero needs the block's inside width only (a uniform bound: its
        // loads are still issued together, no gathers wait on them)
        if (!ZERO || t < (B.info & 0xff)) {
            a[t] = av[e0 + t * 64];
            id[t] = bgs_code<C16>(ci, c16, e0 + t * 64);
        }
    }
    T acc = 0;
    if (!ZERO) {
#pragma unroll
        for (int t = 0; t < NIN; ++t) {
            const int j = t < W ? bgs_col<C16>(t, nin, id[t], row0, cb) : row0;
            acc = fma(t < W ? a[t] : T(0), x[j], acc);
        }
    }
#pragma unroll
    for (int t = 0; t < NIN; ++t) {   // keep the inside couplings: value 0 / own position elsewhere
        const bool in = t < nin;
        a[t] = in ? a[t] : T(0);
        id[t] = in ? id[t] : lane;
    }
    if (!ZERO) {
#pragma unroll 8
        for (int t = NIN; t < W; ++t) {   // outside entries (or padding) in every row
            const int e = e0 + t * 64;
            const int code = bgs_code<C16>(ci, c16, e);
            acc = fma(av[e], x[C16 ? cb + code : code], acc);
        }
    }
    const T r0 = br - acc;
    wave_sync();
    // forward: (D_l1 + L) u = r0, colours in increasing order
    T uq = 0;
    for (int c = 0; c < ncol; ++c) {
        if (colour == c) {
            T s = 0;
#pragma unroll
            for (int t = 0; t < NIN; ++t) s = fma(a[t], su[wv][id[t]], s);
            uq = (r0 - s) * di;
            su[wv][lane] = uq;
        }
        wave_sync();
    }
    // backward: (D_l1 + U) w = (D + 2 D_l1) u, colours in decreasing order
    const T v = mi * uq;
    T wq = 0;
    for (int c = ncol - 1; c >= 0; --c) {
        if (colour == c) {
            T s = 0;
#pragma unroll
            for (int t = 0; t < NIN; ++t) s = fma(a[t], sw[wv][id[t]], s);
            wq = (v - s) * di;
            sw[wv][lane] = wq;
        }
        wave_sync();
    }
    if (live) y[i] = ZERO ? wq : xr + wq;
}

// y = b - A x on the same layout (the residual ahead of the restriction, so that the
// V-cycle reads one copy of A).  TV: value type; FP64 values with FP32 vectors sum in
// FP64 and round once.
template <typename T, bool C16, typename TV>
__global__ void __launch_bounds__(BLOCK)
k_bgs_resid(int nblk, int n, const BgsBlock* __restrict__ blocks, const uint16_t* __restrict__ meta,
            const int* __restrict__ ci, const uint16_t* __restrict__ c16, const TV* __restrict__ av,
            const T* __restrict__ x, const T* __restrict__ b, T* __restrict__ y, const int* __restrict__ stop) {
    using TA = typename std::conditional<(sizeof(TV) > sizeof(T)), TV, T>::type;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int blk = xcd_block(blockIdx.x, gridDim.x) * WAVES + wv;
    const int bl = min(blk, nblk - 1);
    const int stopped = *stop;
    const BgsBlock B = blocks[bl];
    if (stopped | (blk >= nblk)) return;
    const int row0 = bl * 64;
    const int i = row0 + lane;
    const bool live = i < n;
    const int ir = live ? i : row0;
    const int nin = live ? (meta[ir] & 0xff) : 0;
    const T br = b[ir];
    const int e0 = B.base + lane;
    const int cb = B.cbase;
    TA acc = 0;
#pragma unroll 8
    for (int t = 0; t < B.width; ++t) {
        const int e = e0 + t * 64;
        const int code = bgs_code<C16>(ci, c16, e);
        acc = fma((TA)av[e], (TA)x[bgs_col<C16>(t, nin, code, row0, cb)], acc);
    }
    if (live) y[i] = (T)((TA)br - acc);
}

// ---------------------------------------------------------------------------------
// Batched sweeps (n x NC row-major blocks): the block layout above, each wave a 64-row
// block and V consecutive columns of the first W (L = W / V waves per block, each
// reading the block's entries; the entries are L1/L2 hits after the first).  Every
// column goes through exactly the arithmetic of the single-column sweep, so a column's
// result depends neither on W, V nor the other columns.  Bodies of grid objects G
// (grouped.hpp), launched solo or grouped.
namespace bgsmm {

template <typename T, int V>
struct Row {
    T v[V];
};

template <typename T, int V>
__device__ __forceinline__ void load_row(Row<T, V>& r, const T* p) {
    if constexpr (V * sizeof(T) >= 16 && (V * sizeof(T)) % 16 == 0) {
        using VT = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
        constexpr int W = 16 / sizeof(T);
#pragma unroll
        for (int c = 0; c < V; c += W) {
            const VT w = *reinterpret_cast<const VT*>(p + c);
            const T* s = reinterpret_cast<const T*>(&w);
#pragma unroll
            for (int i = 0; i < W; ++i) r.v[c + i] = s[i];
        }
    } else {
#pragma unroll
        for (int i = 0; i < V; ++i) r.v[i] = p[i];
    }
}

template <typename T, int V>
__device__ __forceinline__ void store_row(const Row<T, V>& r, T* p) {
    if constexpr (V * sizeof(T) >= 16 && (V * sizeof(T)) % 16 == 0) {
        using VT = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
        constexpr int W = 16 / sizeof(T);
#pragma unroll
        for (int c = 0; c < V; c += W) {
            VT w;
            T* s = reinterpret_cast<T*>(&w);
#pragma unroll
            for (int i = 0; i < W; ++i) s[i] = r.v[c + i];
            *reinterpret_cast<VT*>(p + c) = w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < V; ++i) p[i] = r.v[i];
    }
}

}  // namespace bgsmm

template <typename T, int V, bool C16, bool ZERO, int NIN, class G>
__device__ __forceinline__ void
bgs_mm(G g, int nblk, int n, int L, int NC, const BgsBlock* __restrict__ blocks, const uint16_t* __restrict__ meta,
       const int* __restrict__ ci, const uint16_t* __restrict__ c16, const T* __restrict__ av,
       const T* __restrict__ dinv, const T* __restrict__ mid, const T* __restrict__ X, const T* __restrict__ Bv,
       T* __restrict__ Y, const int* __restrict__ stop) {
    using R = bgsmm::Row<T, V>;
    __shared__ R su[WAVES][64], sw[WAVES][64];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int gw = xcd_block(g.bid(), g.nb()) * WAVES + wv;
    const int blk = gw / L;
    const int col = (gw % L) * V;
    const int bl = min(blk, nblk - 1);
    const int stopped = *stop;
    const BgsBlock B = blocks[bl];
    if (stopped | (blk >= nblk)) return;   // whole waves only
    const int row0 = bl * 64;
    const int i = row0 + lane;
    const bool live = i < n;
    const int ir = live ? i : row0;
    const int mt = meta[ir];
    const int nin = live ? (mt & 0xff) : 0;
    const int colour = live ? (mt >> 8) : -1;
    const T di = dinv[ir], mi = mid[ir];
    R br, xr;
    bgsmm::load_row(br, Bv + (int64_t)ir * NC + col);
#pragma unroll
    for (int c = 0; c < V; ++c) xr.v[c] = T(0);
    if (!ZERO) bgsmm::load_row(xr, X + (int64_t)ir * NC + col);
#pragma unroll
    for (int c = 0; c < V; ++c) {
        su[wv][lane].v[c] = T(0);
        sw[wv][lane].v[c] = T(0);
    }
    const int W = B.width, cb = B.cbase;
    const int e0 = B.base + lane;
    T a[NIN];
    int id[NIN];
#pragma unroll
    for (int t = 0; t < NIN; ++t) {
        a[t] = T(0);
        id[t] = lane;
        if (!ZERO || t < (B.info & 0xff)) {
            a[t] = av[e0 + t * 64];
            id[t] = bgs_code<C16>(ci, c16, e0 + t * 64);
        }
    }
    R acc;
#pragma unroll
    for (int c = 0; c < V; ++c) acc.v[c] = T(0);
    if (!ZERO) {
#pragma unroll
        for (int t = 0; t < NIN; ++t) {
            const int j = t < W ? bgs_col<C16>(t, nin, id[t], row0, cb) : row0;
            const T v = t < W ? a[t] : T(0);
            R xj;
            bgsmm::load_row(xj, X + (int64_t)j * NC + col);
#pragma unroll
            for (int c = 0; c < V; ++c) acc.v[c] = fma(v, xj.v[c], acc.v[c]);
        }
#pragma unroll 4
        for (int t = NIN; t < W; ++t) {   // outside entries (or padding) in every row
            const int e = e0 + t * 64;
            const int code = bgs_code<C16>(ci, c16, e);
            const T v = av[e];
            R xj;
            bgsmm::load_row(xj, X + (int64_t)(C16 ? cb + code : code) * NC + col);
#pragma unroll
            for (int c = 0; c < V; ++c) acc.v[c] = fma(v, xj.v[c], acc.v[c]);
        }
    }
#pragma unroll
    for (int t = 0; t < NIN; ++t) {   // keep the inside couplings: value 0 / own position elsewhere
        const bool in = t < nin;
        a[t] = in ? a[t] : T(0);
        id[t] = in ? id[t] : lane;
    }
    R r0;
#pragma unroll
    for (int c = 0; c < V; ++c) r0.v[c] = br.v[c] - acc.v[c];
    wave_sync();
    R uq, wq;
#pragma unroll
    for (int c = 0; c < V; ++c) uq.v[c] = wq.v[c] = T(0);
    for (int k = 0; k < (B.info >> 8); ++k) {
        if (colour == k) {
            R s;
#pragma unroll
            for (int c = 0; c < V; ++c) s.v[c] = T(0);
#pragma unroll
            for (int t = 0; t < NIN; ++t) {
                const R z = su[wv][id[t]];
#pragma unroll
                for (int c = 0; c < V; ++c) s.v[c] = fma(a[t], z.v[c], s.v[c]);
            }
#pragma unroll
            for (int c = 0; c < V; ++c) uq.v[c] = (r0.v[c] - s.v[c]) * di;
            su[wv][lane] = uq;
        }
        wave_sync();
    }
    for (int k = (B.info >> 8) - 1; k >= 0; --k) {
        if (colour == k) {
            R s;
#pragma unroll
            for (int c = 0; c < V; ++c) s.v[c] = T(0);
#pragma unroll
            for (int t = 0; t < NIN; ++t) {
                const R z = sw[wv][id[t]];
#pragma unroll
                for (int c = 0; c < V; ++c) s.v[c] = fma(a[t], z.v[c], s.v[c]);
            }
#pragma unroll
            for (int c = 0; c < V; ++c) wq.v[c] = (mi * uq.v[c] - s.v[c]) * di;
            sw[wv][lane] = wq;
        }
        wave_sync();
    }
    if (!live) return;
    R out;
#pragma unroll
    for (int c = 0; c < V; ++c) out.v[c] = ZERO ? wq.v[c] : xr.v[c] + wq.v[c];
    bgsmm::store_row(out, Y + (int64_t)i * NC + col);
}

template <typename T, int V, bool C16, bool ZERO, int NIN>
struct BgsMM {
    static constexpr int block = BLOCK;
    using sig = decltype(&bgs_mm<T, V, C16, ZERO, NIN, HwGrid>);
    template <class G, class... A>
    __device__ static void run(G g, A... a) { bgs_mm<T, V, C16, ZERO, NIN, G>(g, a...); }
};

// Y = B - A X on the block layout for V columns per wave (TV: value type, FP64 values
// with FP32 blocks sum in FP64 and round once).
template <typename T, int V, bool C16, typename TV, class G>
__device__ __forceinline__ void
bgs_resid_mm(G g, int nblk, int n, int L, int NC, const BgsBlock* __restrict__ blocks,
             const uint16_t* __restrict__ meta, const int* __restrict__ ci, const uint16_t* __restrict__ c16,
             const TV* __restrict__ av, const T* __restrict__ X, const T* __restrict__ Bv, T* __restrict__ Y,
             const int* __restrict__ stop) {
    using TA = typename std::conditional<(sizeof(TV) > sizeof(T)), TV, T>::type;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int gw = xcd_block(g.bid(), g.nb()) * WAVES + wv;
    const int blk = gw / L;
    const int col = (gw % L) * V;
    const int bl = min(blk, nblk - 1);
    const int stopped = *stop;
    const BgsBlock B = blocks[bl];
    if (stopped | (blk >= nblk)) return;
    const int row0 = bl * 64;
    const int i = row0 + lane;
    const bool live = i < n;
    const int ir = live ? i : row0;
    const int nin = live ? (meta[ir] & 0xff) : 0;
    const int e0 = B.base + lane;
    const int cb = B.cbase;
    TA acc[V];
#pragma unroll
    for (int c = 0; c < V; ++c) acc[c] = 0;
#pragma unroll 4
    for (int t = 0; t < B.width; ++t) {
        const int e = e0 + t * 64;
        const int code = bgs_code<C16>(ci, c16, e);
        const TA v = av[e];
        bgsmm::Row<T, V> xj;
        bgsmm::load_row(xj, X + (int64_t)bgs_col<C16>(t, nin, code, row0, cb) * NC + col);
#pragma unroll
        for (int c = 0; c < V; ++c) acc[c] = fma(v, (TA)xj.v[c], acc[c]);
    }
    if (!live) return;
    bgsmm::Row<T, V> br, out;
    bgsmm::load_row(br, Bv + (int64_t)i * NC + col);
#pragma unroll
    for (int c = 0; c < V; ++c) out.v[c] = (T)((TA)br.v[c] - acc[c]);
    bgsmm::store_row(out, Y + (int64_t)i * NC + col);
}

template <typename T, int V, bool C16, typename TV>
struct BgsResidMM {
    static constexpr int block = BLOCK;
    using sig = decltype(&bgs_resid_mm<T, V, C16, TV, HwGrid>);
    template <class G, class... A>
    __device__ static void run(G g, A... a) { bgs_resid_mm<T, V, C16, TV, G>(g, a...); }
};

}  // namespace dev
}  // namespace amge
