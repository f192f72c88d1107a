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
// Layout per block (jagged diagonals): the lanes hold the block's rows sorted by length,
// longest first, and slab t holds entry t of the rows longer than t, contiguously, so
// the block stores exactly its entries (no padding): entry t of lane q sits at
// base + (entries of slabs 0..t-1) + q.  Slabs below the block's shortest row hold every
// row (sizes from the block record, so these loads need no per-lane word); past it the
// slab sizes come from a ballot of the lanes' lengths.  A row's entries inside the block
// come first (code: the column's position in the block), then the others (code: column,
// or a 16-bit offset from the block's base column).  Per lane a 32-bit word: inside
// entries | colour << 8 | length << 16 | position of its row in the block << 24 (0xff:
// no row); u and w live in LDS by position in the block.  Every lane loads every slab of
// a loop, its entries past its row's length included (they lie inside the arrays, which
// end with spare slots; the values are masked), so a row's loads are in flight together:
// the first NIN slabs (NIN >= every block's inside width, so they hold the inside
// entries) are loaded together, then gathered together; the rest follow in a uniform
// loop; the colour passes read LDS without per-lane branches.  The inside couplings stay
// in registers, u and w in LDS; the single-column sweep synchronises the wave only.  A
// sweep from x0 = 0 reads the block's first wi slabs only (wi: its most inside entries
// of a row).
//
// Bytes: a full sweep reads every entry once (value + 2- or 4-byte code) plus b, x, the
// row data and writes y, like an l1-Jacobi sweep.
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

// Column of entry t of a row with nin inside entries (code: the column's position in the
// block, else the column or its offset from the block's base column).
template <bool C16>
__device__ __forceinline__ int bgs_col(int t, int nin, int code, int row0, int cb) {
    return t < nin ? row0 + code : (C16 ? cb + code : code);
}

template <bool C16>
__device__ __forceinline__ int bgs_code(const int* __restrict__ ci, const uint16_t* __restrict__ c16, int e) {
    return C16 ? (int)c16[e] : ci[e];
}

// A product rounded on its own: never contracted with the sum that follows it, so that
// every instance of a sweep (single column, any batched shape) rounds alike.
__device__ __forceinline__ float bgs_mul(float a, float b) { return __fmul_rn(a, b); }
__device__ __forceinline__ double bgs_mul(double a, double b) { return __dmul_rn(a, b); }

// Lanes whose rows are longer than t: a prefix of the wave (rows sorted by length).
__device__ __forceinline__ int bgs_slab(int len, int t) {
    return __popcll(__ballot(len > t));
}

// Shape of a block from its record: shortest row length and rows (the slabs below the
// shortest length are full).
struct BgsShape {
    int minlen, nlive;
    __device__ explicit BgsShape(int info) : minlen((info >> 16) & 0xff), nlive(info >> 24) {}
};

// Offsets of slabs t0 .. t0 + CH - 1 for this lane, e advanced past them.  Full slabs
// (the uniform branch) take their sizes from the block record, so their loads do not
// wait for the lane's length.
template <int CH>
__device__ __forceinline__ void bgs_offsets(int& e, int len, int t0, BgsShape sh, int (&ee)[CH]) {
    if (t0 + CH <= sh.minlen) {
#pragma unroll
        for (int k = 0; k < CH; ++k) ee[k] = e + k * sh.nlive;
        e += CH * sh.nlive;
    } else {
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            ee[k] = e;
            e += bgs_slab(len, t0 + k);
        }
    }
}

// Entries t0 .. t0 + CH - 1 of this lane's row (or a masked stand-in past its length):
// offsets first, then the CH loads together.
template <int CH, typename TV, bool C16>
__device__ __forceinline__ void bgs_chunk(int& e, int len, int t0, BgsShape sh, const TV* __restrict__ av,
                                          const int* __restrict__ ci, const uint16_t* __restrict__ c16,
                                          TV (&v)[CH], int (&code)[CH]) {
    int ee[CH];
    bgs_offsets<CH>(e, len, t0, sh, ee);
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        v[k] = av[ee[k]];
        code[k] = bgs_code<C16>(ci, c16, ee[k]);
    }
}

// Slabs per chunk of the streaming loops: 16 for kernels with few inside entries (long
// rows of coarse levels), 8 otherwise.
template <int NIN>
constexpr int bgs_ch() {
    return NIN <= 8 ? 16 : 8;
}

// y = x + w (ZERO: x = 0, y = w) for every block; NIN >= every block's inside width.
template <typename T, bool C16, bool ZERO, int NIN>
__global__ void __launch_bounds__(BLOCK)
k_bgs(int nblk, int n, const BgsBlock* __restrict__ blocks, const uint32_t* __restrict__ meta,
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
    const uint32_t mt = meta[row0 + lane];
    const int pos = mt >> 24;                 // this lane's row in the block (0xff: none)
    const bool live = pos != 0xff;
    const int nin = mt & 0xff, colour = live ? (int)((mt >> 8) & 0xff) : -1;
    const int len = (mt >> 16) & 0xff;
    const int ir = row0 + (live ? pos : 0);
    const T br = b[ir], di = dinv[ir], mi = mid[ir];
    const T xr = ZERO ? T(0) : x[ir];
    su[wv][lane] = T(0);
    sw[wv][lane] = T(0);
    const int W = B.width, cb = B.cbase;
    const int wi = B.info & 0xff, ncol = (B.info >> 8) & 0xff;
    const BgsShape sh(B.info);
    int e = B.base + lane;    // entry t of this lane: slab base + lane
    T a[NIN];
    int id[NIN];
    {
        int ee[NIN];
        bgs_offsets<NIN>(e, len, 0, sh, ee);
#pragma unroll
        for (int t = 0; t < NIN; ++t) {
            a[t] = T(0);
            id[t] = 0;
            if (!ZERO || t < wi) {   // a sweep from zero reads the inside slabs only
                a[t] = av[ee[t]];
                id[t] = bgs_code<C16>(ci, c16, ee[t]);
            }
        }
    }
    T acc = 0;
    if (!ZERO) {
#pragma unroll
        for (int t = 0; t < NIN; ++t) {
            const bool on = t < len;
            const int j = on ? bgs_col<C16>(t, nin, id[t], row0, cb) : row0;
            acc = fma(on ? a[t] : T(0), x[j], acc);
        }
        constexpr int CH = bgs_ch<NIN>();
        for (int t0 = NIN; t0 < W; t0 += CH) {   // outside entries, CH slabs at a time
            T v[CH];
            int code[CH];
            bgs_chunk<CH, T, C16>(e, len, t0, sh, av, ci, c16, v, code);
#pragma unroll
            for (int k = 0; k < CH; ++k) {
                const bool on = t0 + k < len;
                acc = fma(on ? v[k] : T(0), x[on ? (C16 ? cb + code[k] : code[k]) : row0], acc);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < NIN; ++t) {   // keep the inside couplings: value 0 / own position elsewhere
        const bool in = t < nin;
        a[t] = in ? a[t] : T(0);
        id[t] = in ? id[t] : (live ? pos : 0);
    }
    const T r0 = br - acc;
    wave_sync();
    // forward: (D_l1 + L) u = r0, colours in increasing order (u by position in the block)
    T uq = 0;
    for (int c = 0; c < ncol; ++c) {
        if (colour == c) {
            T s = 0;
#pragma unroll
            for (int t = 0; t < NIN; ++t) s = fma(a[t], su[wv][id[t]], s);
            uq = bgs_mul(r0 - s, di);
            su[wv][pos] = uq;
        }
        wave_sync();
    }
    // backward: (D_l1 + U) w = (D + 2 D_l1) u, colours in decreasing order
    const T v = bgs_mul(mi, uq);
    T wq = 0;
    for (int c = ncol - 1; c >= 0; --c) {
        if (colour == c) {
            T s = 0;
#pragma unroll
            for (int t = 0; t < NIN; ++t) s = fma(a[t], sw[wv][id[t]], s);
            wq = bgs_mul(v - s, di);
            sw[wv][pos] = wq;
        }
        wave_sync();
    }
    if (live) y[ir] = ZERO ? wq : xr + wq;
}

// y = b - A x on the same layout (the residual ahead of the restriction, so that the
// V-cycle reads one copy of A).  TV: value type; FP64 values with FP32 vectors sum in
// FP64 and round once.
template <typename T, bool C16, typename TV>
__global__ void __launch_bounds__(BLOCK)
k_bgs_resid(int nblk, int n, const BgsBlock* __restrict__ blocks, const uint32_t* __restrict__ meta,
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
    const uint32_t mt = meta[row0 + lane];
    const int pos = mt >> 24;
    const bool live = pos != 0xff;
    const int nin = mt & 0xff, len = (mt >> 16) & 0xff;
    const int ir = row0 + (live ? pos : 0);
    const T br = b[ir];
    const int cb = B.cbase;
    const BgsShape sh(B.info);
    int e = B.base + lane;
    TA acc = 0;
    for (int t0 = 0; t0 < B.width; t0 += 8) {   // eight slabs at a time
        TV v[8];
        int code[8];
        bgs_chunk<8, TV, C16>(e, len, t0, sh, av, ci, c16, v, code);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const bool on = t0 + k < len;
            acc = fma(on ? (TA)v[k] : TA(0), (TA)x[on ? bgs_col<C16>(t0 + k, nin, code[k], row0, cb) : row0], acc);
        }
    }
    if (live) y[ir] = (T)((TA)br - acc);
}

// ---------------------------------------------------------------------------------
// Batched sweeps (n x NC row-major blocks): the block layout above on the first W
// columns, a lane holding V consecutive columns of a row.  P = 1: a wave holds a 64-row
// block, one row per lane; P = 4: the four waves of a workgroup share a block, 16 rows
// each, with a row's four column groups in neighbouring lanes.  L = W / (P V) groups of
// waves per block each read the block's entries (L1/L2 hits after the first).  Every
// column goes through exactly the arithmetic of the single-column sweep, so a column's
// result depends neither on W, V, P nor the other columns.  Bodies of grid objects G
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

template <typename T, int V, int P, bool C16, bool ZERO, int NIN, class G>
__device__ __forceinline__ void
bgs_mm(G g, int nblk, int n, int L, int NC, const BgsBlock* __restrict__ blocks, const uint32_t* __restrict__ meta,
       const int* __restrict__ ci, const uint16_t* __restrict__ c16, const T* __restrict__ av,
       const T* __restrict__ dinv, const T* __restrict__ mid, const T* __restrict__ X, const T* __restrict__ Bv,
       T* __restrict__ Y, const int* __restrict__ stop) {
    static_assert(P == 1 || P == 4, "one or four waves per block");
    static_assert(P == 1 || P == WAVES, "four waves per block fill the workgroup");
    using R = bgsmm::Row<T, V>;
    // u and w by position in the block: P = 1, wave wv's block at wv * 64 + position;
    // P = 4, the workgroup's block, position * 4 + the lane's column group
    __shared__ R su[WAVES * 64], sw[WAVES * 64];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int gw = xcd_block(g.bid(), g.nb()) * WAVES + wv;
    const int task = gw / P, sub = gw % P;   // P waves per (block, group of P x V columns)
    const int blk = task / L;
    const int q = lane % P;
    const int col = (task % L) * (P * V) + q * V;
    const int bl = min(blk, nblk - 1);
    const int stopped = *stop;
    const BgsBlock B = blocks[bl];
    if (stopped | (blk >= nblk)) return;   // whole waves (P = 4: the whole workgroup)
    const int row0 = bl * 64;
    const int slot = sub * (64 / P) + lane / P;   // this lane's row slot in the block
    const uint32_t ws = meta[row0 + lane];         // slot `lane`: the slab sizes
    const uint32_t mt = P == 1 ? ws : (uint32_t)__shfl((int)ws, slot);
    const int pos = mt >> 24;
    const bool live = pos != 0xff;
    const int nin = mt & 0xff, colour = live ? (int)((mt >> 8) & 0xff) : -1;
    const int len = (mt >> 16) & 0xff;
    const int ir = row0 + (live ? pos : 0);
    const int lb = P == 1 ? wv * 64 : q;   // LDS index of position p: lb + p * P
    const T di = dinv[ir], mi = mid[ir];
    R br, xr;
    bgsmm::load_row(br, Bv + (int64_t)ir * NC + col);
#pragma unroll
    for (int c = 0; c < V; ++c) xr.v[c] = T(0);
    if (!ZERO) bgsmm::load_row(xr, X + (int64_t)ir * NC + col);
#pragma unroll
    for (int c = 0; c < V; ++c) {
        su[lb + slot * P].v[c] = T(0);
        sw[lb + slot * P].v[c] = T(0);
    }
    const int W = B.width, cb = B.cbase;
    const int wi = B.info & 0xff, ncol = (B.info >> 8) & 0xff;
    const BgsShape sh(B.info);
    int e = B.base + slot;
    T a[NIN];
    int id[NIN];
    {
        int ee[NIN];
        bgs_offsets<NIN>(e, (ws >> 16) & 0xff, 0, sh, ee);
#pragma unroll
        for (int t = 0; t < NIN; ++t) {
            a[t] = T(0);
            id[t] = 0;
            if (!ZERO || t < wi) {
                a[t] = av[ee[t]];
                id[t] = bgs_code<C16>(ci, c16, ee[t]);
            }
        }
    }
    R acc;
#pragma unroll
    for (int c = 0; c < V; ++c) acc.v[c] = T(0);
    if (!ZERO) {
#pragma unroll
        for (int t = 0; t < NIN; ++t) {
            const bool on = t < len;
            const int j = on ? bgs_col<C16>(t, nin, id[t], row0, cb) : row0;
            const T v = on ? a[t] : T(0);
            R xj;
            bgsmm::load_row(xj, X + (int64_t)j * NC + col);
#pragma unroll
            for (int c = 0; c < V; ++c) acc.v[c] = fma(v, xj.v[c], acc.v[c]);
        }
        constexpr int CH = bgs_ch<NIN>();
        for (int t0 = NIN; t0 < W; t0 += CH) {   // outside entries, CH slabs at a time
            T v[CH];
            int code[CH];
            bgs_chunk<CH, T, C16>(e, (ws >> 16) & 0xff, t0, sh, av, ci, c16, v, code);
#pragma unroll
            for (int k = 0; k < CH; ++k) {
                const bool on = t0 + k < len;
                R xj;
                bgsmm::load_row(xj, X + (int64_t)(on ? (C16 ? cb + code[k] : code[k]) : row0) * NC + col);
#pragma unroll
                for (int c = 0; c < V; ++c) acc.v[c] = fma(on ? v[k] : T(0), xj.v[c], acc.v[c]);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < NIN; ++t) {   // keep the inside couplings: value 0 / own position elsewhere
        const bool in = t < nin;
        a[t] = in ? a[t] : T(0);
        id[t] = in ? id[t] : (live ? pos : 0);
    }
    R r0;
#pragma unroll
    for (int c = 0; c < V; ++c) r0.v[c] = br.v[c] - acc.v[c];
    // P = 1 orders the wave's own LDS accesses; P = 4 the workgroup's (one block)
    auto sync = [] {
        if (P == 1) wave_sync();
        else __syncthreads();
    };
    sync();
    R uq, wq;
#pragma unroll
    for (int c = 0; c < V; ++c) uq.v[c] = wq.v[c] = T(0);
    for (int k = 0; k < ncol; ++k) {
        if (colour == k) {
            R s;
#pragma unroll
            for (int c = 0; c < V; ++c) s.v[c] = T(0);
#pragma unroll
            for (int t = 0; t < NIN; ++t) {
                const R z = su[lb + id[t] * P];
#pragma unroll
                for (int c = 0; c < V; ++c) s.v[c] = fma(a[t], z.v[c], s.v[c]);
            }
#pragma unroll
            for (int c = 0; c < V; ++c) uq.v[c] = bgs_mul(r0.v[c] - s.v[c], di);
            su[lb + pos * P] = uq;
        }
        sync();
    }
    for (int k = ncol - 1; k >= 0; --k) {
        if (colour == k) {
            R s;
#pragma unroll
            for (int c = 0; c < V; ++c) s.v[c] = T(0);
#pragma unroll
            for (int t = 0; t < NIN; ++t) {
                const R z = sw[lb + id[t] * P];
#pragma unroll
                for (int c = 0; c < V; ++c) s.v[c] = fma(a[t], z.v[c], s.v[c]);
            }
#pragma unroll
            for (int c = 0; c < V; ++c) wq.v[c] = bgs_mul(bgs_mul(mi, uq.v[c]) - s.v[c], di);
            sw[lb + pos * P] = wq;
        }
        sync();
    }
    if (!live) return;
    R out;
#pragma unroll
    for (int c = 0; c < V; ++c) out.v[c] = ZERO ? wq.v[c] : xr.v[c] + wq.v[c];
    bgsmm::store_row(out, Y + (int64_t)ir * NC + col);
}

template <typename T, int V, int P, bool C16, bool ZERO, int NIN>
struct BgsMM {
    static constexpr int block = BLOCK;
    using sig = decltype(&bgs_mm<T, V, P, C16, ZERO, NIN, HwGrid>);
    template <class G, class... A>
    __device__ static void run(G g, A... a) { bgs_mm<T, V, P, C16, ZERO, NIN, G>(g, a...); }
};

// Y = B - A X on the block layout for P x V columns per group of P waves (TV: value
// type, FP64 values with FP32 blocks sum in FP64 and round once).  P = 1: a wave holds
// the block's 64 rows, one per lane, and V columns.  P = 4: four waves share a block,
// each 16 rows, and the four lanes of a row hold V consecutive columns each, so that a
// row's P x V columns (128 bytes) are one cache line for the four lanes' vector accesses.
template <typename T, int V, int P, bool C16, typename TV, class G>
__device__ __forceinline__ void
bgs_resid_mm(G g, int nblk, int n, int L, int NC, const BgsBlock* __restrict__ blocks,
             const uint32_t* __restrict__ meta, const int* __restrict__ ci, const uint16_t* __restrict__ c16,
             const TV* __restrict__ av, const T* __restrict__ X, const T* __restrict__ Bv, T* __restrict__ Y,
             const int* __restrict__ stop) {
    static_assert(P == 1 || P == 4, "one or four waves per block");
    using TA = typename std::conditional<(sizeof(TV) > sizeof(T)), TV, T>::type;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int gw = xcd_block(g.bid(), g.nb()) * WAVES + wv;
    const int task = gw / P, sub = gw % P;   // P waves per (block, group of P x V columns)
    const int blk = task / L;
    const int col = (task % L) * (P * V) + (lane % P) * V;
    const int bl = min(blk, nblk - 1);
    const int stopped = *stop;
    const BgsBlock B = blocks[bl];
    if (stopped | (blk >= nblk)) return;
    const int row0 = bl * 64;
    const int slot = sub * (64 / P) + lane / P;   // this lane's row slot in the block
    const uint32_t ws = meta[row0 + lane];         // slot `lane`: the slab sizes
    const uint32_t mt = P == 1 ? ws : (uint32_t)__shfl((int)ws, slot);
    const int pos = mt >> 24;
    const bool live = pos != 0xff;
    const int nin = mt & 0xff, len = (mt >> 16) & 0xff;
    const int ir = row0 + (live ? pos : 0);
    const int cb = B.cbase;
    const BgsShape sh(B.info);
    int e = B.base + slot;
    TA acc[V];
#pragma unroll
    for (int c = 0; c < V; ++c) acc[c] = 0;
    for (int t0 = 0; t0 < B.width; t0 += 8) {   // eight slabs at a time
        TV v[8];
        int code[8];
        bgs_chunk<8, TV, C16>(e, (ws >> 16) & 0xff, t0, sh, av, ci, c16, v, code);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const bool on = t0 + k < len;
            bgsmm::Row<T, V> xj;
            bgsmm::load_row(xj, X + (int64_t)(on ? bgs_col<C16>(t0 + k, nin, code[k], row0, cb) : row0) * NC + col);
#pragma unroll
            for (int c = 0; c < V; ++c) acc[c] = fma(on ? (TA)v[k] : TA(0), (TA)xj.v[c], acc[c]);
        }
    }
    if (!live) return;
    bgsmm::Row<T, V> br, out;
    bgsmm::load_row(br, Bv + (int64_t)ir * NC + col);
#pragma unroll
    for (int c = 0; c < V; ++c) out.v[c] = (T)((TA)br.v[c] - acc[c]);
    bgsmm::store_row(out, Y + (int64_t)ir * NC + col);
}

template <typename T, int V, int P, bool C16, typename TV>
struct BgsResidMM {
    static constexpr int block = BLOCK;
    using sig = decltype(&bgs_resid_mm<T, V, P, C16, TV, HwGrid>);
    template <class G, class... A>
    __device__ static void run(G g, A... a) { bgs_resid_mm<T, V, P, C16, TV, G>(g, a...); }
};

}  // namespace dev
}  // namespace amge
