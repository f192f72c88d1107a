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

}  // namespace dev
}  // namespace amge
