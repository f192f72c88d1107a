// Batched (multiple right-hand sides) kernels: the V-cycle and PCG on NC columns at once.
//
// Vectors are row-major n x NC.  A row of a level matrix is read once for all active
// columns: the lanes of a row own disjoint groups of V consecutive columns (V-wide
// vector loads), so every matrix entry is a broadcast load shared by the row's lanes
// and each gathered vector row is a contiguous segment.  No cross-lane reduction is
// needed; each lane runs the row's entries sequentially, in CSR order.  The matrices
// are in the sliced-ELL layout with one lane per row (K = 1), so the entries read by a
// wave are consecutive.
#pragma once

#include <type_traits>

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "grouped.hpp"
#include "kernels.hpp"

namespace amge {
namespace dev {

// Product rounded on its own (never contracted into a following addition).
__device__ __forceinline__ float mul_rn(float a, float b) { return __fmul_rn(a, b); }
__device__ __forceinline__ double mul_rn(double a, double b) { return __dmul_rn(a, b); }

// V consecutive values of one row of a vector block, moved with 16-byte (or narrower)
// vector loads and stores.
template <typename T, int V> struct Vec;
template <> struct Vec<float, 1> { using type = float; };
template <> struct Vec<float, 2> { using type = float2; };
template <> struct Vec<float, 4> { using type = float4; };
template <> struct Vec<double, 1> { using type = double; };
template <> struct Vec<double, 2> { using type = double2; };

template <typename T, int V>
struct Pack {
    static constexpr int W = (V * (int)sizeof(T) > 16) ? 16 / (int)sizeof(T) : V;   // values per access
    using VT = typename Vec<T, W>::type;
    T v[V];
    __device__ __forceinline__ void load(const T* p) {
#pragma unroll
        for (int c = 0; c < V; c += W) {
            const VT w = *reinterpret_cast<const VT*>(p + c);
            const T* s = reinterpret_cast<const T*>(&w);
#pragma unroll
            for (int i = 0; i < W; ++i) v[c + i] = s[i];
        }
    }
    __device__ __forceinline__ void store(T* p) const {
#pragma unroll
        for (int c = 0; c < V; c += W) {
            VT w;
            T* s = reinterpret_cast<T*>(&w);
#pragma unroll
            for (int i = 0; i < W; ++i) s[i] = v[c + i];
            *reinterpret_cast<VT*>(p + c) = w;
        }
    }
};

// Row-major SpMM level operator on the sliced-ELL layout with one lane per row (K = 1:
// entry t of slot rr of a slice at base + t * 64 + rr, rows in CSR entry order).  The
// first W of the NC columns are computed: L = W / V lanes share a row, each owning V
// consecutive columns (16- to 64-byte vector loads of the gathered rows), so a wave
// covers 64 / L consecutive slots of one slice and a slice takes L waves; the matrix
// entries of those slots are consecutive (coalesced), each broadcast to the L lanes of
// its row.  Every column sums its row's entries in CSR order whatever W, L and V are.
// Modes as in Mode (kernels.hpp); YD (SPMV, SPLIT) also receives dinv * y.  TV: the
// matrix value type (T by default; FP64 values with FP32 blocks sum in FP64 and round
// each result once, as in k_sell).
template <typename T, int V, int MODE, bool C16, class G, typename TV = T>
__device__ __forceinline__ void
sell_mm(G g, int nslices, int L, int NC, const int* __restrict__ sptr, const int* __restrict__ srow,
          const int* __restrict__ ci, const uint16_t* __restrict__ c16, const int* __restrict__ cbase,
          const TV* __restrict__ av, const T* __restrict__ X, const T* __restrict__ B, const T* __restrict__ dinv,
          T* __restrict__ Y, T* __restrict__ YD, const uint16_t* __restrict__ lead, const int* __restrict__ stop) {
    using TA = typename std::conditional<(sizeof(TV) > sizeof(T)), TV, T>::type;   // accumulation
    const int gw = xcd_block(g.bid(), g.nb()) * WAVES + ((int)threadIdx.x >> 6);
    const int slice = gw / L;
    const int lane = threadIdx.x & 63;
    const int rr = (gw % L) * (64 / L) + lane / L;
    const int col = (lane % L) * V;
    // stop flag (every column of the batch has converged) and layout words requested
    // together, from a clamped (valid) slice index, as in k_sell
    const int sl = min(slice, nslices - 1);
    const int stopped = *stop;
    const int base = sptr[sl];
    const int end = sptr[sl + 1];
    const int row = srow[sl * 64 + rr];
    const int cb = C16 ? cbase[sl] : 0;
    const int nlead = MODE == SPLIT ? lead[sl * 64 + rr] : 0;
    if (stopped | (slice >= nslices) | (end < base) | (row < -1) | (cb < 0)) return;   // last three never hold
    const int width = (end - base) >> 6;
    Pack<TA, V> acc;
#pragma unroll
    for (int i = 0; i < V; ++i) acc.v[i] = 0;
#pragma unroll 4
    for (int k = 0; k < width; ++k) {
        const int e = base + k * 64 + rr;
        const int j = C16 ? cb + (int)c16[e] : ci[e];
        const TA a = av[e];
        Pack<T, V> xv;
        if (MODE == SPLIT) {
            xv.load((k < nlead ? B : X) + (int64_t)j * NC + col);
        } else if (MODE == JAC0) {   // x_j = dinv_j b_j, the product the producer of b would store
            xv.load(B + (int64_t)j * NC + col);
            const T dj = dinv[j];
#pragma unroll
            for (int i = 0; i < V; ++i) xv.v[i] = dj * xv.v[i];
        } else {
            xv.load(X + (int64_t)j * NC + col);
        }
#pragma unroll
        for (int i = 0; i < V; ++i) acc.v[i] = fma(a, (TA)xv.v[i], acc.v[i]);
    }
    if (row < 0) return;
    const int64_t o = (int64_t)row * NC + col;
    Pack<T, V> out;
    if (MODE == SPMV || MODE == SPLIT) {
#pragma unroll
        for (int i = 0; i < V; ++i) out.v[i] = (T)acc.v[i];
        out.store(Y + o);
        if (YD) {
            const T d = dinv[row];
#pragma unroll
            for (int i = 0; i < V; ++i) out.v[i] = d * (T)acc.v[i];
            out.store(YD + o);
        }
    } else if (MODE == SPMV_ADD) {
        out.load(Y + o);
#pragma unroll
        for (int i = 0; i < V; ++i) out.v[i] += (T)acc.v[i];
        out.store(Y + o);
    } else if (MODE == RESID) {
        Pack<T, V> bv;
        bv.load(B + o);
#pragma unroll
        for (int i = 0; i < V; ++i) out.v[i] = (T)((TA)bv.v[i] - acc.v[i]);
        out.store(Y + o);
    } else if (MODE == JAC0) {
        Pack<T, V> bv;
        bv.load(B + o);
        const T d = dinv[row];
        // x0 = dinv b rounded on its own (not contracted into the update), as if stored
#pragma unroll
        for (int i = 0; i < V; ++i) out.v[i] = mul_rn(d, bv.v[i]) + d * (bv.v[i] - (T)acc.v[i]);
        out.store(Y + o);
    } else {   // JAC
        Pack<T, V> bv, xv;
        bv.load(B + o);
        xv.load(X + o);
        const T d = dinv[row];
#pragma unroll
        for (int i = 0; i < V; ++i) out.v[i] = xv.v[i] + d * (bv.v[i] - (T)acc.v[i]);
        out.store(Y + o);
    }
}

// Launch tags of the batched bodies: block size, the solo signature, the body.
template <typename T, int V, int MODE, bool C16, typename TV = T>
struct SellMM {
    static constexpr int block = BLOCK;
    using sig = decltype(&sell_mm<T, V, MODE, C16, HwGrid, TV>);
    template <class G, class... A>
    __device__ static void run(G g, A... a) { sell_mm<T, V, MODE, C16, G, TV>(g, a...); }
};

// Y += D X for a signed incidence in the same layout (index-only entries, bit 31 =
// sign, padding 0xffffffff).
template <typename T, int V, class G>
__device__ __forceinline__ void
sell_inc_mm_add(G g, int nslices, int L, int NC, const int* __restrict__ sptr, const int* __restrict__ srow,
                const uint32_t* __restrict__ ent, const T* __restrict__ X, T* __restrict__ Y,
                const int* __restrict__ stop) {
    const int gw = xcd_block(g.bid(), g.nb()) * WAVES + ((int)threadIdx.x >> 6);
    const int slice = gw / L;
    const int lane = threadIdx.x & 63;
    const int rr = (gw % L) * (64 / L) + lane / L;
    const int col = (lane % L) * V;
    const int sl = min(slice, nslices - 1);
    const int stopped = *stop;
    const int base = sptr[sl];
    const int end = sptr[sl + 1];
    const int row = srow[sl * 64 + rr];
    if (stopped | (slice >= nslices) | (end < base) | (row < 0)) return;
    const int width = (end - base) >> 6;
    Pack<T, V> acc;
    acc.load(Y + (int64_t)row * NC + col);
    for (int k = 0; k < width; ++k) {
        const uint32_t w = ent[base + k * 64 + rr];
        if (w == 0xffffffffu) continue;   // padding
        Pack<T, V> xv;
        xv.load(X + (int64_t)(w & 0x7fffffffu) * NC + col);
        const bool neg = w >> 31;
#pragma unroll
        for (int i = 0; i < V; ++i) acc.v[i] += neg ? -xv.v[i] : xv.v[i];
    }
    acc.store(Y + (int64_t)row * NC + col);
}

template <typename T, int V>
struct IncMMAdd {
    static constexpr int block = BLOCK;
    using sig = decltype(&sell_inc_mm_add<T, V, HwGrid>);
    template <class G, class... A>
    __device__ static void run(G g, A... a) { sell_inc_mm_add<T, V>(g, a...); }
};

// Dense FP64 operator (the coarsest inverse or the folded coarse tail): X = M B on the
// first W = 2^lgW of the NC = 2^lg stored columns; FP64 arithmetic.  A block computes
// R rows (R tuned per hierarchy; a row's sums do not depend on it).  Thread t owns columns c0 .. c0 + CPT - 1 (c0 = (t % TPJ) CPT, TPJ = NC /
// CPT threads per term) and the terms j = s, s + J, ... with s = t / TPJ, J = BLOCK /
// TPJ: the lanes of a wave read different entries of a row of M (coalesced), and a row of
// B in CPT-wide vector loads; four terms' loads of every row are issued at a time and
// summed in order.  The partial sums are then added over the terms' slots of a wave (a
// fixed butterfly) and over the waves in order.  The layout depends on NC only, so a
// column's result does not depend on W.
template <typename T, int CPT, int R, class Grid>
__device__ __forceinline__ void
coarse_mm(Grid gr, int n, int lgW, int lg, const double* __restrict__ Ainv, const T* __restrict__ B,
          T* __restrict__ X, const int* __restrict__ stop) {
    __shared__ double sh[WAVES * R * 64];   // per wave: R x NC sums (NC <= 64)
    const int stopped = *stop;   // tested before the store: its load overlaps the product
    const int NC = 1 << lg, W = 1 << lgW;
    const int TPJ = NC / CPT, J = BLOCK / TPJ;
    const int t = threadIdx.x;
    const int c0 = (t % TPJ) * CPT;
    const int r0 = (int)gr.bid() * R;
    const double* a[R];
#pragma unroll
    for (int r = 0; r < R; ++r) a[r] = Ainv + (int64_t)min(r0 + r, n - 1) * n;   // rows >= n: not stored
    double acc[R][CPT];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int i = 0; i < CPT; ++i) acc[r][i] = 0;
    if (c0 < W) {
        int j = t / TPJ;
        for (; j + 3 * J < n; j += 4 * J) {
            double av[4][R];
            Pack<T, CPT> bv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
#pragma unroll
                for (int r = 0; r < R; ++r) av[u][r] = __builtin_nontemporal_load(a[r] + j + u * J);
                bv[u].load(B + (int64_t)(j + u * J) * NC + c0);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int r = 0; r < R; ++r)
#pragma unroll
                    for (int i = 0; i < CPT; ++i) acc[r][i] = fma(av[u][r], (double)bv[u].v[i], acc[r][i]);
        }
        for (; j < n; j += J) {
            Pack<T, CPT> bv;
            bv.load(B + (int64_t)j * NC + c0);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double av = __builtin_nontemporal_load(a[r] + j);
#pragma unroll
                for (int i = 0; i < CPT; ++i) acc[r][i] = fma(av, (double)bv.v[i], acc[r][i]);
            }
        }
    }
    const int wave = t >> 6, lane = t & 63;
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int i = 0; i < CPT; ++i) {
            double v = acc[r][i];
            for (int m = TPJ; m < 64; m <<= 1) v += __shfl_xor(v, m, 64);
            if (lane < TPJ) sh[(wave * R + r) * 64 + c0 + i] = v;
        }
    __syncthreads();
    if (t < R * NC) {
        const int r = t >> lg, c = t & (NC - 1);
        if (c < W && r0 + r < n && !stopped) {
            double v = sh[r * 64 + c];
#pragma unroll
            for (int w = 1; w < WAVES; ++w) v += sh[(w * R + r) * 64 + c];
            X[(int64_t)(r0 + r) * NC + c] = (T)v;
        }
    }
}

template <typename T, int CPT, int R>
struct CoarseMM {
    static constexpr int block = BLOCK;
    using sig = decltype(&coarse_mm<T, CPT, R, HwGrid>);
    template <class G, class... A>
    __device__ static void run(G g, A... a) { coarse_mm<T, CPT, R>(g, a...); }
};

// ---------------------------------------------------------------- batched PCG
// Per-column partial sums over the rows of a block: the block's threads hold column
// (tid % NC) sums for row group tid / NC; reduced over row groups through LDS.
__device__ __forceinline__ void column_partials(double v, int W, int NC, double* sh, double* part, int nblk,
                                                unsigned bid) {
    sh[threadIdx.x] = v;
    __syncthreads();
    if ((int)threadIdx.x < W) {
        double t = 0;
        for (int g = threadIdx.x; g < BLOCK; g += NC) t += sh[g];
        part[(int64_t)threadIdx.x * nblk + bid] = t;
    }
    __syncthreads();
}

// Q = A P (FP64, the one-lane-per-row sliced ELL of A) and block partials of p.q per
// column.  Every block owns a contiguous range of slices; its threads are laid out for
// all NC columns (L = NC / V lanes per row, V columns each), so every column's sums run
// in the same order whatever the active width W is; lanes of columns >= W do no work.
template <int V, bool C16, class G>
__device__ __forceinline__ void
bpcg_ap(G gr, int nslices, int W, int NC, const int* __restrict__ sptr, const int* __restrict__ srow,
          const int* __restrict__ ci, const uint16_t* __restrict__ c16, const int* __restrict__ cbase,
          const double* __restrict__ av, const double* __restrict__ P, double* __restrict__ Q,
          double* __restrict__ part, const BatchStatus* __restrict__ bs) {
    __shared__ double sh[BLOCK * V];
    if (bs->all_done) return;
    const int L = NC / V, rpb = BLOCK / L;   // rpb: row slots per step (a multiple of 64 / L)
    const int g = (int)threadIdx.x / L, col = ((int)threadIdx.x % L) * V;
    const bool active = col < W;
    const int per = (nslices + (int)gr.nb() - 1) / (int)gr.nb();
    const int s0 = xcd_block(gr.bid(), gr.nb()) * per;
    const int s1 = min(nslices, s0 + per);
    Pack<double, V> dot;
#pragma unroll
    for (int i = 0; i < V; ++i) dot.v[i] = 0;
    for (int u = s0 * 64 + g; active && u < s1 * 64; u += rpb) {
        const int slice = u >> 6, rr = u & 63;
        const int base = sptr[slice];
        const int width = (sptr[slice + 1] - base) >> 6;
        const int row = srow[slice * 64 + rr];
        const int cb = C16 ? cbase[slice] : 0;
        Pack<double, V> acc;
#pragma unroll
        for (int i = 0; i < V; ++i) acc.v[i] = 0;
#pragma unroll 4
        for (int k = 0; k < width; ++k) {
            const int e = base + k * 64 + rr;
            const int j = C16 ? cb + (int)c16[e] : ci[e];
            const double a = av[e];
            Pack<double, V> xv;
            xv.load(P + (int64_t)j * NC + col);
#pragma unroll
            for (int i = 0; i < V; ++i) acc.v[i] = fma(a, xv.v[i], acc.v[i]);
        }
        if (row < 0) continue;
        const int64_t o = (int64_t)row * NC + col;
        acc.store(Q + o);
        Pack<double, V> pv;
        pv.load(P + o);
#pragma unroll
        for (int i = 0; i < V; ++i) dot.v[i] = fma(pv.v[i], acc.v[i], dot.v[i]);
    }
#pragma unroll
    for (int i = 0; i < V; ++i) sh[g * NC + col + i] = dot.v[i];
    __syncthreads();
    if ((int)threadIdx.x < W) {
        double t = 0;
        for (int q = 0; q < rpb; ++q) t += sh[q * NC + threadIdx.x];
        part[(int64_t)threadIdx.x * gr.nb() + gr.bid()] = t;
    }
}

template <int V, bool C16>
struct BpcgAp {
    static constexpr int block = BLOCK;
    using sig = decltype(&bpcg_ap<V, C16, HwGrid>);
    template <class G, class... A>
    __device__ static void run(G g, A... a) { bpcg_ap<V, C16>(g, a...); }
};

// Per-column totals of nq quantities from their block partials, stored at
// part[(q * NC + c) * nblk + block]: one wave per (q, c), fixed summation order
// (strided lane sums, then the butterfly).  Results in sh[q * NC + c].
__device__ __forceinline__ void col_totals(const double* __restrict__ part, int nblk, int nq, int W, int NC,
                                           double* sh) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    for (int qc = wave; qc < nq * NC; qc += nwaves) {
        if (qc % NC >= W) continue;   // idle columns beyond the active width
        const double* p = part + (int64_t)qc * nblk;
        // lane-wise sums in index order, eight loads issued at a time
        double t = 0;
        int i = lane;
        for (; i + 7 * 64 < nblk; i += 8 * 64) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = p[i + u * 64];
#pragma unroll
            for (int u = 0; u < 8; ++u) t += v[u];
        }
        for (; i < nblk; i += 64) t += p[i];
        t = wave_sum(t);
        if (lane == 0) sh[qc] = t;
    }
    __syncthreads();
}

// Block size of the single-block finalize kernels (one wave per column sum).
constexpr int FIN_BLOCK = 1024;

// alpha_c = delta_c / pq_c for live columns (breakdown if pq_c <= 0); fresh and idle
// columns take no step.  One block.
template <class G>
__device__ __forceinline__ void
bpcg_alpha(G, int W, int NC, const double* __restrict__ part, int nblk, ColState* __restrict__ cs,
             BatchStatus* __restrict__ bs) {
    __shared__ double sh[64];
    if (bs->all_done) return;
    col_totals(part, nblk, 1, W, NC, sh);
    const int c = threadIdx.x;
    if (c < W) {
        ColState& s = cs[c];
        const double pq = sh[c];
        s.pq = pq;
        s.pinit = 0;
        s.alpha = 0;
        if (!s.done && !s.fresh) {
            if (pq > 0 && isfinite(pq)) {
                s.alpha = s.delta / pq;
            } else {
                s.breakdown = isfinite(pq) ? 1 : 0;
                s.nonfinite = isfinite(pq) ? 0 : 1;
                s.done = 1;
            }
        }
    }
}

struct BpcgAlpha {
    static constexpr int block = FIN_BLOCK;
    using sig = decltype(&bpcg_alpha<HwGrid>);
    template <class G, class... A>
    __device__ static void run(G g, A... a) { bpcg_alpha(g, a...); }
};

// X += alpha P, R -= alpha Q per column; R32 = (float) R, RD32 = dinv32 * R32 (FP32
// preconditioner) or RD64 = dinv64 * R (FP64 preconditioner).
template <class G>
__device__ __forceinline__ void
bpcg_xr(G g, int64_t nn, int lgW, int lg, const ColState* __restrict__ cs, const double* __restrict__ Q,
          double* __restrict__ R, float* __restrict__ R32, float* __restrict__ RD32,
          const float* __restrict__ dinv32, double* __restrict__ RD64, const double* __restrict__ dinv64,
          const BatchStatus* __restrict__ bs) {
    if (bs->all_done) return;
    for (int64_t u = (int64_t)g.bid() * BLOCK + threadIdx.x; u < nn; u += (int64_t)g.nb() * BLOCK) {
        const int c = (int)(u & ((1 << lgW) - 1));
        const int64_t row = u >> lgW;
        const int64_t t = (row << lg) + c;
        const double a = cs[c].alpha;
        double r = R[t];
        if (a != 0) {
            r = fma(-a, Q[t], r);
            R[t] = r;
        }
        if (R32) {
            const float rf = (float)r;
            R32[t] = rf;
            if (RD32) RD32[t] = dinv32[row] * rf;
        }
        if (RD64) RD64[t] = dinv64[row] * r;
    }
}

struct BpcgXr {
    static constexpr int block = BLOCK;
    using sig = decltype(&bpcg_xr<HwGrid>);
    template <class G, class... A>
    __device__ static void run(G g, A... a) { bpcg_xr(g, a...); }
};

// Partials of r.z_new, r.z_old, r.r per column (the new and old z are the two z blocks,
// alternating with the iteration parity).  z has the preconditioner's precision (an
// FP32 z is exact in FP32), sums are FP64.
template <typename TZ, class G>
__device__ __forceinline__ void
bpcg_dots(G g, int n, int W, int NC, const TZ* __restrict__ Znew, const TZ* __restrict__ Zold,
          const double* __restrict__ R, double* __restrict__ part, const BatchStatus* __restrict__ bs) {
    __shared__ double sh[BLOCK];
    if (bs->all_done) return;
    const int rpb = BLOCK / NC;
    const int c = threadIdx.x % NC;   // layout of all NC columns; columns >= W idle
    double a = 0, b = 0, d = 0;
    for (int row = g.bid() * rpb + threadIdx.x / NC; c < W && row < n; row += g.nb() * rpb) {
        const int64_t t = (int64_t)row * NC + c;
        const double zn = (double)Znew[t], zo = (double)Zold[t], r = R[t];
        a = fma(r, zn, a);
        b = fma(r, zo, b);
        d = fma(r, r, d);
    }
    const int nb = g.nb();
    column_partials(a, W, NC, sh, part, nb, g.bid());
    column_partials(b, W, NC, sh, part + (int64_t)NC * nb, nb, g.bid());
    column_partials(d, W, NC, sh, part + (int64_t)2 * NC * nb, nb, g.bid());
}

template <typename TZ>
struct BpcgDots {
    static constexpr int block = BLOCK;
    using sig = decltype(&bpcg_dots<TZ, HwGrid>);
    template <class G, class... A>
    __device__ static void run(G g, A... a) { bpcg_dots<TZ>(g, a...); }
};

// Per-column stopping test and beta (one block).  A fresh column takes its initial
// quantities here (delta0 = r.z0, ||b||) and becomes live; a zero right-hand side is
// finished with 0 steps.
template <class G>
__device__ __forceinline__ void
bpcg_update(G, int W, int NC, const double* __restrict__ part, int nblk, ColState* __restrict__ cs,
              BatchStatus* __restrict__ bs) {
    __shared__ double sh[3 * 64];
    __shared__ int flags[2 * 64];
    if (bs->all_done) return;
    col_totals(part, nblk, 3, W, NC, sh);
    const int c = threadIdx.x;
    if (c >= W && c < NC) {   // idle columns beyond the active width
        flags[c] = cs[c].done;
        flags[64 + c] = cs[c].breakdown;
    }
    if (c < W) {
        ColState& s = cs[c];
        const double rz = sh[c], rzo = sh[NC + c], rr = sh[2 * NC + c];
        if (s.done) {
        } else if (s.fresh) {
            s.fresh = 0;
            s.delta0 = rz;
            s.delta = rz;
            s.bnorm = sqrt(rr);
            s.rr = rr;
            s.rz = rz;
            s.rzold = 0;
            s.relres = 1.0;
            s.iters = 0;
            s.beta = 0;
            if (!isfinite(rz) || !isfinite(rr)) {
                s.nonfinite = 1;
                s.done = 1;
            } else if (rr == 0) {
                s.relres = 0;
                s.done = 1;
            } else if (!(rz > 0)) {
                s.breakdown = 1;
                s.done = 1;
            } else {
                s.pinit = 1;
            }
        } else {
            s.rz = rz;
            s.rzold = rzo;
            s.rr = rr;
            s.iters += 1;
            const double rel = s.stop_l2 ? sqrt(rr) / s.bnorm : sqrt(fmax(rz, 0.0) / s.delta0);
            s.relres = rel;
            if (!isfinite(rz)) {
                s.nonfinite = 1;
                s.done = 1;
            } else if ((s.rtol > 0 && rel <= s.rtol) || s.iters >= s.maxit) {
                s.done = 1;
                s.beta = 0;
            } else {
                s.beta = (rz - rzo) / s.delta;
                s.delta = rz;
            }
        }
        flags[c] = s.done;
        flags[64 + c] = s.breakdown;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int live = 0, brk = 0;
        for (int j = 0; j < NC; ++j) {
            live += flags[j] ? 0 : 1;
            brk |= flags[64 + j];
        }
        bs->it += 1;
        bs->all_done_next = live == 0;
        bs->any_breakdown = brk;
    }
}

struct BpcgUpdate {
    static constexpr int block = FIN_BLOCK;
    using sig = decltype(&bpcg_update<HwGrid>);
    template <class G, class... A>
    __device__ static void run(G g, A... a) { bpcg_update(g, a...); }
};

// P = Z + beta P for live columns; P = Z for a column that has just taken its initial
// quantities.
template <typename TZ, class G>
__device__ __forceinline__ void
bpcg_p(G g, int64_t nn, int lgW, int lg, const ColState* __restrict__ cs, const TZ* __restrict__ Z,
         double* __restrict__ P, double* __restrict__ X, const BatchStatus* __restrict__ bs) {
    if (bs->all_done) return;   // the value at the start of the iteration (see bpcg_finish)
    for (int64_t u = (int64_t)g.bid() * BLOCK + threadIdx.x; u < nn; u += (int64_t)g.nb() * BLOCK) {
        const int c = (int)(u & ((1 << lgW) - 1));
        const int64_t t = ((u >> lgW) << lg) + c;
        const ColState& s = cs[c];
        const double z = (double)Z[t];
        const double p = P[t];
        // the step of this iteration, taken with the p it used (alpha is 0 for a column
        // that took none: idle, fresh, or stopped before the step)
        if (s.alpha != 0) X[t] = fma(s.alpha, p, X[t]);
        if (s.pinit) P[t] = z;
        else if (!s.done) P[t] = fma(s.beta, p, z);
    }
}

template <typename TZ>
struct BpcgP {
    static constexpr int block = BLOCK;
    using sig = decltype(&bpcg_p<TZ, HwGrid>);
    template <class G, class... A>
    __device__ static void run(G g, A... a) { bpcg_p<TZ>(g, a...); }
};

// Last kernel of a batched iteration (one thread): the stop flag computed by
// bpcg_update becomes current (bpcg_p, which applies the iteration's step to X, must
// still run in the iteration that finishes the last column).
template <class G>
__device__ __forceinline__ void bpcg_finish(G, BatchStatus* __restrict__ bs) {
    if (bs->all_done) return;
    bs->all_done = bs->all_done_next;
}

struct BpcgFinish {
    static constexpr int block = 1;
    using sig = decltype(&bpcg_finish<HwGrid>);
    template <class G, class... A>
    __device__ static void run(G g, A... a) { bpcg_finish(g, a...); }
};

// Loads a block of right-hand sides (caller layout n x nrhs) as fresh columns: R = b,
// X = P = 0; columns nrhs..NC-1 are idle and zero.
__global__ void __launch_bounds__(BLOCK)
k_bpcg_load(int64_t n, int nrhs, int lg, const double* __restrict__ b, double* __restrict__ R, double* __restrict__ X,
            double* __restrict__ P, ColState* __restrict__ cs, BatchStatus* __restrict__ bs, double rtol, int maxit,
            int stop_l2) {
    const int NC = 1 << lg;
    for (int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x; t < (n << lg); t += (int64_t)gridDim.x * BLOCK) {
        const int c = (int)(t & (NC - 1));
        R[t] = c < nrhs ? b[(t >> lg) * nrhs + c] : 0.0;
        X[t] = 0.0;
        P[t] = 0.0;
    }
    if (blockIdx.x == 0) {
        const int c = threadIdx.x;
        if (c < NC) {
            ColState s = {};
            s.rtol = rtol;
            s.maxit = maxit;
            s.stop_l2 = stop_l2;
            s.fresh = c < nrhs ? 1 : 0;
            s.done = c < nrhs ? 0 : 1;
            cs[c] = s;
        }
        if (c == 0) {
            bs->it = 0;
            bs->all_done = nrhs > 0 ? 0 : 1;
            bs->any_breakdown = 0;
        }
    }
}

// Caller layout n x nrhs (FP64) -> internal n x NC of type T, extra columns zero;
// optionally BD = dinv[row] * B (the first l1-Jacobi sweep from zero).
template <typename T>
__global__ void __launch_bounds__(BLOCK)
k_pack(int64_t n, int nrhs, int lg, const double* __restrict__ src, const T* __restrict__ dinv, T* __restrict__ B,
       T* __restrict__ BD) {
    const int NC = 1 << lg;
    for (int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x; t < (n << lg); t += (int64_t)gridDim.x * BLOCK) {
        const int c = (int)(t & (NC - 1));
        const int64_t row = t >> lg;
        const T v = c < nrhs ? (T)src[row * nrhs + c] : (T)0;
        B[t] = v;
        if (BD) BD[t] = dinv[row] * v;
    }
}

// Internal n x NC (type T) -> caller layout n x nrhs (FP64).
template <typename T>
__global__ void __launch_bounds__(BLOCK)
k_unpack(int64_t n, int nrhs, int lg, const T* __restrict__ src, double* __restrict__ dst) {
    for (int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x; t < n * nrhs; t += (int64_t)gridDim.x * BLOCK)
        dst[t] = (double)src[((t / nrhs) << lg) + t % nrhs];
}

template <typename T, class G>
__device__ __forceinline__ void fill(G g, int64_t n, T* __restrict__ x, const int* __restrict__ stop) {
    if (*stop) return;
    for (int64_t t = (int64_t)g.bid() * BLOCK + threadIdx.x; t < n; t += (int64_t)g.nb() * BLOCK) x[t] = (T)0;
}

template <typename T>
struct Fill {
    static constexpr int block = BLOCK;
    using sig = decltype(&fill<T, HwGrid>);
    template <class G, class... A>
    __device__ static void run(G g, A... a) { fill<T>(g, a...); }
};

template <typename T, class G>
__device__ __forceinline__ void copy(G g, int64_t n, const T* __restrict__ a, T* __restrict__ b,
                                     const int* __restrict__ stop) {
    if (*stop) return;
    for (int64_t t = (int64_t)g.bid() * BLOCK + threadIdx.x; t < n; t += (int64_t)g.nb() * BLOCK) b[t] = a[t];
}

template <typename T>
struct Copy {
    static constexpr int block = BLOCK;
    using sig = decltype(&copy<T, HwGrid>);
    template <class G, class... A>
    __device__ static void run(G g, A... a) { copy<T>(g, a...); }
};

}  // namespace dev
}  // namespace amge
