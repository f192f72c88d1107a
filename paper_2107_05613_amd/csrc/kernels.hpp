// Device kernels of the solve phase (gfx950, wave64).
//
// All level operations are HBM-bandwidth bound sparse products; nothing here is a
// dense contraction, so no MFMA.  Level matrices are stored in a sliced ELL layout
// matched to the 64-wide wavefront: rows are grouped in slices of 64 (one row per
// lane), stored column-major inside the slice so that every load instruction of a
// wave reads 64 consecutive entries; rows are sorted by length inside windows of 8
// slices to keep the padding small, and `srow` maps a slot back to its row.  Signed
// incidence matrices (entries +-1) are stored index-only: bit 31 of a column word is
// the sign.  Block indices are remapped so that each of the 8 XCDs (own L2) works on
// a contiguous range of slices, which keeps the gathered vector entries of one range
// in one L2.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "kernels_base.hpp"
#include "state.hpp"

namespace amge {
namespace dev {

enum Mode : int {
    SPMV = 0,      // y = A x
    SPMV_ADD = 1,  // y += A x
    RESID = 2,     // y = b - A x
    JAC = 3,       // y = x + dinv * (b - A x)
    JAC0 = 4,      // batched only: JAC from x = dinv * b, formed where x is read
    SPLIT = 5,     // y = A [b; x]: the first lead entries of a row read b, the others x
};

// Sliced ELL with K lanes per row (K | 64): a slice holds R = 64/K rows; entry t of
// the slice's row rr is stored at base + (t / K) * 64 + rr * K + t % K, so every load
// instruction of the wave reads 64 consecutive entries for every K.  Lane l works on
// entries t = l % K (mod K) of row l / K; the K partial sums are combined with
// cross-lane shuffles.  Small K suits many short rows, large K few long rows.
template <int K, typename T>
__device__ __forceinline__ T row_sum(T v) {
#pragma unroll
    for (int off = K / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, K);
    return v;
}

// Column index of stored entry e of a slice: 32-bit indices, or (C16) a 16-bit offset
// from the slice's base column.
// Matrix value streams: FP64 values are read with non-temporal loads (they cannot stay
// cache-resident and would evict what can); FP32 values of A_k and the column indices of
// A_k are read with plain loads so that they stay in the last-level cache between the
// uses of A_k (measured on the 64^3 H(curl) workload: FP32 sweep 52 -> 43 us, FP64
// sweep 95 -> 84 us together with the non-temporal loads of the other operators).
template <bool C16, bool NT>
__device__ __forceinline__ int col_at(const int* __restrict__ ci, const uint16_t* __restrict__ c16, int cb, int e) {
    if (C16) return cb + (int)(NT ? __builtin_nontemporal_load(c16 + e) : c16[e]);
    return NT ? __builtin_nontemporal_load(ci + e) : ci[e];
}

template <typename T, bool NT = (sizeof(T) == 8)>
__device__ __forceinline__ T stream_load(const T* __restrict__ p) {
    if (NT) return __builtin_nontemporal_load(p);
    return *p;
}

// NT: non-temporal loads of the matrix streams (FP64 always; FP32 for the operators
// other than A_k, so that A_k, used four times per V-cycle, stays in the last-level
// cache between its uses: the fine-level FP32 sweep of the 64^3 H(curl) workload takes
// 45 instead of 50 us).  UNR: entries per lane whose loads are issued together (8 for
// the long rows of a large fine level, 4 otherwise).  TV: the matrix value type, T by
// default; FP64 values with FP32 vectors (the fine-level residual of an FP32 V-cycle on
// high-contrast problems) sum in FP64 and round the result to T once.
template <typename T, int K, int MODE, bool C16, bool NT, int UNR = 4, typename TV = T>
__global__ void __launch_bounds__(BLOCK)
k_sell(int nslices, const int* __restrict__ sptr, const int* __restrict__ srow, const int* __restrict__ ci,
       const uint16_t* __restrict__ c16, const int* __restrict__ cbase, const TV* __restrict__ av,
       const T* __restrict__ x, const T* __restrict__ b, const T* __restrict__ dinv, T* __restrict__ y,
       T* __restrict__ yd, const uint16_t* __restrict__ lead, const int* __restrict__ stop) {
    using TA = typename std::conditional<(sizeof(TV) > sizeof(T)), TV, T>::type;   // accumulation
    // SPMV / SPLIT with yd != null also write yd = dinv * y: the first l1-Jacobi sweep
    // from zero on the next operator, produced where its right-hand side is produced.
    // Every launch of the PCG iteration returns without writing when *stop is set
    // (converged).
    const int slice = xcd_block(blockIdx.x, gridDim.x) * WAVES + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    // The stop flag and the slice's layout words are requested together (the slice index
    // is clamped so every address is valid; nslices >= 1 for every launch): on the small
    // coarse levels a launch is one chain of dependent loads, and each link costs a
    // memory latency.
    const int sl = min(slice, nslices - 1);
    const int stopped = *stop;
    const int base = sptr[sl];
    const int end = sptr[sl + 1];
    const int row = srow[sl * (64 / K) + lane / K];
    const int cb = C16 ? cbase[sl] : 0;
    const int nlead = MODE == SPLIT ? lead[sl * (64 / K) + lane / K] : 0;
    // (end < base, row < -1 and cb < 0 never hold: they keep the loads ahead of the branch)
    if (stopped | (slice >= nslices) | (end < base) | (row < -1) | (cb < 0)) return;
    const int width = (end - base) >> 6;
    const int e0 = base + lane;
    const TV* v = av + e0;
    // the row's own operands of the update are requested before the product, so their
    // latency overlaps it
    const bool owner = row >= 0 && !(lane & (K - 1));
    const int rw = owner ? row : 0;
    T xr = 0, br = 0, dr = 0;
    if (MODE == JAC) {
        xr = x[rw];
        br = b[rw];
        dr = dinv[rw];
    } else if (MODE == RESID) {
        br = b[rw];
    } else if (MODE == SPMV_ADD) {
        xr = y[rw];
    } else if (yd) {
        dr = dinv[rw];
    }
    TA acc = 0;
#pragma unroll UNR
    for (int k = 0; k < width; ++k) {
        const int j = col_at<C16, NT>(ci, c16, cb, e0 + k * 64);
        T xv;
        if (MODE == SPLIT) xv = (k * K + (lane & (K - 1)) < nlead ? b : x)[j];   // entry k*K + lane%K
        else xv = x[j];
        acc = fma((TA)stream_load<TV, NT || sizeof(TV) == 8>(v + k * 64), (TA)xv, acc);
    }
    acc = row_sum<K>(acc);
    if (!owner) return;
    if (MODE == SPMV || MODE == SPLIT) {
        y[row] = (T)acc;
        if (yd) yd[row] = dr * (T)acc;
    } else if (MODE == SPMV_ADD) y[row] = xr + (T)acc;
    else if (MODE == RESID) y[row] = (T)((TA)br - acc);
    else y[row] = xr + dr * (T)((TA)br - acc);
}

// One colour of a multicolour Gauss-Seidel sweep, in place: for the rows of the colour
// (the sliced ELL holds only them; srow maps slots to global rows)
//   x_i += dg_i (b_i - (A x)_i),  dg_i = 1 / a_ii.
// No row of a colour is coupled to another row of the same colour, so every x_j a lane
// gathers belongs to another colour and is not written by this launch: x is read and
// written through one unrestricted pointer, without a race.
template <typename T, int K, bool C16, bool NT, int UNR = 4>
__global__ void __launch_bounds__(BLOCK)
k_sell_gs(int nslices, const int* __restrict__ sptr, const int* __restrict__ srow, const int* __restrict__ ci,
          const uint16_t* __restrict__ c16, const int* __restrict__ cbase, const T* __restrict__ av,
          const T* __restrict__ b, const T* __restrict__ dg, T* x, const int* __restrict__ stop) {
    const int slice = xcd_block(blockIdx.x, gridDim.x) * WAVES + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int sl = min(slice, nslices - 1);
    const int stopped = *stop;
    const int base = sptr[sl];
    const int end = sptr[sl + 1];
    const int row = srow[sl * (64 / K) + lane / K];
    const int cb = C16 ? cbase[sl] : 0;
    if (stopped | (slice >= nslices) | (end < base) | (row < -1) | (cb < 0)) return;
    const int width = (end - base) >> 6;
    const int e0 = base + lane;
    const T* v = av + e0;
    const bool owner = row >= 0 && !(lane & (K - 1));
    const int rw = owner ? row : 0;
    const T br = b[rw], dr = dg[rw];
    T acc = 0;
#pragma unroll UNR
    for (int k = 0; k < width; ++k) {
        const int j = col_at<C16, NT>(ci, c16, cb, e0 + k * 64);
        acc = fma(stream_load<T, NT || sizeof(T) == 8>(v + k * 64), x[j], acc);
    }
    acc = row_sum<K>(acc);
    if (!owner) return;
    x[row] = x[row] + dr * (br - acc);
}

// Signed incidence, index-only (same layout): y = D x (ADD = 0) or y += D x (ADD = 1).
template <typename T, int K, int ADD>
__global__ void __launch_bounds__(BLOCK)
k_sell_inc(int nslices, const int* __restrict__ sptr, const int* __restrict__ srow, const uint32_t* __restrict__ ent,
           const T* __restrict__ x, T* __restrict__ y, const int* __restrict__ stop) {
    const int slice = xcd_block(blockIdx.x, gridDim.x) * WAVES + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    // flag and layout words requested together, as in k_sell
    const int sl = min(slice, nslices - 1);
    const int stopped = *stop;
    const int base = sptr[sl];
    const int end = sptr[sl + 1];
    const int row = srow[sl * (64 / K) + lane / K];
    if (stopped | (slice >= nslices) | (end < base) | (row < -1)) return;
    const int width = (end - base) >> 6;
    const bool owner = row >= 0 && !(lane & (K - 1));
    const T yr = ADD ? y[owner ? row : 0] : T(0);   // requested before the product
    const uint32_t* e = ent + base + lane;
    T acc = 0;
#pragma unroll 4
    for (int k = 0; k < width; ++k) {
        const uint32_t w = e[k * 64];
        if (w == 0xffffffffu) continue;    // padding
        const T v = x[w & 0x7fffffffu];
        acc += (w >> 31) ? -v : v;
    }
    acc = row_sum<K>(acc);
    if (!owner) return;
    y[row] = ADD ? yr + acc : acc;
}

// Signed incidence with the same number W of entries in every row (the fine-level
// derivatives: an edge has two vertices, a triangle three edges), stored row-major as
// n x W words (column | sign << 31), no padding and no slice layout: y = D x (ADD = 0)
// or y += D x (ADD = 1), summed in entry order like k_sell_inc.  Thread t takes rows t,
// t + S, ... (S = grid size), INC_ROWS of them per step with all their loads issued
// before any is used, so a wave keeps several rows' loads in flight.  The words are read
// with non-temporal loads, like every fine-level operator but A_k.
constexpr int INC_ROWS = 4;

template <typename T, int W>
__device__ __forceinline__ T inc_row(const uint32_t (&e)[W], const T (&v)[W]) {
    T acc = 0;
#pragma unroll
    for (int k = 0; k < W; ++k) acc += (e[k] >> 31) ? -v[k] : v[k];
    return acc;
}

template <typename T, int W, int ADD>
__global__ void __launch_bounds__(BLOCK)
k_inc_fixed(int n, const uint32_t* __restrict__ ent, const T* __restrict__ x, T* __restrict__ y,
            const int* __restrict__ stop) {
    constexpr int R = INC_ROWS;
    if (*stop) return;
    const int64_t S = (int64_t)gridDim.x * BLOCK;
    int64_t r0 = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    for (; r0 + (R - 1) * S < n; r0 += R * S) {
        uint32_t e[R][W];
        T yr[R];
#pragma unroll
        for (int u = 0; u < R; ++u) {
#pragma unroll
            for (int k = 0; k < W; ++k) e[u][k] = __builtin_nontemporal_load(ent + (r0 + u * S) * W + k);
            yr[u] = ADD ? y[r0 + u * S] : T(0);
        }
        T v[R][W];
#pragma unroll
        for (int u = 0; u < R; ++u)
#pragma unroll
            for (int k = 0; k < W; ++k) v[u][k] = x[e[u][k] & 0x7fffffffu];
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const T acc = inc_row<T, W>(e[u], v[u]);
            y[r0 + u * S] = ADD ? yr[u] + acc : acc;
        }
    }
    for (; r0 < n; r0 += S) {
        uint32_t e[W];
        T v[W];
#pragma unroll
        for (int k = 0; k < W; ++k) e[k] = __builtin_nontemporal_load(ent + r0 * W + k);
#pragma unroll
        for (int k = 0; k < W; ++k) v[k] = x[e[k] & 0x7fffffffu];
        const T acc = inc_row<T, W>(e, v);
        y[r0] = ADD ? y[r0] + acc : acc;
    }
}

// y = dinv * x (one sweep from zero)
template <typename T>
__global__ void __launch_bounds__(BLOCK)
k_scale(int n, const T* __restrict__ dinv, const T* __restrict__ x, T* __restrict__ y) {
    const int i = blockIdx.x * BLOCK + threadIdx.x;
    if (i < n) y[i] = dinv[i] * x[i];
}

// ---------------------------------------------------------------- dense operators
// x = M b for a dense row-major FP64 n x n operator: the coarsest inverse Ainv = W^T W,
// W = L^{-1} from the FP64 Cholesky factor A = L L^T formed at set-up, or the folded
// coarse tail of the V-cycle.  FP64 arithmetic whatever T is.  One wave per row; lane l
// sums j = l, l + 64, ... in order, eight terms' loads issued at a time.  The operator is
// read with non-temporal loads (a folded tail is tens of MB, read once per V-cycle).
template <typename T>
__global__ void __launch_bounds__(BLOCK)
k_coarse(int n, const double* __restrict__ Ainv, const T* __restrict__ b, T* __restrict__ x,
         const int* __restrict__ stop) {
    const int stopped = *stop;
    const int row = blockIdx.x * WAVES + (threadIdx.x >> 6);
    if (row >= n) return;
    const int lane = threadIdx.x & 63;
    const double* a = Ainv + (int64_t)row * n;
    double acc = 0;
    int j = lane;
    for (; j + 7 * 64 < n; j += 8 * 64) {
        double av[8], bv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            av[u] = __builtin_nontemporal_load(a + j + u * 64);
            bv[u] = (double)b[j + u * 64];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = fma(av[u], bv[u], acc);
    }
    for (; j < n; j += 64) acc = fma(__builtin_nontemporal_load(a + j), (double)b[j], acc);
    acc = wave_sum(acc);
    // the stop flag is tested only before the store: its load overlaps the product
    // (a stopped launch reads the small inverse once and writes nothing)
    if (lane == 0 && !stopped) x[row] = (T)acc;
}

// ---------------------------------------------------------------- conversions
template <typename S, typename D>
__global__ void __launch_bounds__(BLOCK) k_convert(int64_t n, const S* __restrict__ a, D* __restrict__ b) {
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * BLOCK)
        b[i] = (D)a[i];
}

// ---------------------------------------------------------------- PCG (FP64 outer loop)
// Deterministic reductions: every producer writes NRED block partials; every consumer
// block re-reduces the same NRED values in the same order.
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double t = 0;
    if (threadIdx.x == 0) {
        for (int w = 0; w < BLOCK / 64; ++w) t += sh[w];
        sh[BLOCK / 64] = t;
    }
    __syncthreads();
    t = sh[BLOCK / 64];
    __syncthreads();
    return t;
}

__device__ __forceinline__ double sum_partials(const double* __restrict__ part, double* sh) {
    double v = 0;
    for (int i = threadIdx.x; i < NRED; i += BLOCK) v += part[i];
    return block_sum(v, sh);
}

// N sums of NRED partials each, in the order of sum_partials (so with the same
// results), with every load issued before the first reduction and one exchange through
// LDS for all N (sh: N * (WAVES + 1) doubles).
template <int N>
__device__ __forceinline__ void sum_partials_n(const double* const (&part)[N], double* sh, double (&out)[N]) {
    static_assert(NRED % BLOCK == 0, "partials per thread");
    double v[N];
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] = 0;
#pragma unroll
    for (int i = 0; i < NRED / BLOCK; ++i)
#pragma unroll
        for (int q = 0; q < N; ++q) v[q] += part[q][threadIdx.x + i * BLOCK];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < N; ++q) {
        v[q] = wave_sum(v[q]);
        if (lane == 0) sh[q * WAVES + wave] = v[q];
    }
    __syncthreads();
    if ((int)threadIdx.x < N) {
        double t = 0;
        for (int w = 0; w < WAVES; ++w) t += sh[threadIdx.x * WAVES + w];
        sh[N * WAVES + threadIdx.x] = t;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < N; ++q) out[q] = sh[N * WAVES + q];
    __syncthreads();
}

// q = A p (FP64 sliced ELL) and partial sums of p.q.  NRED blocks, each over a
// contiguous range of slices; UNR as in k_sell.
template <int K, bool C16, int UNR = 4>
__global__ void __launch_bounds__(BLOCK)
k_pcg_ap(int nslices, const int* __restrict__ sptr, const int* __restrict__ srow, const int* __restrict__ ci,
         const uint16_t* __restrict__ c16, const int* __restrict__ cbase, const double* __restrict__ av,
         const double* __restrict__ p, double* __restrict__ q, double* __restrict__ part,
         const int* __restrict__ done) {
    __shared__ double sh[WAVES + 1];
    if (*done) return;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int chunk = (nslices + gridDim.x - 1) / gridDim.x;
    const int s0 = blk * chunk, s1 = min(nslices, s0 + chunk);
    const int lane = threadIdx.x & 63;
    double mydot = 0;
    for (int slice = s0 + (threadIdx.x >> 6); slice < s1; slice += WAVES) {
        const int base = sptr[slice];
        const int width = (sptr[slice + 1] - base) >> 6;
        const int row = srow[slice * (64 / K) + lane / K];
        const int cb = C16 ? cbase[slice] : 0;
        const int e0 = base + lane;
        const double* v = av + e0;
        double acc = 0;
#pragma unroll UNR
        for (int k = 0; k < width; ++k)
            acc = fma(stream_load(v + k * 64), p[col_at<C16, false>(ci, c16, cb, e0 + k * 64)], acc);
        acc = row_sum<K>(acc);
        if (row >= 0 && !(lane & (K - 1))) {
            q[row] = acc;
            mydot = fma(p[row], acc, mydot);
        }
    }
    const double t = block_sum(mydot, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// alpha = delta / (p.q); x += alpha p; r -= alpha q.  Also the level-1 inputs of the
// V-cycle: r32 = (float) r and rd32 = dinv32 * r32 (FP32 preconditioner) or
// rd64 = dinv64 * r (FP64 preconditioner), whichever pointers are non-null.
__global__ void __launch_bounds__(BLOCK)
k_pcg_xr(int n, const double* __restrict__ part_pq, const double* __restrict__ part_delta,
         const double* __restrict__ p, const double* __restrict__ q, double* __restrict__ x,
         double* __restrict__ r, float* __restrict__ r32, float* __restrict__ rd32,
         const float* __restrict__ dinv32, double* __restrict__ rd64, const double* __restrict__ dinv64,
         int* __restrict__ done, int* __restrict__ flag) {
    __shared__ double sh[2 * (WAVES + 1)];
    const int stopped = *done;   // tested after the reductions, whose loads it overlaps
    double sums[2];
    sum_partials_n<2>({part_pq, part_delta}, sh, sums);
    const double pq = sums[0], delta = sums[1];
    if (stopped) return;
    if (!(pq > 0) || !isfinite(pq)) {      // breakdown: recorded, iterate no further
        if (blockIdx.x == 0 && threadIdx.x == 0) *flag = 1;
        return;
    }
    const double alpha = delta / pq;
    for (int i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK) {
        // x is used by this kernel only: streamed past the caches (non-temporal load and store)
        __builtin_nontemporal_store(fma(alpha, p[i], __builtin_nontemporal_load(x + i)), x + i);
        const double ri = fma(-alpha, q[i], r[i]);
        r[i] = ri;
        if (r32) {
            const float rf = (float)ri;
            r32[i] = rf;
            rd32[i] = dinv32[i] * rf;
        }
        if (rd64) rd64[i] = dinv64[i] * ri;
    }
}

// Partials of r.z, r.zold, r.r.  z and zold are in the preconditioner's precision TZ
// (an FP32 V-cycle output is used as it is: widening it to FP64 is exact).
template <typename TZ>
__global__ void __launch_bounds__(BLOCK)
k_pcg_dots(int n, const TZ* __restrict__ z, const TZ* __restrict__ zold, const double* __restrict__ r,
           double* __restrict__ part, const int* __restrict__ done) {
    __shared__ double sh[WAVES + 1];
    if (*done) return;
    double a = 0, bsum = 0, c = 0;
    for (int i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK) {
        const double zi = (double)z[i];
        const double ri = r[i];
        a = fma(ri, zi, a);
        if (zold) bsum = fma(ri, (double)zold[i], bsum);
        c = fma(ri, ri, c);
    }
    a = block_sum(a, sh);
    bsum = block_sum(bsum, sh);
    c = block_sum(c, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = a;
        part[NRED + blockIdx.x] = bsum;
        part[2 * NRED + blockIdx.x] = c;
    }
}

// Status written by the last kernel of every iteration (read by the host).

// beta = (r.z - r.zold) / delta_old; p = z + beta p; stopping test, then (one thread)
// the iteration's status, the stop flag and the host record.
// Every block takes the same decision from the same partial sums.  The blocks read only
// fields of st that are fixed during a solve, and the iteration count from it_in, while
// the count is written to it_out (the two alternate with the buffer parity): so no
// block sees a value written by this launch.  The stop flag may be set while late
// blocks start; they then return early, which changes nothing, since p is left as it
// is when the loop stops.  The host record is written first and its tag after a
// system-scope fence, so a host that sees the tag of iteration k reads its status.
template <typename TZ>
__global__ void __launch_bounds__(BLOCK)
k_pcg_p(int n, const double* __restrict__ part_new, const double* __restrict__ part_old,
        const TZ* __restrict__ z, double* __restrict__ p, PcgStatus* __restrict__ st,
        int* __restrict__ done, const int* __restrict__ flag, const int* __restrict__ it_in,
        int* __restrict__ it_out, PcgRecord* __restrict__ ring) {
    __shared__ double sh[4 * (WAVES + 1)];
    const int stopped = *done;   // tested after the reductions, whose loads it overlaps
    const int it = *it_in, maxit = st->maxit, stop_l2 = st->stop_l2;
    const double rtol = st->rtol;
    double sums[4];
    sum_partials_n<4>({part_new, part_new + NRED, part_new + 2 * NRED, part_old}, sh, sums);
    const double dnew = sums[0], rzold = sums[1], rr = sums[2], dold = sums[3];
    if (stopped) return;
    const double rel = stop_l2 ? sqrt(rr) / st->bnorm : sqrt(fmax(dnew, 0.0) / st->delta0);
    const bool stop = (*flag != 0) || (rtol > 0 && rel <= rtol) || (it + 1 >= maxit) || !isfinite(dnew);
    if (!stop) {
        const double beta = (dnew - rzold) / dold;
        for (int i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK)
            p[i] = fma(beta, p[i], (double)z[i]);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->delta = dnew;
        st->rr = rr;
        st->relres = rel;
        st->breakdown = *flag;
        st->iters = it + 1;
        *it_out = it + 1;
        if (stop) {
            *done = 1;
            st->done = 1;
        }
        PcgRecord* rec = ring + (it + 1) % PCG_RING;
        rec->st = *st;
        __threadfence_system();
        rec->tag = ((uint64_t)st->epoch << 32) | (uint32_t)(it + 1);
    }
}

// Initial quantities: delta0 = r.z, bnorm = ||b||, from the dots partials; stopping
// parameters of the solve.
__global__ void k_pcg_init(const double* __restrict__ part, PcgStatus* __restrict__ st, double rtol, int maxit,
                           int stop_l2, uint32_t epoch) {
    __shared__ double sh[WAVES + 1];
    const double d = sum_partials(part, sh);
    const double rr = sum_partials(part + 2 * NRED, sh);
    if (threadIdx.x == 0) {
        st->delta0 = d;
        st->delta = d;
        st->rr = rr;
        st->bnorm = sqrt(rr);
        st->relres = 1.0;
        st->iters = 0;
        st->done = 0;
        st->breakdown = 0;
        st->rtol = rtol;
        st->maxit = maxit;
        st->stop_l2 = stop_l2;
        st->epoch = epoch;
    }
}

// ---- set-up: entry arrays of the sliced ELL from a device copy of the CSR matrix.
// One wave per slice; the row part of the layout (slot -> row map srow, slice offsets
// sptr) comes from the host.  Lane l of a slice serves entries t = l % K (mod K) of the
// row in slot l / K, so for every chunk c of 64 consecutive slots the wave writes
// slots sptr + 64 c .. sptr + 64 c + 63 at once.

// Column range of every slice: cbase = smallest column (0 for an empty slice); *wide
// set if some slice spans more than 65536 consecutive columns.
__global__ void __launch_bounds__(BLOCK)
k_slice_range(int ns, int K, const int* __restrict__ srow, const int* __restrict__ rowptr,
              const int* __restrict__ col, int* __restrict__ cbase, int* __restrict__ wide) {
    const int w = blockIdx.x * WAVES + threadIdx.x / 64, lane = threadIdx.x % 64;
    if (w >= ns) return;
    const int R = 64 / K;
    const int r = srow[(int64_t)w * R + lane / K];
    int lo = 0x7fffffff, hi = -1;
    if (r >= 0)
        for (int t = rowptr[r] + lane % K; t < rowptr[r + 1]; t += K) {
            lo = min(lo, col[t]);
            hi = max(hi, col[t]);
        }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        lo = min(lo, __shfl_xor(lo, off, 64));
        hi = max(hi, __shfl_xor(hi, off, 64));
    }
    if (lane == 0) {
        cbase[w] = hi < 0 ? 0 : lo;
        if (hi >= 0 && hi - lo > 65535) atomicOr(wide, 1);
    }
}

// Entry arrays: value matrices write the columns (ci, or c16 offsets from cbase) and the
// values (v64 and/or v32, rounded to nearest); incidence matrices write column | sign
// << 31 to ent and set *bad on an entry other than +-1.  Padding: column 0, value 0,
// incidence word 0xffffffff.
template <bool INC>
__global__ void __launch_bounds__(BLOCK)
k_sell_fill(int ns, int K, const int* __restrict__ sptr, const int* __restrict__ srow, const int* __restrict__ rowptr,
            const int* __restrict__ col, const double* __restrict__ val, const int* __restrict__ cbase,
            int* __restrict__ ci, uint16_t* __restrict__ c16, double* __restrict__ v64, float* __restrict__ v32,
            uint32_t* __restrict__ ent, int* __restrict__ bad) {
    const int w = blockIdx.x * WAVES + threadIdx.x / 64, lane = threadIdx.x % 64;
    if (w >= ns) return;
    const int R = 64 / K, j = lane % K;
    const int r = srow[(int64_t)w * R + lane / K];
    const int b0 = r >= 0 ? rowptr[r] : 0;
    const int len = r >= 0 ? rowptr[r + 1] - b0 : 0;
    const int64_t base = sptr[w];
    const int width = (sptr[w + 1] - sptr[w]) / 64;
    const int cb = c16 ? cbase[w] : 0;
    for (int c = 0; c < width; ++c) {
        const int t = c * K + j;
        const int64_t idx = base + (int64_t)c * 64 + lane;
        const bool in = t < len;
        const int cc = in ? col[b0 + t] : 0;
        const double v = in ? val[b0 + t] : 0.0;
        if (INC) {
            if (in && v != 1.0 && v != -1.0) *bad = 1;
            ent[idx] = in ? ((uint32_t)cc | (v < 0 ? 0x80000000u : 0u)) : 0xffffffffu;
        } else {
            if (c16) c16[idx] = (uint16_t)(in ? cc - cb : 0);
            else ci[idx] = cc;
            if (v64) v64[idx] = v;
            if (v32) v32[idx] = (float)v;
        }
    }
}

}  // namespace dev
}  // namespace amge
