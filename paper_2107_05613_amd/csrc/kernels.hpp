// Device kernels of the solve phase (gfx950, wave64).
//
// All level operations are HBM-bandwidth bound sparse products; nothing here is a
// dense contraction, so no MFMA.  CSR rows are processed by LANES-wide lane groups
// inside a 64-wide wavefront (LANES a power of two chosen per matrix from its mean row
// length): consecutive lanes read consecutive nonzeros, so value/column loads are
// coalesced, and the row sum is finished with cross-lane shuffles inside the group.
// Signed incidence matrices (entries +-1) are stored index-only: bit 31 of a column
// word is the sign.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace amge {
namespace dev {

constexpr int BLOCK = 256;
constexpr int NRED = 1024;        // blocks (and partial sums) of the streaming reductions

enum CsrMode : int {
    SPMV = 0,      // y = A x
    SPMV_ADD = 1,  // y += A x
    RESID = 2,     // y = b - A x
    JAC = 3,       // y = x + dinv * (b - A x)
    JAC2Z = 4,     // y = dinv*b + dinv*(b - A (dinv*b))   (two sweeps from x = 0)
};

template <int LANES, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int off = LANES / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, LANES);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ---------------------------------------------------------------- CSR level operator
template <typename T, int LANES, int MODE>
__global__ void __launch_bounds__(BLOCK)
k_csr(int n, const int* __restrict__ rp, const int* __restrict__ ci, const T* __restrict__ av,
      const T* __restrict__ x, const T* __restrict__ b, const T* __restrict__ dinv, T* __restrict__ y) {
    const int64_t tid = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const int row = (int)(tid / LANES);
    const int lane = threadIdx.x & (LANES - 1);
    if (row >= n) return;          // whole lane groups leave together
    const int s = rp[row], e = rp[row + 1];
    T acc = 0;
    for (int k = s + lane; k < e; k += LANES) {
        const int j = ci[k];
        const T xv = (MODE == JAC2Z) ? b[j] * dinv[j] : x[j];
        acc = fma(av[k], xv, acc);
    }
    acc = group_sum<LANES>(acc);
    if (lane == 0) {
        if (MODE == SPMV) y[row] = acc;
        else if (MODE == SPMV_ADD) y[row] += acc;
        else if (MODE == RESID) y[row] = b[row] - acc;
        else if (MODE == JAC) y[row] = x[row] + dinv[row] * (b[row] - acc);
        else {
            const T x1 = dinv[row] * b[row];
            y[row] = x1 + dinv[row] * (b[row] - acc);
        }
    }
}

// ---------------------------------------------------------------- signed incidences
// y = D x (ADD = 0) or y += D x (ADD = 1); entries are +-1 encoded in the column word.
template <typename T, int LANES, int ADD>
__global__ void __launch_bounds__(BLOCK)
k_inc(int n, const int* __restrict__ rp, const uint32_t* __restrict__ ent, const T* __restrict__ x,
      T* __restrict__ y) {
    const int64_t tid = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const int row = (int)(tid / LANES);
    const int lane = threadIdx.x & (LANES - 1);
    if (row >= n) return;
    const int s = rp[row], e = rp[row + 1];
    T acc = 0;
    for (int k = s + lane; k < e; k += LANES) {
        const uint32_t w = ent[k];
        const T v = x[w & 0x7fffffffu];
        acc += (w >> 31) ? -v : v;
    }
    acc = group_sum<LANES>(acc);
    if (lane == 0) {
        if (ADD) y[row] += acc;
        else y[row] = acc;
    }
}

// y = dinv * x (one sweep from zero)
template <typename T>
__global__ void __launch_bounds__(BLOCK)
k_scale(int n, const T* __restrict__ dinv, const T* __restrict__ x, T* __restrict__ y) {
    const int i = blockIdx.x * BLOCK + threadIdx.x;
    if (i < n) y[i] = dinv[i] * x[i];
}

// ---------------------------------------------------------------- coarsest level
// x = W^T (W b) with W = L^{-1} the inverse Cholesky factor (lower triangular, row
// major) and WT its transpose; FP64 arithmetic whatever T is.  One workgroup.
template <typename T>
__global__ void __launch_bounds__(1024)
k_coarse(int n, const double* __restrict__ W, const double* __restrict__ WT, const T* __restrict__ b,
         T* __restrict__ x) {
    extern __shared__ double sm[];
    double* sb = sm;
    double* st = sm + n;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    for (int i = tid; i < n; i += blockDim.x) sb[i] = (double)b[i];
    __syncthreads();
    for (int i = wave; i < n; i += nw) {
        const double* w = W + (int64_t)i * n;
        double acc = 0;
        for (int j = lane; j <= i; j += 64) acc = fma(w[j], sb[j], acc);
        acc = wave_sum(acc);
        if (lane == 0) st[i] = acc;
    }
    __syncthreads();
    for (int i = wave; i < n; i += nw) {
        const double* w = WT + (int64_t)i * n;
        double acc = 0;
        for (int j = i + lane; j < n; j += 64) acc = fma(w[j], st[j], acc);
        acc = wave_sum(acc);
        if (lane == 0) x[i] = (T)acc;
    }
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

// q = A p and partial sums of p.q (grid-stride over lane groups).
template <int LANES>
__global__ void __launch_bounds__(BLOCK)
k_pcg_ap(int n, const int* __restrict__ rp, const int* __restrict__ ci, const double* __restrict__ av,
         const double* __restrict__ p, double* __restrict__ q, double* __restrict__ part,
         const int* __restrict__ done) {
    __shared__ double sh[BLOCK / 64 + 1];
    if (*done) return;
    const int lane = threadIdx.x & (LANES - 1);
    double mydot = 0;
    const int groups_per_grid = gridDim.x * (BLOCK / LANES);
    for (int row = blockIdx.x * (BLOCK / LANES) + threadIdx.x / LANES; row < n; row += groups_per_grid) {
        const int s = rp[row], e = rp[row + 1];
        double acc = 0;
        for (int k = s + lane; k < e; k += LANES) acc = fma(av[k], p[ci[k]], acc);
        acc = group_sum<LANES>(acc);
        if (lane == 0) {
            q[row] = acc;
            mydot = fma(p[row], acc, mydot);
        }
    }
    const double t = block_sum(mydot, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// alpha = delta / (p.q); x += alpha p; r -= alpha q; r32 = (float) r (if r32 != null).
__global__ void __launch_bounds__(BLOCK)
k_pcg_xr(int n, const double* __restrict__ part_pq, const double* __restrict__ part_delta,
         const double* __restrict__ p, const double* __restrict__ q, double* __restrict__ x,
         double* __restrict__ r, float* __restrict__ r32, int* __restrict__ done, int* __restrict__ flag) {
    __shared__ double sh[BLOCK / 64 + 1];
    if (*done) return;
    const double pq = sum_partials(part_pq, sh);
    const double delta = sum_partials(part_delta, sh);
    if (!(pq > 0) || !isfinite(pq)) {      // breakdown: recorded, iterate no further
        if (blockIdx.x == 0 && threadIdx.x == 0) *flag = 1;
        return;
    }
    const double alpha = delta / pq;
    for (int i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK) {
        x[i] = fma(alpha, p[i], x[i]);
        const double ri = fma(-alpha, q[i], r[i]);
        r[i] = ri;
        if (r32) r32[i] = (float)ri;
    }
}

// z = (double) z32 (if z32 != null); partials of r.z, r.zold, r.r.
__global__ void __launch_bounds__(BLOCK)
k_pcg_dots(int n, const float* __restrict__ z32, double* __restrict__ z, const double* __restrict__ zold,
           const double* __restrict__ r, double* __restrict__ part, const int* __restrict__ done) {
    __shared__ double sh[BLOCK / 64 + 1];
    if (*done) return;
    double a = 0, bsum = 0, c = 0;
    for (int i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK) {
        double zi;
        if (z32) { zi = (double)z32[i]; z[i] = zi; }
        else zi = z[i];
        const double ri = r[i];
        a = fma(ri, zi, a);
        if (zold) bsum = fma(ri, zold[i], bsum);
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
struct PcgStatus {
    double delta0, delta, rr, relres, bnorm;
    int iters, done, breakdown, pad;
};

// beta = (r.z - r.zold) / delta_old; p = z + beta p; stopping test.
__global__ void __launch_bounds__(BLOCK)
k_pcg_p(int n, const double* __restrict__ part_new, const double* __restrict__ part_old,
        const double* __restrict__ z, double* __restrict__ p, PcgStatus* __restrict__ st,
        int* __restrict__ done, const int* __restrict__ flag, double rtol, int stop_l2, int maxit, int it) {
    __shared__ double sh[BLOCK / 64 + 1];
    if (*done) return;
    const double dnew = sum_partials(part_new, sh);
    const double rzold = sum_partials(part_new + NRED, sh);
    const double rr = sum_partials(part_new + 2 * NRED, sh);
    const double dold = sum_partials(part_old, sh);
    const double rel = stop_l2 ? sqrt(rr) / st->bnorm : sqrt(fmax(dnew, 0.0) / st->delta0);
    const bool stop = (*flag != 0) || (rtol > 0 && rel <= rtol) || (it + 1 >= maxit) || !isfinite(dnew);
    if (!stop) {
        const double beta = (dnew - rzold) / dold;
        for (int i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK) p[i] = fma(beta, p[i], z[i]);
    }
    // every block has finished reading `done` at entry; only one block publishes
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->delta = dnew;
        st->rr = rr;
        st->relres = rel;
        st->iters = it + 1;
        st->breakdown = *flag;
    }
}

// Marks the iteration loop finished (separate launch, so no block of k_pcg_p can
// observe the flag change mid-kernel).
__global__ void k_pcg_finish(const PcgStatus* __restrict__ st, int* __restrict__ done, double rtol, int maxit) {
    if (*done) return;
    const bool stop = st->breakdown || (rtol > 0 && st->relres <= rtol) || (st->iters >= maxit) || !isfinite(st->delta);
    if (stop) *done = 1;
}

// Initial quantities: delta0 = r.z, bnorm = ||b||, from the dots partials.
__global__ void k_pcg_init(const double* __restrict__ part, PcgStatus* __restrict__ st) {
    __shared__ double sh[BLOCK / 64 + 1];
    const double d = sum_partials(part, sh);
    const double rr = sum_partials(part + 2 * NRED, sh);
    if (threadIdx.x == 0) {
        st->delta0 = d;
        st->delta = d;
        st->rr = rr;
        st->bnorm = sqrt(rr);
        st->relres = 1.0;
        st->iters = 0;
        st->breakdown = 0;
    }
}

}  // namespace dev
}  // namespace amge
