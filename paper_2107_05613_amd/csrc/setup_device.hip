// Device side of the set-up phase: the weighted local extension problems of the first
// agglomeration step (eqs. (3.6), (3.8) with the coefficient-weighted masses of the
// remark closing section 3.3), one workgroup of 64 lanes per agglomerate.
//
// Every agglomerate shares the block topology, constraints, PV traces, face extensions
// and the null spaces of its constraints (the host's KuhnPlan); its RT and ND masses are
// sums of eight per-hex unit masses times the hex weights.  Per agglomerate:
//   RT:  Hw = sum_s w_s H_s, hw = sum_s w_s h_s, Cw = sum_s w_s C_s,
//        y = -Hw^{-1} hw, u = u_p + Q2 y, next element Cw + hw^T y;
//   ND:  G = u C^H - G0, u_n = Wn G, Mw = sum_s v_s Mn_s, Fw, Cnw likewise,
//        y_n = -(Q2n^T Mw Q2n)^{-1} Q2n^T (Mw u_n + Fw), u_n += Q2n y_n,
//        next element u_n^T Mw u_n + u_n^T Fw + Fw^T u_n + Cnw.
// All of it is small dense algebra in LDS; every sum runs in a fixed order, so results
// do not depend on the launch.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "common.hpp"
#include "setup_device.hpp"

namespace amge {
namespace {

constexpr int LANES = 64;
constexpr int MAXI = 80;    // RT interior faces of a block
constexpr int MAXZ = 32;    // RT null-space dimension
constexpr int MAXIN = 32;   // ND interior edges
constexpr int MAXZN = 32;   // ND null-space dimension
static_assert(MAXIN * MAXZN <= MAXZ * MAXZ, "the ND product Mw Q2n reuses the RT matrix's LDS");

// Cholesky factor (lower, in place, leading dimension ld) of an n x n SPD matrix in
// LDS, then the solution of A X = B for nrhs columns of B (in place).  Returns false
// (to every lane) if a pivot is not positive.
__device__ bool lds_chol_solve(double* A, int n, int ld, double* B, int nrhs, int ldb, int* ok) {
    const int lane = threadIdx.x;
    if (lane == 0) *ok = 1;
    __syncthreads();
    for (int j = 0; j < n; ++j) {
        if (lane == 0) {
            double d = A[j * ld + j];
            for (int k = 0; k < j; ++k) d -= A[j * ld + k] * A[j * ld + k];
            if (!(d > 0)) *ok = 0;
            A[j * ld + j] = d > 0 ? sqrt(d) : 1.0;
        }
        __syncthreads();
        for (int i = j + 1 + lane; i < n; i += LANES) {
            double v = A[i * ld + j];
            for (int k = 0; k < j; ++k) v -= A[i * ld + k] * A[j * ld + k];
            A[i * ld + j] = v / A[j * ld + j];
        }
        __syncthreads();
    }
    // L Y = B, then L^T X = Y; lanes own right-hand sides
    for (int i = 0; i < n; ++i) {
        for (int t = lane; t < nrhs; t += LANES) {
            double v = B[i * ldb + t];
            for (int k = 0; k < i; ++k) v -= A[i * ld + k] * B[k * ldb + t];
            B[i * ldb + t] = v / A[i * ld + i];
        }
        __syncthreads();
    }
    for (int i = n - 1; i >= 0; --i) {
        for (int t = lane; t < nrhs; t += LANES) {
            double v = B[i * ldb + t];
            for (int k = i + 1; k < n; ++k) v -= A[k * ld + i] * B[k * ldb + t];
            B[i * ldb + t] = v / A[i * ld + i];
        }
        __syncthreads();
    }
    return *ok != 0;
}

__global__ void __launch_bounds__(LANES)
k_kuhn_local(KuhnPlanView p, const double* __restrict__ w, double* __restrict__ U, double* __restrict__ elrt,
             double* __restrict__ Un, double* __restrict__ elnd, int* __restrict__ bad) {
    __shared__ double wl[16];
    __shared__ double Hw[MAXZ * MAXZ], hw[MAXZ * 6], y[MAXZ * 6], u[MAXI * 6];
    __shared__ double G[MAXI * 12], un[MAXIN * 12], Mw[MAXIN * MAXIN], Fw[MAXIN * 12], R[MAXIN * 12];
    __shared__ double Hn[MAXZN * MAXZN], yn[MAXZN * 12], Cnw[144];
    __shared__ int ok;
    const int64_t a = blockIdx.x;
    const int lane = threadIdx.x;
    const int nI = p.nI, nz = p.nz;
    if (lane < 16) wl[lane] = w[a * 16 + lane];
    __syncthreads();
    const double* wnd = wl;
    const double* wrt = wl + 8;
    // ---- RT: weighted sums of the per-slot reduced matrices
    for (int e = lane; e < nz * nz; e += LANES) {
        double v = 0;
        for (int s = 0; s < 8; ++s) v += wrt[s] * p.H[s * nz * nz + e];
        Hw[e] = v;
    }
    for (int e = lane; e < nz * 6; e += LANES) {
        double v = 0;
        for (int s = 0; s < 8; ++s) v += wrt[s] * p.h[s * nz * 6 + e];
        hw[e] = v;
        y[e] = -v;
    }
    __syncthreads();
    if (nz > 0 && !lds_chol_solve(Hw, nz, nz, y, 6, 6, &ok)) {
        if (lane == 0) bad[a] = 1;
        return;
    }
    // u = u_p + Q2 y
    for (int e = lane; e < nI * 6; e += LANES) {
        const int i = e / 6, t = e % 6;
        double v = p.up[e];
        for (int k = 0; k < nz; ++k) v += p.Q2[i * nz + k] * y[k * 6 + t];
        u[e] = v;
        U[a * nI * 6 + e] = v;
    }
    // next-level RT element: Cw + hw^T y
    for (int e = lane; e < 36; e += LANES) {
        const int i = e / 6, j = e % 6;
        double v = 0;
        for (int s = 0; s < 8; ++s) v += wrt[s] * p.C[s * 36 + e];
        for (int k = 0; k < nz; ++k) v += hw[k * 6 + i] * y[k * 6 + j];
        elrt[a * 36 + e] = v;
    }
    if (!p.nd) return;
    __syncthreads();
    // ---- ND: G = u C^H - G0, u_n = Wn G
    const int nIn = p.nIn, nzn = p.nzn;
    for (int e = lane; e < nI * 12; e += LANES) {
        const int i = e / 12, E = e % 12;
        double v = -p.G0[e];
        for (int F = 0; F < 6; ++F) v += u[i * 6 + F] * p.CH[F * 12 + E];
        G[e] = v;
    }
    for (int e = lane; e < nIn * nIn; e += LANES) {
        double v = 0;
        for (int s = 0; s < 8; ++s) v += wnd[s] * p.Mn[s * nIn * nIn + e];
        Mw[e] = v;
    }
    for (int e = lane; e < nIn * 12; e += LANES) {
        double v = 0;
        for (int s = 0; s < 8; ++s) v += wnd[s] * p.Fn[s * nIn * 12 + e];
        Fw[e] = v;
    }
    for (int e = lane; e < 144; e += LANES) {
        double v = 0;
        for (int s = 0; s < 8; ++s) v += wnd[s] * p.Cn[s * 144 + e];
        Cnw[e] = v;
    }
    __syncthreads();
    for (int e = lane; e < nIn * 12; e += LANES) {
        const int i = e / 12, E = e % 12;
        double v = 0;
        for (int k = 0; k < nI; ++k) v += p.Wn[i * nI + k] * G[k * 12 + E];
        un[e] = v;
    }
    __syncthreads();
    if (nzn > 0) {
        // R = Mw u_n + Fw; Hn = Q2n^T Mw Q2n; y_n = -Q2n^T R
        for (int e = lane; e < nIn * 12; e += LANES) {
            const int i = e / 12, E = e % 12;
            double v = Fw[e];
            for (int k = 0; k < nIn; ++k) v += Mw[i * nIn + k] * un[k * 12 + E];
            R[e] = v;
        }
        // Mw Q2n into Hw (free after the RT problem), then Hn = Q2n^T (Mw Q2n)
        double* MQ = Hw;
        for (int e = lane; e < nIn * nzn; e += LANES) {
            const int k = e / nzn, j = e % nzn;
            double v = 0;
            for (int l = 0; l < nIn; ++l) v += Mw[k * nIn + l] * p.Q2n[l * nzn + j];
            MQ[e] = v;
        }
        __syncthreads();
        for (int e = lane; e < nzn * nzn; e += LANES) {
            const int i = e / nzn, j = e % nzn;
            double v = 0;
            for (int k = 0; k < nIn; ++k) v += p.Q2n[k * nzn + i] * MQ[k * nzn + j];
            Hn[e] = v;
        }
        __syncthreads();
        for (int e = lane; e < nzn * 12; e += LANES) {
            const int i = e / 12, E = e % 12;
            double v = 0;
            for (int k = 0; k < nIn; ++k) v += p.Q2n[k * nzn + i] * R[k * 12 + E];
            yn[e] = -v;
        }
        __syncthreads();
        if (!lds_chol_solve(Hn, nzn, nzn, yn, 12, 12, &ok)) {
            if (lane == 0) bad[a] = 1;
            return;
        }
        for (int e = lane; e < nIn * 12; e += LANES) {
            const int i = e / 12, E = e % 12;
            double v = un[e];
            for (int k = 0; k < nzn; ++k) v += p.Q2n[i * nzn + k] * yn[k * 12 + E];
            un[e] = v;
        }
        __syncthreads();
    }
    for (int e = lane; e < nIn * 12; e += LANES) Un[a * nIn * 12 + e] = un[e];
    // R = Mw u_n, then the next-level ND element u_n^T R + u_n^T Fw + Fw^T u_n + Cnw
    for (int e = lane; e < nIn * 12; e += LANES) {
        const int i = e / 12, E = e % 12;
        double v = 0;
        for (int k = 0; k < nIn; ++k) v += Mw[i * nIn + k] * un[k * 12 + E];
        R[e] = v;
    }
    __syncthreads();
    for (int e = lane; e < 144; e += LANES) {
        const int E = e / 12, E2 = e % 12;
        double v = Cnw[e];
        for (int k = 0; k < nIn; ++k)
            v += un[k * 12 + E] * R[k * 12 + E2] + un[k * 12 + E] * Fw[k * 12 + E2] + Fw[k * 12 + E] * un[k * 12 + E2];
        elnd[a * 144 + e] = v;
    }
}

#define SCHECK(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            fail(e_ == hipErrorOutOfMemory ? AMGE_ERR_OOM : AMGE_ERR_HIP,                         \
                 std::string(#expr) + ": " + hipGetErrorString(e_));                              \
    } while (0)

// Device buffers of one call, freed on every exit.
struct Buffers {
    std::vector<void*> p;
    ~Buffers() {
        for (void* x : p) (void)hipFree(x);
    }
    double* up(const double* src, size_t n) {
        double* d = get<double>(n);
        if (n) SCHECK(hipMemcpy(d, src, n * sizeof(double), hipMemcpyHostToDevice));
        return d;
    }
    template <class T>
    T* get(size_t n) {
        void* x = nullptr;
        SCHECK(hipMalloc(&x, std::max<size_t>(n, 1) * sizeof(T)));
        p.push_back(x);
        return (T*)x;
    }
};

}  // namespace

void kuhn_local_device(const KuhnPlanView& h, const double* w, int64_t nagg, double* U, double* elrt, double* Un,
                       double* elnd) {
    if (nagg <= 0) return;
    if (h.nI > MAXI || h.nz > MAXZ || h.nIn > MAXIN || h.nzn > MAXZN || h.nz < 0 || h.nzn < 0)
        fail(AMGE_ERR_ARG, "local problem larger than the device kernel's tiles");
    using clock = std::chrono::steady_clock;
    const auto t0 = clock::now();
    Buffers B;
    KuhnPlanView d = h;
    const int nz = h.nz, nI = h.nI, nIn = h.nIn, nzn = h.nzn;
    d.H = B.up(h.H, 8 * (size_t)nz * nz);
    d.h = B.up(h.h, 8 * (size_t)nz * 6);
    d.C = B.up(h.C, 8 * 36);
    d.up = B.up(h.up, (size_t)nI * 6);
    d.Q2 = B.up(h.Q2, (size_t)nI * nz);
    if (h.nd) {
        d.CH = B.up(h.CH, 72);
        d.G0 = B.up(h.G0, (size_t)nI * 12);
        d.Wn = B.up(h.Wn, (size_t)nIn * nI);
        d.Q2n = B.up(h.Q2n, (size_t)nIn * nzn);
        d.Mn = B.up(h.Mn, 8 * (size_t)nIn * nIn);
        d.Fn = B.up(h.Fn, 8 * (size_t)nIn * 12);
        d.Cn = B.up(h.Cn, 8 * 144);
    }
    double* dw = B.up(w, (size_t)nagg * 16);
    double* dU = B.get<double>((size_t)nagg * nI * 6);
    double* de = B.get<double>((size_t)nagg * 36);
    double* dUn = B.get<double>(h.nd ? (size_t)nagg * nIn * 12 : 1);
    double* den = B.get<double>(h.nd ? (size_t)nagg * 144 : 1);
    int* bad = B.get<int>((size_t)nagg);
    SCHECK(hipMemset(bad, 0, sizeof(int) * nagg));
    SCHECK(hipStreamSynchronize(nullptr));
    const auto t1 = clock::now();
    k_kuhn_local<<<(unsigned)nagg, LANES>>>(d, dw, dU, de, dUn, den, bad);
    SCHECK(hipGetLastError());
    SCHECK(hipStreamSynchronize(nullptr));
    const auto t2 = clock::now();
    std::vector<int> hb(nagg);
    SCHECK(hipMemcpy(hb.data(), bad, sizeof(int) * nagg, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < nagg; ++i)
        if (hb[i]) fail(AMGE_ERR_NOT_SPD, "local mass not positive definite on the null space");
    SCHECK(hipMemcpy(U, dU, sizeof(double) * nagg * nI * 6, hipMemcpyDeviceToHost));
    SCHECK(hipMemcpy(elrt, de, sizeof(double) * nagg * 36, hipMemcpyDeviceToHost));
    if (h.nd) {
        SCHECK(hipMemcpy(Un, dUn, sizeof(double) * nagg * nIn * 12, hipMemcpyDeviceToHost));
        SCHECK(hipMemcpy(elnd, den, sizeof(double) * nagg * 144, hipMemcpyDeviceToHost));
    }
    const char* v = getenv("AMGE_VERBOSE");
    if (v && *v && *v != '0') {
        auto ms = [](clock::time_point a, clock::time_point b) {
            return std::chrono::duration<double, std::milli>(b - a).count();
        };
        fprintf(stderr, "[amge build] device local problems: %lld agglomerates, upload %.1f ms, kernel %.1f ms, "
                "download %.1f ms\n", (long long)nagg, ms(t0, t1), ms(t1, t2), ms(t2, clock::now()));
    }
}

}  // namespace amge
