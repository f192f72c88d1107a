// Sparse matrix products of set-up on the device (row-wise Gustavson products with a
// hash table per row in LDS).
//
// Every row i of C = A B is built by one 64-lane workgroup: for each entry a_ik of A's
// row in order, the lanes take the entries b_kj of B's row k (distinct columns, so no
// two lanes touch one table slot) and add a_ik * b_kj to the slot of column j; a
// barrier separates the entries of A's row.  Each sum therefore runs in A's row order
// with separately rounded products and sums (no fused multiply-add), which is what the
// host product computes; the table is then read out in increasing column order.  Rows
// are binned by the number of products they take (an upper bound on their distinct
// columns) for the count, and by their exact count for the fill, into tables of 256,
// 1024 and 4096 slots.
#include "spgemm_device.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

namespace amge {
namespace {

constexpr int LANES = 64;
constexpr int TS_SMALL = 256, TS_MID = 1024, TS_LARGE = 4096;

#define PCHECK(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            fail(e_ == hipErrorOutOfMemory ? AMGE_ERR_OOM : AMGE_ERR_HIP,                         \
                 std::string(#expr) + ": " + hipGetErrorString(e_));                              \
    } while (0)

// Products per row of C = A B (sum of the lengths of the B rows A's row selects),
// clamped to INT_MAX.
__global__ void __launch_bounds__(256)
k_row_products(int nrows, const int* __restrict__ arp, const int* __restrict__ acol, const int* __restrict__ brp,
               int* __restrict__ ub) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrows) return;
    int64_t s = 0;
    for (int k = arp[i]; k < arp[i + 1]; ++k) s += brp[acol[k] + 1] - brp[acol[k]];
    ub[i] = (int)std::min<int64_t>(s, INT_MAX);
}

__device__ __forceinline__ unsigned slot_of(int c, int TS) { return ((unsigned)c * 2654435761u) & (unsigned)(TS - 1); }

// Insert column c (linear probing); returns its slot, or -1 if the table is full.  fresh:
// whether this call placed it.
template <int TS>
__device__ __forceinline__ int insert(int* keys, int c, bool& fresh) {
    unsigned s = slot_of(c, TS);
    for (int probe = 0; probe < TS; ++probe) {
        const int prev = atomicCAS(&keys[s], -1, c);
        if (prev == -1 || prev == c) {
            fresh = prev == -1;
            return (int)s;
        }
        s = (s + 1) & (unsigned)(TS - 1);
    }
    fresh = false;
    return -1;
}

// Distinct columns of the rows in `rows`; *full set if a row does not fit the table.
template <int TS>
__global__ void __launch_bounds__(LANES)
k_row_count(const int* __restrict__ rows, const int* __restrict__ arp, const int* __restrict__ acol,
            const int* __restrict__ brp, const int* __restrict__ bcol, int* __restrict__ cnt, int* __restrict__ full) {
    __shared__ int keys[TS];
    __shared__ int n;
    const int i = rows[blockIdx.x];
    const int lane = threadIdx.x;
    for (int s = lane; s < TS; s += LANES) keys[s] = -1;
    if (lane == 0) n = 0;
    __syncthreads();
    bool over = false;
    for (int k = arp[i]; k < arp[i + 1]; ++k) {
        const int j = acol[k];
        for (int l = brp[j] + lane; l < brp[j + 1]; l += LANES) {
            bool fresh;
            if (insert<TS>(keys, bcol[l], fresh) < 0) over = true;
            else if (fresh) atomicAdd(&n, 1);
        }
    }
    if (over) atomicOr(full, 1);
    __syncthreads();
    if (lane == 0) cnt[i] = n;
}

// Values and sorted columns of the rows in `rows` (their counts are known to fit).
template <int TS>
__global__ void __launch_bounds__(LANES)
k_row_fill(const int* __restrict__ rows, const int* __restrict__ arp, const int* __restrict__ acol,
           const double* __restrict__ aval, const int* __restrict__ brp, const int* __restrict__ bcol,
           const double* __restrict__ bval, const int* __restrict__ crp, int* __restrict__ ccol,
           double* __restrict__ cval) {
    __shared__ int keys[TS];
    __shared__ double vals[TS];
    const int i = rows[blockIdx.x];
    const int lane = threadIdx.x;
    for (int s = lane; s < TS; s += LANES) {
        keys[s] = -1;
        vals[s] = 0.0;
    }
    __syncthreads();
    // the first chunk of the next entry's B row is loaded while this entry's terms are
    // added
    const int k0 = arp[i], k1 = arp[i + 1];
    int lb = 0, le = 0, c = -1;
    double a = 0.0, b = 0.0;
    if (k0 < k1) {
        const int j = acol[k0];
        a = aval[k0];
        lb = brp[j];
        le = brp[j + 1];
        if (lb + lane < le) {
            c = bcol[lb + lane];
            b = bval[lb + lane];
        }
    }
    for (int k = k0; k < k1; ++k) {
        int lb2 = 0, le2 = 0, c2 = -1;
        double a2 = 0.0, b2 = 0.0;
        if (k + 1 < k1) {
            const int j = acol[k + 1];
            a2 = aval[k + 1];
            lb2 = brp[j];
            le2 = brp[j + 1];
            if (lb2 + lane < le2) {
                c2 = bcol[lb2 + lane];
                b2 = bval[lb2 + lane];
            }
        }
        {
            // a product and a sum, each rounded (the compiler would otherwise fuse them)
#pragma clang fp contract(off)
            bool fresh;
            if (c >= 0) {
                const int s = insert<TS>(keys, c, fresh);
                if (s >= 0) vals[s] = vals[s] + a * b;
            }
            for (int l = lb + LANES + lane; l < le; l += LANES) {
                const int s = insert<TS>(keys, bcol[l], fresh);
                if (s >= 0) vals[s] = vals[s] + a * bval[l];
            }
        }
        __syncthreads();   // the next entry of A's row adds after this one
        lb = lb2;
        le = le2;
        c = c2;
        a = a2;
        b = b2;
    }
    // compact the stored columns to the front of the table, in slot order (a chunk's
    // loads precede its stores, and its stores land below the next chunk)
    int n = 0;
    for (int s0 = 0; s0 < TS; s0 += LANES) {
        const int key = keys[s0 + lane];
        const double v = vals[s0 + lane];
        const uint64_t m = __ballot(key >= 0);
        const int pos = n + __popcll(m & ((1ull << lane) - 1));
        if (key >= 0) {
            keys[pos] = key;
            vals[pos] = v;
        }
        n += __popcll(m);
    }
    __syncthreads();
    // rank of each column among the row's columns = its position in the output
    const int base = crp[i];
    for (int e = lane; e < n; e += LANES) {
        const int key = keys[e];
        int r = 0;
        for (int t = 0; t < n; ++t) r += keys[t] < key;
        ccol[base + r] = key;
        cval[base + r] = vals[e];
    }
}

// A CSR matrix in device memory (allocations owned by a DeviceProducts).
struct DevCsr {
    int32_t nrows = 0, ncols = 0;
    int64_t nnz = 0;
    int32_t* rowptr = nullptr;
    int32_t* col = nullptr;
    double* val = nullptr;
};

// Device memory and stream of a chain of products; everything it allocated is freed with
// it.
class DeviceProducts {
public:
    DeviceProducts(hipStream_t s, const amge_opts* o) : s_(s) {
        if (o && o->alloc && o->dealloc) {
            alloc_ = o->alloc;
            dealloc_ = o->dealloc;
            user_ = o->alloc_user;
        }
    }
    ~DeviceProducts();
    DeviceProducts(const DeviceProducts&) = delete;
    DeviceProducts& operator=(const DeviceProducts&) = delete;
    DevCsr upload(const Csr& A);
    Csr download(const DevCsr& A);
    // C = A B; false (C untouched) when a row of C has more distinct columns than the
    // largest table
    bool multiply(const DevCsr& A, const DevCsr& B, DevCsr& C);

private:
    template <class T>
    T* alloc(size_t n);
    hipStream_t s_;
    void* (*alloc_)(size_t, void*) = nullptr;
    void (*dealloc_)(void*, void*) = nullptr;
    void* user_ = nullptr;
    std::vector<void*> mem_;
};

// Wall-clock phases of the device products, printed with AMGE_VERBOSE.
struct ProductClock {
    std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
    double up = 0, mul = 0, down = 0;
    bool on;
    ProductClock() {
        const char* e = getenv("AMGE_VERBOSE");
        on = e && *e && *e != '0';
    }
    void lap(double& acc) {
        const auto now = std::chrono::steady_clock::now();
        acc += std::chrono::duration<double, std::milli>(now - t).count();
        t = now;
    }
    ~ProductClock() {
        if (on) fprintf(stderr, "[amge product] upload %.1f ms, products %.1f ms, download %.1f ms\n", up, mul, down);
    }
};

}  // namespace

bool device_products() {
    const char* e = getenv("AMGE_HOST_PRODUCTS");
    return !(e && *e && *e != '0');
}

int device_product_max_row() { return TS_LARGE; }

DeviceProducts::~DeviceProducts() {
    // a caller's allocator may hand the memory out again at once: nothing may still use it
    if (dealloc_) (void)hipDeviceSynchronize();
    else (void)hipStreamSynchronize(s_);
    for (void* p : mem_) {
        if (dealloc_) dealloc_(p, user_);
        else (void)hipFree(p);
    }
}

template <class T>
T* DeviceProducts::alloc(size_t n) {
    const size_t nb = std::max<size_t>(n, 1) * sizeof(T);
    void* p = nullptr;
    if (alloc_) {
        p = alloc_(nb, user_);
        if (!p) fail(AMGE_ERR_OOM, "the caller's allocator returned no memory for a set-up product");
    } else {
        PCHECK(hipMalloc(&p, nb));
    }
    mem_.push_back(p);
    return (T*)p;
}

DevCsr DeviceProducts::upload(const Csr& A) {
    DevCsr d;
    d.nrows = A.nrows;
    d.ncols = A.ncols;
    d.nnz = A.nnz();
    d.rowptr = alloc<int32_t>(A.rowptr.size());
    d.col = alloc<int32_t>(A.col.size());
    d.val = alloc<double>(A.val.size());
    PCHECK(hipMemcpyAsync(d.rowptr, A.rowptr.data(), A.rowptr.size() * sizeof(int32_t), hipMemcpyHostToDevice, s_));
    if (d.nnz) {
        PCHECK(hipMemcpyAsync(d.col, A.col.data(), A.col.size() * sizeof(int32_t), hipMemcpyHostToDevice, s_));
        PCHECK(hipMemcpyAsync(d.val, A.val.data(), A.val.size() * sizeof(double), hipMemcpyHostToDevice, s_));
    }
    PCHECK(hipStreamSynchronize(s_));   // the host vectors may go after return
    return d;
}

Csr DeviceProducts::download(const DevCsr& d) {
    Csr A;
    A.nrows = d.nrows;
    A.ncols = d.ncols;
    A.rowptr.resize((size_t)d.nrows + 1);
    A.col.resize(d.nnz);
    A.val.resize(d.nnz);
    PCHECK(hipMemcpyAsync(A.rowptr.data(), d.rowptr, A.rowptr.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s_));
    if (d.nnz) {
        PCHECK(hipMemcpyAsync(A.col.data(), d.col, A.col.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s_));
        PCHECK(hipMemcpyAsync(A.val.data(), d.val, A.val.size() * sizeof(double), hipMemcpyDeviceToHost, s_));
    }
    PCHECK(hipStreamSynchronize(s_));
    return A;
}

bool DeviceProducts::multiply(const DevCsr& A, const DevCsr& B, DevCsr& C) {
    if (A.ncols != B.nrows) fail(AMGE_ERR_SHAPE, "spgemm: inner dimensions differ");
    const int nr = A.nrows;
    DevCsr R;
    R.nrows = nr;
    R.ncols = B.ncols;
    R.rowptr = alloc<int32_t>((size_t)nr + 1);
    if (nr == 0) {
        PCHECK(hipMemsetAsync(R.rowptr, 0, sizeof(int32_t), s_));
        PCHECK(hipStreamSynchronize(s_));
        R.col = alloc<int32_t>(0);
        R.val = alloc<double>(0);
        C = R;
        return true;
    }
    // bins by products per row
    int* ub = alloc<int>(nr);
    k_row_products<<<(nr + 255) / 256, 256, 0, s_>>>(nr, A.rowptr, A.col, B.rowptr, ub);
    PCHECK(hipGetLastError());
    std::vector<int> hub(nr);
    PCHECK(hipMemcpyAsync(hub.data(), ub, sizeof(int) * nr, hipMemcpyDeviceToHost, s_));
    PCHECK(hipStreamSynchronize(s_));
    std::vector<int> bins[3];
    for (int i = 0; i < nr; ++i) bins[hub[i] <= TS_SMALL / 2 ? 0 : hub[i] <= TS_MID / 2 ? 1 : 2].push_back(i);
    int* drows[3];
    for (int b = 0; b < 3; ++b) {
        drows[b] = alloc<int>(bins[b].size());
        if (!bins[b].empty())
            PCHECK(hipMemcpyAsync(drows[b], bins[b].data(), sizeof(int) * bins[b].size(), hipMemcpyHostToDevice, s_));
    }
    int* cnt = alloc<int>(nr);
    int* full = alloc<int>(1);
    PCHECK(hipMemsetAsync(full, 0, sizeof(int), s_));
    const unsigned nb[3] = {(unsigned)bins[0].size(), (unsigned)bins[1].size(), (unsigned)bins[2].size()};
    if (nb[0]) k_row_count<TS_SMALL><<<nb[0], LANES, 0, s_>>>(drows[0], A.rowptr, A.col, B.rowptr, B.col, cnt, full);
    if (nb[1]) k_row_count<TS_MID><<<nb[1], LANES, 0, s_>>>(drows[1], A.rowptr, A.col, B.rowptr, B.col, cnt, full);
    if (nb[2]) k_row_count<TS_LARGE><<<nb[2], LANES, 0, s_>>>(drows[2], A.rowptr, A.col, B.rowptr, B.col, cnt, full);
    PCHECK(hipGetLastError());
    std::vector<int> hc(nr);
    int hfull = 0;
    PCHECK(hipMemcpyAsync(hc.data(), cnt, sizeof(int) * nr, hipMemcpyDeviceToHost, s_));
    PCHECK(hipMemcpyAsync(&hfull, full, sizeof(int), hipMemcpyDeviceToHost, s_));
    PCHECK(hipStreamSynchronize(s_));
    if (hfull) return false;
    std::vector<int32_t> rp((size_t)nr + 1, 0);
    int64_t tot = 0;
    for (int i = 0; i < nr; ++i) {
        tot += hc[i];
        if (tot > INT32_MAX) fail(AMGE_ERR_SHAPE, "spgemm: result exceeds int32 nnz");
        rp[i + 1] = (int32_t)tot;
    }
    R.nnz = tot;
    R.col = alloc<int32_t>(tot);
    R.val = alloc<double>(tot);
    // the fill's tables sized by the exact counts (load <= 1/2 below the largest table)
    for (int b = 0; b < 3; ++b) bins[b].clear();
    for (int i = 0; i < nr; ++i) bins[hc[i] <= TS_SMALL / 2 ? 0 : hc[i] <= TS_MID / 2 ? 1 : 2].push_back(i);
    unsigned nf[3];
    int* frows[3];
    for (int b = 0; b < 3; ++b) {
        nf[b] = (unsigned)bins[b].size();
        frows[b] = alloc<int>(bins[b].size());
        if (!bins[b].empty())
            PCHECK(hipMemcpyAsync(frows[b], bins[b].data(), sizeof(int) * bins[b].size(), hipMemcpyHostToDevice, s_));
    }
    PCHECK(hipMemcpyAsync(R.rowptr, rp.data(), sizeof(int32_t) * rp.size(), hipMemcpyHostToDevice, s_));
    if (nf[0])
        k_row_fill<TS_SMALL><<<nf[0], LANES, 0, s_>>>(frows[0], A.rowptr, A.col, A.val, B.rowptr, B.col, B.val,
                                                      R.rowptr, R.col, R.val);
    if (nf[1])
        k_row_fill<TS_MID><<<nf[1], LANES, 0, s_>>>(frows[1], A.rowptr, A.col, A.val, B.rowptr, B.col, B.val,
                                                    R.rowptr, R.col, R.val);
    if (nf[2])
        k_row_fill<TS_LARGE><<<nf[2], LANES, 0, s_>>>(frows[2], A.rowptr, A.col, A.val, B.rowptr, B.col, B.val,
                                                      R.rowptr, R.col, R.val);
    PCHECK(hipGetLastError());
    PCHECK(hipStreamSynchronize(s_));   // rp goes out of scope
    C = R;
    return true;
}

Csr spgemm_on_device(const Csr& A, const Csr& B, void* stream, const amge_opts* opts) {
    if (!device_products()) return spgemm(A, B);
    ProductClock clk;
    DeviceProducts dp((hipStream_t)stream, opts);
    const DevCsr a = dp.upload(A), b = dp.upload(B);
    clk.lap(clk.up);
    DevCsr c;
    if (!dp.multiply(a, b, c)) return spgemm(A, B);
    clk.lap(clk.mul);
    Csr r = dp.download(c);
    clk.lap(clk.down);
    return r;
}

Csr triple_on_device(const Csr& L, const Csr& A, const Csr& R, void* stream, const amge_opts* opts) {
    if (!device_products()) return spgemm(L, spgemm(A, R));
    ProductClock clk;
    DeviceProducts dp((hipStream_t)stream, opts);
    const DevCsr l = dp.upload(L), a = dp.upload(A), r = dp.upload(R);
    clk.lap(clk.up);
    DevCsr ar, lar;
    if (!dp.multiply(a, r, ar)) return spgemm(L, spgemm(A, R));
    if (!dp.multiply(l, ar, lar)) return spgemm(L, dp.download(ar));
    clk.lap(clk.mul);
    Csr res = dp.download(lar);
    clk.lap(clk.down);
    return res;
}

std::pair<Csr, Csr> chain_on_device(const Csr& X, const Csr& Y, const Csr& Z, void* stream,
                                    const amge_opts* opts) {
    if (!device_products()) {
        Csr xy = spgemm(X, Y);
        Csr xyz = spgemm(xy, Z);
        return {std::move(xy), std::move(xyz)};
    }
    ProductClock clk;
    DeviceProducts dp((hipStream_t)stream, opts);
    const DevCsr x = dp.upload(X), y = dp.upload(Y), z = dp.upload(Z);
    clk.lap(clk.up);
    DevCsr xy, xyz;
    if (!dp.multiply(x, y, xy)) {
        Csr h = spgemm(X, Y);
        Csr h2 = spgemm(h, Z);
        return {std::move(h), std::move(h2)};
    }
    clk.lap(clk.mul);
    Csr hxy = dp.download(xy);
    clk.lap(clk.down);
    if (!dp.multiply(xy, z, xyz)) {
        Csr h2 = spgemm(hxy, Z);
        return {std::move(hxy), std::move(h2)};
    }
    clk.lap(clk.mul);
    Csr hxyz = dp.download(xyz);
    clk.lap(clk.down);
    return {std::move(hxy), std::move(hxyz)};
}

}  // namespace amge
