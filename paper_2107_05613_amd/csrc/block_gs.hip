// l1-scaled symmetric block Gauss-Seidel smoother (section 4.1, last paragraph; section
// 5.1): layout of the level matrices for k_bgs, its launches, and the host sweep used
// when a coarse tail is folded.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <limits>
#include <type_traits>

#include "block_gs.hpp"
#include "kernels_bgs.hpp"

namespace amge {

namespace {

template <class T>
T* upload_vec(amge_hierarchy* H, const std::vector<T>& v, hipStream_t s) {
    T* d = H->alloc<T>(v.size());
    if (!v.empty()) HIPCHECK(hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return d;
}

}  // namespace

BgsHost bgs_layout(const Csr& A) {
    BgsHost g;
    const int n = A.nrows;
    g.n = n;
    g.nnz = A.nnz();
    g.nblk = (n + BGS_ROWS - 1) / BGS_ROWS;
    g.blk.resize(g.nblk);
    g.meta.assign(n, 0);
    g.dinv.assign(n, 0.0);
    g.mid.assign(n, 0.0);
    std::vector<int> width(g.nblk, 0), wi(g.nblk, 0), cmin(g.nblk, 0), cmax(g.nblk, 0);
    std::vector<int64_t> inside(g.nblk, 0);
    std::vector<std::string> err(g.nblk);
    // colours, inside counts, l1 sums and block shapes, block by block
    parallel_for(g.nblk, [&](int64_t b0, int64_t b1) {
        std::vector<int> colour(BGS_ROWS);
        for (int64_t bk = b0; bk < b1; ++bk) {
            const int r0 = (int)bk * BGS_ROWS, r1 = std::min(n, r0 + BGS_ROWS);
            int w = 0, mi = 0, ncol = 0;
            int lo = std::numeric_limits<int>::max(), hi = -1;
            for (int i = r0; i < r1; ++i) {
                uint64_t used = 0;
                double aii = 0, l1 = 0;
                int k = 0;
                for (int q = A.rowptr[i]; q < A.rowptr[i + 1]; ++q) {
                    const int j = A.col[q];
                    const double v = A.val[q];
                    if (j >= r0 && j < r1) {
                        ++k;
                        if (j == i) aii += v;
                        if (j < i && v != 0) used |= 1ull << colour[j - r0];
                    } else {
                        l1 += std::fabs(v);
                        lo = std::min(lo, j);
                        hi = std::max(hi, j);
                    }
                }
                const int c = __builtin_ctzll(~used);
                colour[i - r0] = c;
                g.meta[i] = (uint16_t)(k | c << 8);
                const double d = aii + l1;
                if (!(aii > 0) || !(d > 0)) {
                    err[bk] = "block Gauss-Seidel needs a positive diagonal";
                    break;
                }
                g.dinv[i] = 1.0 / d;
                g.mid[i] = aii + 2.0 * l1;
                mi = std::max(mi, k);
                w = std::max(w, A.rowptr[i + 1] - A.rowptr[i]);
                ncol = std::max(ncol, c + 1);
                inside[bk] += k;
            }
            width[bk] = w;
            wi[bk] = mi;
            g.blk[bk].width = w;
            g.blk[bk].info = mi | ncol << 8;
            cmin[bk] = hi >= 0 ? lo : 0;
            cmax[bk] = hi >= 0 ? hi : 0;
        }
    });
    for (const std::string& e : err)
        if (!e.empty()) fail(AMGE_ERR_NOT_SPD, e);
    for (int bk = 0; bk < g.nblk; ++bk) {
        g.ninmax = std::max(g.ninmax, wi[bk]);
        g.nnz_in += inside[bk];
    }
    if (g.ninmax > BGS_ROWS) fail(AMGE_ERR_SHAPE, "duplicate entries in a block Gauss-Seidel matrix");
    static const int bounds[] = {8, 12, 16, 32, 64};
    for (int bnd : bounds)
        if (g.ninmax <= bnd) {
            g.nin = bnd;
            break;
        }
    g.c16 = true;
    for (int bk = 0; bk < g.nblk; ++bk) g.c16 = g.c16 && cmax[bk] - cmin[bk] < 65536;
    int64_t base = 0;
    for (int bk = 0; bk < g.nblk; ++bk) {
        g.blk[bk].base = (int)base;
        g.blk[bk].cbase = g.c16 ? cmin[bk] : 0;
        base += (int64_t)BGS_ROWS * width[bk];
        if (base > std::numeric_limits<int>::max()) fail(AMGE_ERR_SHAPE, "block Gauss-Seidel layout too large");
    }
    // the sweeps read the first g.nin entries of every row of a block unconditionally:
    // pad past the end so that the last block's reads stay inside the arrays
    g.code.assign(base + (int64_t)BGS_ROWS * g.nin, 0);
    g.val.assign(base + (int64_t)BGS_ROWS * g.nin, 0.0);
    parallel_for(g.nblk, [&](int64_t b0, int64_t b1) {
        for (int64_t bk = b0; bk < b1; ++bk) {
            const int r0 = (int)bk * BGS_ROWS, r1 = std::min(n, r0 + BGS_ROWS);
            const int64_t e0 = g.blk[bk].base;
            const int cb = g.blk[bk].cbase;
            for (int i = r0; i < r1; ++i) {
                const int lane = i - r0;
                int tin = 0, tout = g.meta[i] & 0xff;
                for (int q = A.rowptr[i]; q < A.rowptr[i + 1]; ++q) {
                    const int j = A.col[q];
                    const bool in = j >= r0 && j < r1;
                    const int64_t e = e0 + (int64_t)(in ? tin++ : tout++) * BGS_ROWS + lane;
                    g.code[e] = in ? j - r0 : j - cb;
                    g.val[e] = A.val[q];
                }
            }
        }
    });
    return g;
}

void build_bgs(amge_hierarchy* H, const Csr& A, DBgs& g, hipStream_t s) {
    BgsHost h = bgs_layout(A);
    g.n = h.n;
    g.nblk = h.nblk;
    g.nin = h.nin;
    g.nnz = h.nnz;
    g.nnz_in = h.nnz_in;
    g.blk = upload_vec(H, h.blk, s);
    g.meta = upload_vec(H, h.meta, s);
    std::vector<float> v32(h.val.begin(), h.val.end());
    std::vector<float> d32(h.dinv.begin(), h.dinv.end()), m32(h.mid.begin(), h.mid.end());
    std::vector<uint16_t> c16;
    if (h.c16) {
        c16.assign(h.code.begin(), h.code.end());
        g.c16 = upload_vec(H, c16, s);
    } else {
        g.ci = upload_vec(H, h.code, s);
    }
    g.v64 = upload_vec(H, h.val, s);
    g.v32 = upload_vec(H, v32, s);
    g.dinv64 = upload_vec(H, h.dinv, s);
    g.mid64 = upload_vec(H, h.mid, s);
    g.dinv32 = upload_vec(H, d32, s);
    g.mid32 = upload_vec(H, m32, s);
    HIPCHECK(hipStreamSynchronize(s));   // the host vectors go out of scope
}

namespace {

template <class T> const T* vals(const DBgs& g);
template <> const double* vals<double>(const DBgs& g) { return g.v64; }
template <> const float* vals<float>(const DBgs& g) { return g.v32; }
template <class T> const T* dinvs(const DBgs& g);
template <> const double* dinvs<double>(const DBgs& g) { return g.dinv64; }
template <> const float* dinvs<float>(const DBgs& g) { return g.dinv32; }
template <class T> const T* mids(const DBgs& g);
template <> const double* mids<double>(const DBgs& g) { return g.mid64; }
template <> const float* mids<float>(const DBgs& g) { return g.mid32; }

template <class T, bool C16, bool ZERO, int NIN>
void go(const DBgs& g, const T* x, const T* b, T* y, hipStream_t s, const int* stop) {
    const unsigned grid = (unsigned)((g.nblk + dev::WAVES - 1) / dev::WAVES);
    dev::k_bgs<T, C16, ZERO, NIN><<<grid, dev::BLOCK, 0, s>>>(g.nblk, g.n, g.blk, g.meta, g.ci, g.c16, vals<T>(g),
                                                               dinvs<T>(g), mids<T>(g), x, b, y, stop);
}

template <class T, bool C16, bool ZERO>
void go_nin(const DBgs& g, const T* x, const T* b, T* y, hipStream_t s, const int* stop) {
    switch (g.nin) {
        case 8: go<T, C16, ZERO, 8>(g, x, b, y, s, stop); break;
        case 12: go<T, C16, ZERO, 12>(g, x, b, y, s, stop); break;
        case 16: go<T, C16, ZERO, 16>(g, x, b, y, s, stop); break;
        case 32: go<T, C16, ZERO, 32>(g, x, b, y, s, stop); break;
        default: go<T, C16, ZERO, 64>(g, x, b, y, s, stop); break;
    }
}

}  // namespace

template <class T>
void bgs_launch(const DBgs& g, bool zero, const T* x, const T* b, T* y, hipStream_t s, const int* stop) {
    if (g.nblk == 0) return;
    const bool c16 = g.c16 != nullptr;
    if (zero) {
        if (c16) go_nin<T, true, true>(g, x, b, y, s, stop);
        else go_nin<T, false, true>(g, x, b, y, s, stop);
    } else {
        if (c16) go_nin<T, true, false>(g, x, b, y, s, stop);
        else go_nin<T, false, false>(g, x, b, y, s, stop);
    }
}

template void bgs_launch<float>(const DBgs&, bool, const float*, const float*, float*, hipStream_t, const int*);
template void bgs_launch<double>(const DBgs&, bool, const double*, const double*, double*, hipStream_t,
                                 const int*);

template <class T>
void bgs_resid_launch(const DBgs& g, bool v64, const T* x, const T* b, T* y, hipStream_t s, const int* stop) {
    if (g.nblk == 0) return;
    const unsigned grid = (unsigned)((g.nblk + dev::WAVES - 1) / dev::WAVES);
    const bool c16 = g.c16 != nullptr;
    if (v64 && !std::is_same<T, double>::value) {
        if (c16)
            dev::k_bgs_resid<T, true, double><<<grid, dev::BLOCK, 0, s>>>(g.nblk, g.n, g.blk, g.meta, g.ci, g.c16,
                                                                           g.v64, x, b, y, stop);
        else
            dev::k_bgs_resid<T, false, double><<<grid, dev::BLOCK, 0, s>>>(g.nblk, g.n, g.blk, g.meta, g.ci, g.c16,
                                                                            g.v64, x, b, y, stop);
        return;
    }
    if (c16)
        dev::k_bgs_resid<T, true, T><<<grid, dev::BLOCK, 0, s>>>(g.nblk, g.n, g.blk, g.meta, g.ci, g.c16, vals<T>(g), x,
                                                                  b, y, stop);
    else
        dev::k_bgs_resid<T, false, T><<<grid, dev::BLOCK, 0, s>>>(g.nblk, g.n, g.blk, g.meta, g.ci, g.c16, vals<T>(g),
                                                                   x, b, y, stop);
}

template void bgs_resid_launch<float>(const DBgs&, bool, const float*, const float*, float*, hipStream_t,
                                      const int*);
template void bgs_resid_launch<double>(const DBgs&, bool, const double*, const double*, double*, hipStream_t,
                                       const int*);

double bgs_bytes(const DBgs& g, bool zero, int vbytes, int cols) {
    const double cb = g.c16 ? 2 : 4;
    const double ent = (double)(zero ? g.nnz_in : g.nnz) * (vbytes + cb);
    // per row: meta (2 bytes), the two scalings, and per column b, y (and x for a full
    // sweep); per block its record
    return ent + (double)g.n * (2 + 2 * vbytes + (zero ? 2 : 3) * (double)cols * vbytes) + 16.0 * g.nblk;
}

double bgs_resid_bytes(const DBgs& g, int vbytes, int xbytes, int cols) {
    const double cb = g.c16 ? 2 : 4;
    // entries; per row: meta, and per column x, b, y; per block its record
    return (double)g.nnz * (vbytes + cb) + (double)g.n * (2 + 3 * (double)cols * xbytes) + 16.0 * g.nblk;
}

void host_bgs_sweep(const BgsHost& g, const double* b, double* x, std::vector<double>& tmp) {
    std::vector<double>& r = tmp;
    r.assign(g.n, 0.0);
    // r = b - A x with the values at the start of the sweep, every row before any changes
    for (int bk = 0; bk < g.nblk; ++bk) {
        const dev::BgsBlock& B = g.blk[bk];
        const int r0 = bk * BGS_ROWS, r1 = std::min(g.n, r0 + BGS_ROWS);
        for (int i = r0; i < r1; ++i) {
            const int lane = i - r0, nin = g.meta[i] & 0xff;
            double acc = 0;
            for (int t = 0; t < B.width; ++t) {
                const int64_t e = B.base + (int64_t)t * BGS_ROWS + lane;
                const int j = t < nin ? r0 + g.code[e] : (g.c16 ? B.cbase + g.code[e] : g.code[e]);
                acc += g.val[e] * x[j];
            }
            r[i] = b[i] - acc;
        }
    }
    double u[BGS_ROWS], w[BGS_ROWS];
    for (int bk = 0; bk < g.nblk; ++bk) {
        const dev::BgsBlock& B = g.blk[bk];
        const int r0 = bk * BGS_ROWS, r1 = std::min(g.n, r0 + BGS_ROWS);
        const int ncol = B.info >> 8;
        std::fill(u, u + BGS_ROWS, 0.0);
        std::fill(w, w + BGS_ROWS, 0.0);
        auto inside = [&](int i, const double* z) {
            const int lane = i - r0, nin = g.meta[i] & 0xff;
            double s = 0;
            for (int t = 0; t < nin; ++t) {
                const int64_t e = B.base + (int64_t)t * BGS_ROWS + lane;
                s += g.val[e] * z[g.code[e]];
            }
            return s;
        };
        for (int c = 0; c < ncol; ++c)
            for (int i = r0; i < r1; ++i)
                if ((g.meta[i] >> 8) == c) u[i - r0] = (r[i] - inside(i, u)) * g.dinv[i];
        for (int c = ncol - 1; c >= 0; --c)
            for (int i = r0; i < r1; ++i)
                if ((g.meta[i] >> 8) == c) w[i - r0] = (g.mid[i] * u[i - r0] - inside(i, w)) * g.dinv[i];
        for (int i = r0; i < r1; ++i) x[i] += w[i - r0];
    }
}

}  // namespace amge
