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
    g.meta.assign((size_t)g.nblk * BGS_ROWS, 0xffu << 24);
    g.dinv.assign(n, 0.0);
    g.mid.assign(n, 0.0);
    std::vector<int> wi(g.nblk, 0), cmin(g.nblk, 0), cmax(g.nblk, 0);
    std::vector<int64_t> inside(g.nblk, 0), stored(g.nblk, 0);
    std::vector<std::string> err(g.nblk);
    std::vector<amge_status> code(g.nblk, AMGE_OK);
    // colours, inside counts, l1 sums, lane order (rows by length, longest first) and block
    // shapes, block by block
    parallel_for(g.nblk, [&](int64_t b0, int64_t b1) {
        int colour[BGS_ROWS], nin[BGS_ROWS], len[BGS_ROWS], lane_row[BGS_ROWS];
        for (int64_t bk = b0; bk < b1; ++bk) {
            const int r0 = (int)bk * BGS_ROWS, r1 = std::min(n, r0 + BGS_ROWS), nr = r1 - r0;
            int mi = 0, ncol = 0;
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
                nin[i - r0] = k;
                len[i - r0] = A.rowptr[i + 1] - A.rowptr[i];
                const double d = aii + l1;
                if (!(aii > 0) || !(d > 0)) {
                    err[bk] = "block Gauss-Seidel needs a positive diagonal";
                    code[bk] = AMGE_ERR_NOT_SPD;
                    break;
                }
                if (len[i - r0] > 255) {
                    err[bk] = "block Gauss-Seidel rows hold at most 255 entries";
                    code[bk] = AMGE_ERR_SHAPE;
                    break;
                }
                g.dinv[i] = 1.0 / d;
                g.mid[i] = aii + 2.0 * l1;
                mi = std::max(mi, k);
                ncol = std::max(ncol, c + 1);
                inside[bk] += k;
                stored[bk] += len[i - r0];
            }
            if (!err[bk].empty()) continue;
            for (int q = 0; q < nr; ++q) lane_row[q] = q;
            std::stable_sort(lane_row, lane_row + nr, [&](int u, int v) { return len[u] > len[v]; });
            for (int q = 0; q < nr; ++q) {
                const int p = lane_row[q];
                g.meta[(size_t)bk * BGS_ROWS + q] =
                    (uint32_t)nin[p] | (uint32_t)colour[p] << 8 | (uint32_t)len[p] << 16 | (uint32_t)p << 24;
            }
            wi[bk] = mi;
            g.blk[bk].width = nr ? len[lane_row[0]] : 0;
            g.blk[bk].info = mi | ncol << 8 | (nr ? len[lane_row[nr - 1]] : 0) << 16 | nr << 24;
            cmin[bk] = hi >= 0 ? lo : 0;
            cmax[bk] = hi >= 0 ? hi : 0;
        }
    });
    for (int bk = 0; bk < g.nblk; ++bk)
        if (!err[bk].empty()) fail(code[bk], err[bk]);
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
        base += stored[bk];
        if (base > std::numeric_limits<int>::max() - 64 * 65) fail(AMGE_ERR_SHAPE, "block Gauss-Seidel layout too large");
    }
    // the kernels issue loads for every lane of every slab up to their register bound
    // (results of lanes past a slab's rows are masked): pad past the end so that the last
    // block's loads stay inside the arrays
    g.code.assign(base + (int64_t)BGS_ROWS * (g.nin + 1), 0);
    g.val.assign(base + (int64_t)BGS_ROWS * (g.nin + 1), 0.0);
    parallel_for(g.nblk, [&](int64_t b0, int64_t b1) {
        for (int64_t bk = b0; bk < b1; ++bk) {
            const int r0 = (int)bk * BGS_ROWS, r1 = std::min(n, r0 + BGS_ROWS);
            const int cb = g.blk[bk].cbase;
            const uint32_t* mt = &g.meta[(size_t)bk * BGS_ROWS];
            int cnt[256] = {0};   // rows longer than t, for every slab t
            for (int q = 0; q < r1 - r0; ++q)
                for (int t = 0; t < (int)((mt[q] >> 16) & 0xff); ++t) ++cnt[t];
            int64_t off[257];
            off[0] = g.blk[bk].base;
            for (int t = 0; t < g.blk[bk].width; ++t) off[t + 1] = off[t] + cnt[t];
            for (int q = 0; q < r1 - r0; ++q) {
                const int i = r0 + (int)(mt[q] >> 24);
                int tin = 0, tout = mt[q] & 0xff;
                for (int p = A.rowptr[i]; p < A.rowptr[i + 1]; ++p) {
                    const int j = A.col[p];
                    const bool in = j >= r0 && j < r1;
                    const int t = in ? tin++ : tout++;
                    const int64_t e = off[t] + q;
                    g.code[e] = in ? j - r0 : j - cb;
                    g.val[e] = A.val[p];
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
    // per row: its 4-byte lane word, the two scalings, and per column b, y (and x for a
    // full sweep); per block its record
    return ent + (double)g.n * (4 + 2 * vbytes + (zero ? 2 : 3) * (double)cols * vbytes) + 16.0 * g.nblk;
}

double bgs_resid_bytes(const DBgs& g, int vbytes, int xbytes, int cols) {
    const double cb = g.c16 ? 2 : 4;
    // entries; per row: its lane word, and per column x, b, y; per block its record
    return (double)g.nnz * (vbytes + cb) + (double)g.n * (4 + 3 * (double)cols * xbytes) + 16.0 * g.nblk;
}

void host_bgs_sweep(const BgsHost& g, const double* b, double* x, std::vector<double>& tmp) {
    std::vector<double>& r = tmp;
    r.assign(g.n, 0.0);
    // entry t of lane q: slab offsets of the block's jagged diagonals
    auto offsets = [&](int bk, int64_t* off) {
        const dev::BgsBlock& B = g.blk[bk];
        int cnt[256] = {0};
        for (int q = 0; q < BGS_ROWS; ++q)
            for (int t = 0; t < (int)((g.meta[(size_t)bk * BGS_ROWS + q] >> 16) & 0xff); ++t) ++cnt[t];
        off[0] = B.base;
        for (int t = 0; t < B.width; ++t) off[t + 1] = off[t] + cnt[t];
    };
    int64_t off[257];
    // r = b - A x with the values at the start of the sweep, every row before any changes
    for (int bk = 0; bk < g.nblk; ++bk) {
        const dev::BgsBlock& B = g.blk[bk];
        const int r0 = bk * BGS_ROWS;
        offsets(bk, off);
        for (int q = 0; q < BGS_ROWS; ++q) {
            const uint32_t mt = g.meta[(size_t)bk * BGS_ROWS + q];
            if ((mt >> 24) == 0xff) continue;
            const int i = r0 + (int)(mt >> 24), nin = mt & 0xff, len = (mt >> 16) & 0xff;
            double acc = 0;
            for (int t = 0; t < len; ++t) {
                const int64_t e = off[t] + q;
                const int j = t < nin ? r0 + g.code[e] : (g.c16 ? B.cbase + g.code[e] : g.code[e]);
                acc += g.val[e] * x[j];
            }
            r[i] = b[i] - acc;
        }
    }
    double u[BGS_ROWS], w[BGS_ROWS];
    for (int bk = 0; bk < g.nblk; ++bk) {
        const dev::BgsBlock& B = g.blk[bk];
        const int r0 = bk * BGS_ROWS;
        const int ncol = (B.info >> 8) & 0xff;
        offsets(bk, off);
        std::fill(u, u + BGS_ROWS, 0.0);   // by position in the block
        std::fill(w, w + BGS_ROWS, 0.0);
        auto inside = [&](int q, int nin, const double* z) {
            double s = 0;
            for (int t = 0; t < nin; ++t) {
                const int64_t e = off[t] + q;
                s += g.val[e] * z[g.code[e]];
            }
            return s;
        };
        for (int c = 0; c < ncol; ++c)
            for (int q = 0; q < BGS_ROWS; ++q) {
                const uint32_t mt = g.meta[(size_t)bk * BGS_ROWS + q];
                if ((mt >> 24) == 0xff || (int)((mt >> 8) & 0xff) != c) continue;
                const int p = mt >> 24, i = r0 + p;
                u[p] = (r[i] - inside(q, mt & 0xff, u)) * g.dinv[i];
            }
        for (int c = ncol - 1; c >= 0; --c)
            for (int q = 0; q < BGS_ROWS; ++q) {
                const uint32_t mt = g.meta[(size_t)bk * BGS_ROWS + q];
                if ((mt >> 24) == 0xff || (int)((mt >> 8) & 0xff) != c) continue;
                const int p = mt >> 24, i = r0 + p;
                w[p] = (g.mid[i] * u[p] - inside(q, mt & 0xff, w)) * g.dinv[i];
            }
        for (int p = 0; p < BGS_ROWS && r0 + p < g.n; ++p) x[r0 + p] += w[p];
    }
}

}  // namespace amge
