// Host construction of the sliced-ELL layout of the level matrices.
#include "sell_layout.hpp"

#include <algorithm>
#include <climits>
#include <cstdlib>
#include <numeric>

namespace amge {

// 16-bit column offsets on (default); AMGE_INDEX32=1 keeps 32-bit indices everywhere.
bool compact_indices() {
    static int v = -1;
    if (v < 0) {
        const char* e = getenv("AMGE_INDEX32");
        v = (e && *e && *e != '0') ? 0 : 1;
    }
    return v == 1;
}

HostSell make_sell(const Csr& A, bool incidence, int K, const std::vector<int>* lead) {
    const int R = 64 / K;
    HostSell h;
    h.K = K;
    h.nslices = (A.nrows + R - 1) / R;
    h.srow.assign((size_t)h.nslices * R, -1);
    const int win = 8 * R;
    std::vector<int> order;
    auto len = [&](int r) { return A.rowptr[r + 1] - A.rowptr[r]; };
    for (int w0 = 0; w0 < A.nrows; w0 += win) {
        int w1 = std::min(A.nrows, w0 + win);
        order.resize(w1 - w0);
        std::iota(order.begin(), order.end(), w0);
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return len(a) > len(b); });
        for (int i = 0; i < w1 - w0; ++i) h.srow[w0 + i] = order[i];
    }
    h.sptr.assign(h.nslices + 1, 0);
    for (int sl = 0; sl < h.nslices; ++sl) {
        int mx = 0;
        for (int l = 0; l < R; ++l) {
            int r = h.srow[(size_t)sl * R + l];
            if (r >= 0) mx = std::max(mx, len(r));
        }
        int64_t width = (mx + K - 1) / K;
        if ((int64_t)h.sptr[sl] + width * 64 > INT32_MAX) fail(AMGE_ERR_SHAPE, "matrix too large for int32 offsets");
        h.sptr[sl + 1] = h.sptr[sl] + (int)(width * 64);
    }
    if (lead) {
        if ((int)lead->size() != A.nrows) fail(AMGE_ERR_SHAPE, "split counts: one per row needed");
        h.lead.assign(h.srow.size(), 0);
        for (size_t i = 0; i < h.srow.size(); ++i) {
            const int r = h.srow[i];
            if (r < 0) continue;
            const int c = (*lead)[r];
            if (c < 0 || c > len(r) || c > 65535) fail(AMGE_ERR_SHAPE, "split count out of range");
            h.lead[i] = (uint16_t)c;
        }
    }
    const size_t stored = h.sptr[h.nslices];
    if (incidence) h.ent.assign(stored, 0xffffffffu);
    else {
        h.ci.assign(stored, 0);
        h.val.assign(stored, 0.0);
    }
    for (int sl = 0; sl < h.nslices; ++sl)
        for (int rr = 0; rr < R; ++rr) {
            int r = h.srow[(size_t)sl * R + rr];
            if (r < 0) continue;
            for (int t = 0; t < len(r); ++t) {
                size_t idx = (size_t)h.sptr[sl] + (size_t)(t / K) * 64 + rr * K + t % K;
                int c = A.col[A.rowptr[r] + t];
                double v = A.val[A.rowptr[r] + t];
                if (incidence) {
                    if (v != 1.0 && v != -1.0) fail(AMGE_ERR_ARG, "derivative matrix entries must be +-1");
                    h.ent[idx] = (uint32_t)c | (v < 0 ? 0x80000000u : 0u);
                } else {
                    h.ci[idx] = c;
                    h.val[idx] = v;
                }
            }
        }
    if (!incidence) {
        h.cbase.assign(h.nslices, 0);
        bool fits = true;
        for (int sl = 0; sl < h.nslices && fits; ++sl) {
            int lo = INT32_MAX, hi = -1;
            for (int rr = 0; rr < R; ++rr) {
                int r = h.srow[(size_t)sl * R + rr];
                if (r < 0) continue;
                for (int t = A.rowptr[r]; t < A.rowptr[r + 1]; ++t) {
                    lo = std::min(lo, A.col[t]);
                    hi = std::max(hi, A.col[t]);
                }
            }
            if (hi < 0) continue;
            h.cbase[sl] = lo;
            fits = hi - lo <= 65535;
        }
        if (fits) {
            h.compact = true;
            h.c16.assign(stored, 0);
            for (int sl = 0; sl < h.nslices; ++sl)
                for (int rr = 0; rr < R; ++rr) {
                    int r = h.srow[(size_t)sl * R + rr];
                    if (r < 0) continue;
                    for (int t = 0; t < len(r); ++t) {
                        size_t idx = (size_t)h.sptr[sl] + (size_t)(t / K) * 64 + rr * K + t % K;
                        h.c16[idx] = (uint16_t)(A.col[A.rowptr[r] + t] - h.cbase[sl]);
                    }
                }
        }
    }
    return h;
}

}  // namespace amge
