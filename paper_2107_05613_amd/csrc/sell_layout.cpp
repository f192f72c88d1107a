// Host construction of the sliced-ELL layout of the level matrices.
#include "sell_layout.hpp"

#include <algorithm>
#include <climits>
#include <cstdlib>
#include <numeric>

namespace amge {

// 16-bit column offsets on (default); AMGE_INDEX32=1 keeps 32-bit indices everywhere.
bool compact_indices() {
    const char* e = getenv("AMGE_INDEX32");   // read per set-up call
    return !(e && *e && *e != '0');
}

bool device_layouts() {
    const char* e = getenv("AMGE_HOST_LAYOUT");   // read per set-up call
    return !(e && *e && *e != '0');
}

HostSell sell_rows(const Csr& A, int K, const std::vector<int>* lead) {
    if (K < 1 || K > 64 || 64 % K) fail(AMGE_ERR_ARG, "lanes per row must divide 64");
    const int R = 64 / K;
    HostSell h;
    h.K = K;
    h.nslices = (A.nrows + R - 1) / R;
    h.srow.assign((size_t)h.nslices * R, -1);
    const int win = 8 * R;
    auto len = [&](int r) { return A.rowptr[r + 1] - A.rowptr[r]; };
    // rows sorted by decreasing length (stable) inside windows of 8 slices
    const int64_t nwin = (A.nrows + win - 1) / win;
    parallel_for(nwin, [&](int64_t a, int64_t b) {
        std::vector<int> order;
        for (int64_t wi = a; wi < b; ++wi) {
            const int w0 = (int)(wi * win), w1 = std::min(A.nrows, w0 + win);
            order.resize(w1 - w0);
            std::iota(order.begin(), order.end(), w0);
            std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return len(x) > len(y); });
            for (int i = 0; i < w1 - w0; ++i) h.srow[w0 + i] = order[i];
        }
    });
    std::vector<int64_t> width(h.nslices);
    parallel_for(h.nslices, [&](int64_t a, int64_t b) {
        for (int64_t sl = a; sl < b; ++sl) {
            int mx = 0;
            for (int l = 0; l < R; ++l) {
                const int r = h.srow[(size_t)sl * R + l];
                if (r >= 0) mx = std::max(mx, len(r));
            }
            width[sl] = (mx + K - 1) / K;
        }
    });
    h.sptr.assign(h.nslices + 1, 0);
    for (int sl = 0; sl < h.nslices; ++sl) {
        if ((int64_t)h.sptr[sl] + width[sl] * 64 > INT32_MAX) fail(AMGE_ERR_SHAPE, "matrix too large for int32 offsets");
        h.sptr[sl + 1] = h.sptr[sl] + (int)(width[sl] * 64);
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
    return h;
}

HostSell make_sell(const Csr& A, bool incidence, int K, const std::vector<int>* lead) {
    HostSell h = sell_rows(A, K, lead);
    const int R = 64 / K;
    auto len = [&](int r) { return A.rowptr[r + 1] - A.rowptr[r]; };
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
