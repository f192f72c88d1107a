// Host-only driver of the library's C++ set-up code (hierarchy builder, host sparse
// kernels, sliced-ELL layout), built with AddressSanitizer and UndefinedBehaviorSanitizer
// by tests/test_host_sanitizers.py.  Any invalid access, leak or undefined behaviour
// aborts the run; the driver itself checks results against plain references.  The device
// entry points the builder can reach (AMGE_BUILD_DEVICE) are replaced by stubs that
// throw: that flag is not used here.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <random>
#include <vector>

#include "../include/amge.h"
#include "../paper_2107_05613_amd/csrc/common.hpp"
#include "../paper_2107_05613_amd/csrc/sell_layout.hpp"
#include "../paper_2107_05613_amd/csrc/setup_device.hpp"
#include "../paper_2107_05613_amd/csrc/spgemm_device.hpp"

namespace amge {
void kuhn_local_device(const KuhnPlanView&, const double*, int64_t, double*, double*, double*, double*) {
    fail(AMGE_ERR_HIP, "no device in the host-only build");
}
Csr triple_on_device(const Csr&, const Csr&, const Csr&, void*, const amge_opts*) {
    fail(AMGE_ERR_HIP, "no device in the host-only build");
}
}  // namespace amge

using namespace amge;

static int failures = 0;
#define CHECK(c)                                                           \
    do {                                                                   \
        if (!(c)) {                                                        \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++failures;                                                    \
        }                                                                  \
    } while (0)

static Csr from_view(const amge_csr& v) { return csr_from_view(v); }

// y = A x by the definition
static std::vector<double> spmv(const Csr& A, const std::vector<double>& x) {
    std::vector<double> y(A.nrows, 0.0);
    for (int i = 0; i < A.nrows; ++i)
        for (int k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) y[i] += A.val[k] * x[A.col[k]];
    return y;
}

static double maxdiff(const std::vector<double>& a, const std::vector<double>& b) {
    double m = 0, s = 0;
    for (size_t i = 0; i < a.size(); ++i) {
        m = std::max(m, std::fabs(a[i] - b[i]));
        s = std::max(s, std::fabs(b[i]));
    }
    return m / std::max(s, 1e-300);
}

// the sliced layout read back entry by entry reproduces A
static void check_layout(const Csr& A, int K, bool lead) {
    std::vector<int> ld;
    if (lead)
        for (int i = 0; i < A.nrows; ++i) ld.push_back((A.rowptr[i + 1] - A.rowptr[i]) / 2);
    HostSell h = make_sell(A, false, K, lead ? &ld : nullptr);
    const int R = 64 / K;
    std::vector<double> x(A.ncols), y(A.nrows, 0.0);
    for (int j = 0; j < A.ncols; ++j) x[j] = std::sin(0.37 * j + 1.0);
    for (int sl = 0; sl < h.nslices; ++sl)
        for (int rr = 0; rr < R; ++rr) {
            const int r = h.srow[(size_t)sl * R + rr];
            if (r < 0) continue;
            const int w = (h.sptr[sl + 1] - h.sptr[sl]) / 64;
            for (int c = 0; c < w; ++c)
                for (int j = 0; j < K; ++j) {
                    const size_t idx = (size_t)h.sptr[sl] + (size_t)c * 64 + rr * K + j;
                    const int col = h.compact ? h.cbase[sl] + h.c16[idx] : h.ci[idx];
                    y[r] += h.val[idx] * x[col];
                }
        }
    CHECK(maxdiff(y, spmv(A, x)) < 1e-13);
    HostSell rows = sell_rows(A, K, lead ? &ld : nullptr);
    CHECK(rows.srow == h.srow && rows.sptr == h.sptr && rows.lead == h.lead);
}

int main() {
    std::mt19937_64 rng(7);
    std::uniform_real_distribution<double> U(-2.0, 2.0);
    int built = 0;
    for (int kind : {(int)AMGE_CURL, (int)AMGE_DIV})
        for (int flags : {0, (int)AMGE_BUILD_ESSENTIAL, (int)AMGE_BUILD_COEFFICIENT,
                          (int)(AMGE_BUILD_ESSENTIAL | AMGE_BUILD_COEFFICIENT)}) {
            const int n = 8, L = 3;
            std::vector<double> a(n * n * n), b(n * n * n);
            for (auto& v : a) v = std::pow(10.0, U(rng));
            for (auto& v : b) v = std::pow(10.0, U(rng));
            amge_problem* p = nullptr;
            CHECK(amge_kuhn_build(kind, n, L, a.data(), b.data(), flags, &p) == AMGE_OK);
            if (!p) continue;
            const int nl = amge_problem_nlevels(p);
            CHECK(nl == L);
            std::vector<amge_level> lv(nl);
            CHECK(amge_problem_levels(p, lv.data()) == AMGE_OK);
            for (int k = 0; k + 1 < nl; ++k) {
                const Csr A = from_view(lv[k].A), P = from_view(lv[k].P), Ac = from_view(lv[k + 1].A);
                // Galerkin: A_{k+1} = P^T A P, checked on a vector
                std::vector<double> x(P.ncols);
                for (auto& v : x) v = U(rng);
                const std::vector<double> y = spmv(transpose(P), spmv(A, spmv(P, x)));
                CHECK(maxdiff(spmv(Ac, x), y) < 1e-11);
                const Csr G = spgemm(transpose(P), spgemm(A, P));
                CHECK(maxdiff(spmv(G, x), y) < 1e-12);
                for (int K : {1, 4, 16}) check_layout(A, K, K == 4);
            }
            amge_problem_free(p);
            ++built;
        }
    // argument errors leave nothing behind
    {
        std::vector<double> one(27, 1.0), neg(27, -1.0);
        amge_problem* p = nullptr;
        CHECK(amge_kuhn_build(AMGE_CURL, 3, 2, one.data(), one.data(), 0, &p) != AMGE_OK);
        CHECK(amge_kuhn_build(AMGE_CURL, 3, 1, neg.data(), one.data(), 0, &p) != AMGE_OK);
        CHECK(amge_kuhn_build(AMGE_DIV, 3, 1, one.data(), one.data(), 64, &p) != AMGE_OK);
        CHECK(amge_kuhn_build(7, 3, 1, one.data(), one.data(), 0, &p) != AMGE_OK);
    }
    // triplet assembly (summed and first-kept) against a map, large enough for the
    // parallel path
    for (bool sum : {true, false}) {
        const int nr = 3000, nc = 2000;
        std::vector<int64_t> keys;
        std::vector<double> vals;
        std::map<int64_t, double> ref;
        std::uniform_int_distribution<int> R(0, nr - 1), Cd(0, nc - 1);
        for (int t = 0; t < 200000; ++t) {
            const int64_t k = (int64_t)R(rng) * nc + Cd(rng);
            const double v = sum ? U(rng) : std::floor(k * 0.5);
            keys.push_back(k);
            vals.push_back(v);
            if (sum) ref[k] += v;
            else ref.emplace(k, v);
        }
        const Csr A = from_triplets(nr, nc, keys, vals, sum);
        CHECK((size_t)A.nnz() == ref.size());
        auto it = ref.begin();
        for (int i = 0; i < nr; ++i)
            for (int q = A.rowptr[i]; q < A.rowptr[i + 1]; ++q, ++it) {
                CHECK(it->first == (int64_t)i * nc + A.col[q]);
                CHECK(std::fabs(it->second - A.val[q]) <= 1e-12 * (1 + std::fabs(it->second)));
            }
    }
    // parallel sort
    {
        std::vector<int64_t> v(300000);
        for (auto& x : v) x = (int64_t)(rng() % 1000003);
        std::vector<int64_t> w = v;
        psort(v);
        std::sort(w.begin(), w.end());
        CHECK(v == w);
    }
    printf("host driver: %d hierarchies built, %d failures\n", built, failures);
    return failures ? 1 : 0;
}
