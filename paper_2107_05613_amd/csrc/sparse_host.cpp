// Host sparse kernels used at set-up: transpose, sparse product, triplet assembly.
#include <exception>
#include <atomic>
#include <climits>
#include <cmath>
#include <memory>
#include <numeric>

#include "common.hpp"

namespace amge {

static thread_local std::string g_last_error;

void set_last_error(const std::string& m) { g_last_error = m; }

}  // namespace amge

extern "C" const char* amge_last_error(void) { return amge::g_last_error.c_str(); }

namespace amge {

int host_threads() { return (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency())); }

void parallel_tasks(int ntasks, const std::function<void(int)>& fn) {
    if (ntasks <= 0) return;
    if (ntasks == 1) {
        fn(0);
        return;
    }
    std::vector<std::thread> th;
    std::vector<std::exception_ptr> err(ntasks);
    for (int t = 0; t < ntasks; ++t)
        th.emplace_back([&fn, &err, t] {
            try {
                fn(t);
            } catch (...) {
                err[t] = std::current_exception();
            }
        });
    for (auto& t : th) t.join();
    for (auto& e : err)
        if (e) std::rethrow_exception(e);
}

void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)>& body) {
    if (n <= 0) return;
    int nt = host_threads();
    if (n < 4096 || nt == 1) {
        body(0, n);
        return;
    }
    // an exception in a worker is carried to the caller (an escaping one would end the
    // process); the first one, in chunk order, is rethrown after every worker has joined
    std::vector<std::thread> th;
    std::vector<std::exception_ptr> err(nt);
    int64_t chunk = (n + nt - 1) / nt;
    for (int t = 0; t < nt; ++t) {
        int64_t s = t * chunk, e = std::min(n, s + chunk);
        if (s >= e) break;
        th.emplace_back([&body, &err, t, s, e] {
            try {
                body(s, e);
            } catch (...) {
                err[t] = std::current_exception();
            }
        });
    }
    for (auto& t : th) t.join();
    for (auto& e : err)
        if (e) std::rethrow_exception(e);
}

Csr csr_from_view(const amge_csr& v) {
    if (v.nrows < 0 || v.ncols < 0 || v.nnz < 0) fail(AMGE_ERR_ARG, "negative CSR size");
    if (v.nrows > 0 && (!v.rowptr || (v.nnz > 0 && (!v.col || !v.val))))
        fail(AMGE_ERR_ARG, "null CSR array");
    Csr A;
    A.nrows = v.nrows;
    A.ncols = v.ncols;
    A.rowptr.assign(v.rowptr, v.rowptr + v.nrows + 1);
    if (A.rowptr[0] != 0 || A.rowptr[v.nrows] != v.nnz) fail(AMGE_ERR_SHAPE, "CSR rowptr does not span nnz");
    for (int32_t i = 0; i < v.nrows; ++i)
        if (A.rowptr[i + 1] < A.rowptr[i]) fail(AMGE_ERR_SHAPE, "CSR rowptr not monotone");
    A.col.assign(v.col, v.col + v.nnz);
    A.val.assign(v.val, v.val + v.nnz);
    // rows checked in parallel; the first failing chunk's error is reported
    parallel_for(v.nrows, [&](int64_t s, int64_t e) {
        for (int64_t i = s; i < e; ++i)
            for (int32_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) {
                if (A.col[k] < 0 || A.col[k] >= v.ncols) fail(AMGE_ERR_SHAPE, "CSR column index out of range");
                if (k > A.rowptr[i] && A.col[k] <= A.col[k - 1])
                    fail(AMGE_ERR_SHAPE, "CSR columns not sorted/unique");
                if (!std::isfinite(A.val[k])) fail(AMGE_ERR_NONFINITE, "non-finite CSR value");
            }
    });
    return A;
}

Csr transpose(const Csr& A) {
    Csr T;
    T.nrows = A.ncols;
    T.ncols = A.nrows;
    T.rowptr.assign(A.ncols + 1, 0);
    for (int32_t c : A.col) T.rowptr[c + 1]++;
    for (int32_t i = 0; i < A.ncols; ++i) T.rowptr[i + 1] += T.rowptr[i];
    T.col.resize(A.col.size());
    T.val.resize(A.val.size());
    std::vector<int32_t> pos(T.rowptr.begin(), T.rowptr.end() - 1);
    for (int32_t i = 0; i < A.nrows; ++i)       // rows in order -> sorted columns in T
        for (int32_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) {
            int32_t p = pos[A.col[k]]++;
            T.col[p] = i;
            T.val[p] = A.val[k];
        }
    return T;
}

// Row-wise product with a dense accumulator per thread (Gustavson), two passes.
Csr spgemm(const Csr& A, const Csr& B) {
    if (A.ncols != B.nrows) fail(AMGE_ERR_SHAPE, "spgemm: inner dimensions differ");
    Csr C;
    C.nrows = A.nrows;
    C.ncols = B.ncols;
    std::vector<int64_t> cnt(A.nrows + 1, 0);
    parallel_for(A.nrows, [&](int64_t s, int64_t e) {
        std::vector<int32_t> mark(B.ncols, -1);
        for (int64_t i = s; i < e; ++i) {
            int64_t c = 0;
            for (int32_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) {
                int32_t j = A.col[k];
                for (int32_t l = B.rowptr[j]; l < B.rowptr[j + 1]; ++l)
                    if (mark[B.col[l]] != (int32_t)i) { mark[B.col[l]] = (int32_t)i; ++c; }
            }
            cnt[i + 1] = c;
        }
    });
    for (int32_t i = 0; i < A.nrows; ++i) cnt[i + 1] += cnt[i];
    if (cnt[A.nrows] > INT32_MAX) fail(AMGE_ERR_SHAPE, "spgemm: result exceeds int32 nnz");
    C.rowptr.assign(cnt.begin(), cnt.end());
    C.col.resize(cnt[A.nrows]);
    C.val.resize(cnt[A.nrows]);
    parallel_for(A.nrows, [&](int64_t s, int64_t e) {
        std::vector<double> acc(B.ncols, 0.0);
        std::vector<char> used(B.ncols, 0);
        std::vector<int32_t> list;
        for (int64_t i = s; i < e; ++i) {
            list.clear();
            for (int32_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) {
                int32_t j = A.col[k];
                double a = A.val[k];
                for (int32_t l = B.rowptr[j]; l < B.rowptr[j + 1]; ++l) {
                    int32_t c = B.col[l];
                    if (!used[c]) { used[c] = 1; list.push_back(c); }
                    acc[c] += a * B.val[l];
                }
            }
            std::sort(list.begin(), list.end());
            int32_t p = C.rowptr[i];
            for (int32_t c : list) {
                C.col[p] = c;
                C.val[p] = acc[c];
                ++p;
                acc[c] = 0.0;
                used[c] = 0;
            }
        }
    });
    return C;
}

Csr from_triplets(int32_t nr, int32_t nc, const int64_t* keys, const double* vals, int64_t m,
                  bool sum_duplicates) {
    // Stable bucketing by row (a counting sort in parallel: each thread counts the rows of
    // its contiguous chunk of triplets, over the row range the chunk touches; a row's
    // entries from chunk t follow those of chunks < t), then each row sorted by column
    // (stable) and its duplicates merged in triplet order: summed (assembly) or the first
    // kept (overwrite assembly: shared entries agree).
    if (nc <= 0 && m > 0) fail(AMGE_ERR_SHAPE, "triplets for a matrix without columns");
    const int nt = m >= (1 << 16) ? host_threads() : 1;
    std::vector<int64_t> cut(nt + 1);
    for (int t = 0; t <= nt; ++t) cut[t] = m * t / nt;
    std::vector<int64_t> rlo(nt, 0), rhi(nt, -1);
    std::vector<std::vector<int64_t>> cnt(nt);
    parallel_tasks(nt, [&](int t) {
        int64_t lo = INT64_MAX, hi = -1;
        for (int64_t q = cut[t]; q < cut[t + 1]; ++q) {
            const int64_t r = keys[q] / nc;
            if (r < 0 || r >= nr || keys[q] % nc < 0) fail(AMGE_ERR_SHAPE, "triplet outside the matrix");
            lo = std::min(lo, r);
            hi = std::max(hi, r);
        }
        if (hi < 0) return;
        rlo[t] = lo;
        rhi[t] = hi;
        cnt[t].assign(hi - lo + 1, 0);
        for (int64_t q = cut[t]; q < cut[t + 1]; ++q) cnt[t][keys[q] / nc - lo]++;
    });
    std::vector<int64_t> start(nr + 1, 0);
    parallel_for(nr, [&](int64_t s, int64_t e) {
        for (int64_t r = s; r < e; ++r) {
            int64_t c = 0;
            for (int t = 0; t < nt; ++t)
                if (r >= rlo[t] && r <= rhi[t]) c += cnt[t][r - rlo[t]];
            start[r + 1] = c;
        }
    });
    for (int32_t i = 0; i < nr; ++i) start[i + 1] += start[i];
    // counts -> first position of each chunk's entries in each row
    parallel_for(nr, [&](int64_t s, int64_t e) {
        for (int64_t r = s; r < e; ++r) {
            int64_t run = start[r];
            for (int t = 0; t < nt; ++t)
                if (r >= rlo[t] && r <= rhi[t]) {
                    const int64_t c = cnt[t][r - rlo[t]];
                    cnt[t][r - rlo[t]] = run;
                    run += c;
                }
        }
    });
    // every slot is written by the scatter: no initialisation
    std::unique_ptr<int32_t[]> bc(new int32_t[std::max<int64_t>(m, 1)]);
    std::unique_ptr<double[]> bv(new double[std::max<int64_t>(m, 1)]);
    parallel_tasks(nt, [&](int t) {
        for (int64_t q = cut[t]; q < cut[t + 1]; ++q) {
            const int64_t r = keys[q] / nc;
            const int64_t p = cnt[t][r - rlo[t]]++;
            bc[p] = (int32_t)(keys[q] % nc);
            bv[p] = vals[q];
        }
    });
    cnt.clear();
    std::vector<int32_t> rowcnt(nr, 0);
    parallel_for(nr, [&](int64_t s, int64_t e) {
        std::vector<std::pair<int32_t, int64_t>> tmp;
        std::vector<double> v2;
        std::vector<int32_t> c2;
        for (int64_t i = s; i < e; ++i) {
            tmp.clear();
            for (int64_t p = start[i]; p < start[i + 1]; ++p) tmp.emplace_back(bc[p], p);
            std::stable_sort(tmp.begin(), tmp.end(),
                             [](const std::pair<int32_t, int64_t>& a, const std::pair<int32_t, int64_t>& b) {
                                 return a.first < b.first;
                             });
            v2.clear();
            c2.clear();
            for (auto& q : tmp) {
                if (!c2.empty() && c2.back() == q.first) {
                    if (sum_duplicates) v2.back() += bv[q.second];
                    continue;
                }
                c2.push_back(q.first);
                v2.push_back(bv[q.second]);
            }
            for (size_t j = 0; j < c2.size(); ++j) {
                bc[start[i] + j] = c2[j];
                bv[start[i] + j] = v2[j];
            }
            rowcnt[i] = (int32_t)c2.size();
        }
    });
    Csr A;
    A.nrows = nr;
    A.ncols = nc;
    A.rowptr.assign(nr + 1, 0);
    for (int32_t i = 0; i < nr; ++i) A.rowptr[i + 1] = A.rowptr[i] + rowcnt[i];
    A.col.resize(A.rowptr[nr]);
    A.val.resize(A.rowptr[nr]);
    parallel_for(nr, [&](int64_t s, int64_t e) {
        for (int64_t i = s; i < e; ++i)
            for (int32_t j = 0; j < rowcnt[i]; ++j) {
                A.col[A.rowptr[i] + j] = bc[start[i] + j];
                A.val[A.rowptr[i] + j] = bv[start[i] + j];
            }
    });
    return A;
}

void drop_small(Csr& A, double rel) {
    double mx = 0;
    for (double v : A.val) mx = std::max(mx, std::fabs(v));
    double thr = rel * mx;
    Csr B;
    B.nrows = A.nrows;
    B.ncols = A.ncols;
    B.rowptr.assign(A.nrows + 1, 0);
    for (int32_t i = 0; i < A.nrows; ++i) {
        for (int32_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k)
            if (std::fabs(A.val[k]) > thr) {
                B.col.push_back(A.col[k]);
                B.val.push_back(A.val[k]);
            }
        B.rowptr[i + 1] = (int32_t)B.col.size();
    }
    A = std::move(B);
}

std::vector<double> l1_row_sums(const Csr& A) {
    std::vector<double> d(A.nrows, 0.0);
    parallel_for(A.nrows, [&](int64_t s, int64_t e) {
        for (int64_t i = s; i < e; ++i)
            for (int32_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) d[i] += std::fabs(A.val[k]);
    });
    return d;
}

}  // namespace amge
