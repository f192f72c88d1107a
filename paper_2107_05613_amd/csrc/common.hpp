// Shared host-side definitions: status/error reporting, host CSR, parallel loops.
#pragma once

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <functional>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "../../include/amge.h"

namespace amge {

// Exception carrying an amge_status; converted to a return code at the ABI.
struct Error : std::runtime_error {
    amge_status code;
    Error(amge_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(amge_status c, const std::string& m) { throw Error(c, m); }

void set_last_error(const std::string& m);

// Host CSR matrix (FP64 values, int32 indices), sorted columns per row.
struct Csr {
    int32_t nrows = 0, ncols = 0;
    std::vector<int32_t> rowptr{0}, col;
    std::vector<double> val;
    int64_t nnz() const { return (int64_t)col.size(); }
    amge_csr view() const {
        amge_csr v;
        v.nrows = nrows; v.ncols = ncols; v.nnz = nnz();
        v.rowptr = rowptr.data(); v.col = col.data(); v.val = val.data();
        return v;
    }
};

Csr csr_from_view(const amge_csr& v);
Csr transpose(const Csr& A);
Csr spgemm(const Csr& A, const Csr& B);                     // A * B
Csr from_triplets(int32_t nr, int32_t nc, const int64_t* keys, const double* vals, int64_t m,
                  bool sum_duplicates);                     // keys = row * nc + col
inline Csr from_triplets(int32_t nr, int32_t nc, const std::vector<int64_t>& keys, const std::vector<double>& vals,
                         bool sum_duplicates) {
    return from_triplets(nr, nc, keys.data(), vals.data(), (int64_t)keys.size(), sum_duplicates);
}
void drop_small(Csr& A, double rel);                        // |a_ij| <= rel * max|A| -> removed
std::vector<double> l1_row_sums(const Csr& A);

// Parallel loop over [0, n) in contiguous chunks on up to hardware_concurrency threads.
void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)>& body);

// Worker threads for the host loops (at most 16).
int host_threads();

// fn(0) .. fn(ntasks - 1), each on its own thread; exceptions as in parallel_for.
void parallel_tasks(int ntasks, const std::function<void(int)>& fn);

// Sort of v by cmp: chunks sorted on their own threads, then merged pairwise (each round
// in parallel).  The result is the sorted sequence; equal elements keep no particular
// order, so use it where equal elements are indistinguishable.
template <class T, class Cmp = std::less<T>>
void psort(std::vector<T>& v, Cmp cmp = Cmp()) {
    const size_t n = v.size();
    const int nt = host_threads();
    if (n < (size_t)1 << 16 || nt == 1) {
        std::sort(v.begin(), v.end(), cmp);
        return;
    }
    std::vector<size_t> cut(nt + 1);
    for (int t = 0; t <= nt; ++t) cut[t] = n * t / nt;
    parallel_tasks(nt, [&](int t) { std::sort(v.begin() + cut[t], v.begin() + cut[t + 1], cmp); });
    std::vector<T> buf(n);
    std::vector<T>*src = &v, *dst = &buf;
    for (size_t width = 1; width < (size_t)nt; width *= 2) {
        const int pairs = (int)((nt + 2 * width - 1) / (2 * width));
        parallel_tasks(pairs, [&](int q) {
            const size_t a = cut[std::min((size_t)nt, 2 * width * q)];
            const size_t m = cut[std::min((size_t)nt, 2 * width * q + width)];
            const size_t b = cut[std::min((size_t)nt, 2 * width * q + 2 * width)];
            std::merge(src->begin() + a, src->begin() + m, src->begin() + m, src->begin() + b, dst->begin() + a, cmp);
        });
        std::swap(src, dst);
    }
    if (src != &v) v.swap(*src);
}

}  // namespace amge
