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
Csr from_triplets(int32_t nr, int32_t nc, std::vector<int64_t>& keys, std::vector<double>& vals,
                  bool sum_duplicates);                     // keys = row * nc + col
void drop_small(Csr& A, double rel);                        // |a_ij| <= rel * max|A| -> removed
std::vector<double> l1_row_sums(const Csr& A);

// Parallel loop over [0, n) in contiguous chunks on up to hardware_concurrency threads.
void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)>& body);

}  // namespace amge
