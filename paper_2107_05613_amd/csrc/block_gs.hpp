// l1-scaled symmetric block Gauss-Seidel smoother: host layout, device data, launches.
#pragma once

#include <vector>

#include "common.hpp"
#include "hierarchy.hpp"

namespace amge {

constexpr int BGS_ROWS = 64;   // rows per block: one wave

// Host form of the layout of DBgs (also the host sweep of a folded coarse tail).
struct BgsHost {
    int n = 0, nblk = 0, nin = 0, ninmax = 0;
    bool c16 = false;
    int64_t nnz = 0, nnz_in = 0;
    std::vector<dev::BgsBlock> blk;
    std::vector<uint32_t> meta;     // per lane (block-major): inside entries | colour << 8 |
                                    // length << 16 | position of its row << 24 (0xff: none);
                                    // colours over the couplings inside the row's block
    std::vector<int32_t> code;      // inside: position in the block; outside: column
                                    // (C16: offset from the block's base column)
    std::vector<double> val, dinv, mid;
};

// Blocks of 64 consecutive rows; colours first fit in increasing row order over the
// nonzero couplings inside a block; d_i = a_ii + sum of |a_ij| outside the block.
// Fails with AMGE_ERR_NOT_SPD if some d_i or a_ii is not positive.
BgsHost bgs_layout(const Csr& A);

// Device data of A's block sweeps (both value precisions).
void build_bgs(amge_hierarchy* H, const Csr& A, DBgs& g, hipStream_t s);

// One sweep y = x + Mb^{-1} (D + 2 D_l1) Mf^{-1} (b - A x); zero: x = 0 (x unused).
template <class T>
void bgs_launch(const DBgs& g, bool zero, const T* x, const T* b, T* y, hipStream_t s, const int* stop);

// y = b - A x on the block layout (values FP64 with FP32 vectors when v64 is set).
template <class T>
void bgs_resid_launch(const DBgs& g, bool v64, const T* x, const T* b, T* y, hipStream_t s, const int* stop);

// Batched sweep and residual on the first W (a power of two) of the NC columns of
// row-major n x NC blocks; launched solo, or recorded while a launch recorder is
// installed (grouped launches of the serving engine).
template <class T>
void bgs_mm_launch(const DBgs& g, bool zero, int W, int NC, const T* X, const T* B, T* Y, const int* stop,
                   hipStream_t s);
template <class T>
void bgs_resid_mm_launch(const DBgs& g, bool v64, int W, int NC, const T* X, const T* B, T* Y, const int* stop,
                         hipStream_t s);

// Algorithmic bytes of one sweep, and of one residual (vbytes: value size; cols: columns
// of the vector blocks, the matrix read once for all of them).
double bgs_bytes(const DBgs& g, bool zero, int vbytes, int cols = 1);
double bgs_resid_bytes(const DBgs& g, int vbytes, int xbytes, int cols = 1);

// One host sweep in FP64 on x in place (tmp: scratch of n values).
void host_bgs_sweep(const BgsHost& g, const double* b, double* x, std::vector<double>& tmp);

}  // namespace amge
