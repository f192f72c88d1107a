// Host construction of the sliced-ELL layout of the level matrices.
#pragma once

#include <cstdint>
#include <vector>

#include "common.hpp"

namespace amge {

// Host conversion CSR -> sliced ELL with K lanes per row.  Rows are sorted by
// decreasing length inside windows of 8 slices; each slice is as wide as its longest
// row (rounded up to a multiple of K).
struct HostSell {
    int K = 1, nslices = 0;
    std::vector<int> sptr, srow, ci;
    std::vector<uint32_t> ent;
    std::vector<double> val;
    // compact column indices: per-slice base + 16-bit offsets, used when every slice's
    // columns fit in 65536 consecutive indices (padding entries: offset 0)
    bool compact = false;
    std::vector<int> cbase;
    std::vector<uint16_t> c16;
    // split rows (lead != null): per slot, how many leading entries of its row read the
    // first operand (the others read the second one)
    std::vector<uint16_t> lead;
};

// The row part of the layout, O(rows): K, nslices, the slot -> row map srow, the slice
// offsets sptr and (lead != null) the per-slot split counts; no entry arrays.
HostSell sell_rows(const Csr& A, int K, const std::vector<int>* lead = nullptr);

// Entry of the sliced ELL: entry t of the row in slot rr of slice sl is stored at
// sptr[sl] + (t / K) * 64 + rr * K + t % K; padding holds column 0 and value 0
// (incidence: the word 0xffffffff).

// Sliced ELL of A with K lanes per row (K | 64): sell_rows, then the entry arrays.  incidence: entries must be +-1 and are
// stored index-only with the sign in bit 31.  lead (optional, one count per row): the
// first lead[r] entries of row r act on a first operand and the rest on a second one
// of the same length (both index the same column range, A.ncols).
HostSell make_sell(const Csr& A, bool incidence, int K, const std::vector<int>* lead = nullptr);

// Whether compact (16-bit) column offsets may be used: on unless AMGE_INDEX32 is set.
bool compact_indices();

// Whether set-up fills the entry arrays on the device from a staged copy of the CSR
// matrix (default) or builds the whole layout on the host and uploads it
// (AMGE_HOST_LAYOUT=1).  Both give the same arrays.
bool device_layouts();

}  // namespace amge
