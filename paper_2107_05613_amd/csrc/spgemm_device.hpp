// Sparse matrix products of set-up on the device: the Galerkin coarse matrices
// P^T (A P) (section 3.2.1) and the auxiliary-space products D^T A, (D^T A) D and P^T A
// of the solver's set-up.  Every product equals the host product (spgemm) bit for bit:
// the same sparsity (every structurally present product, sorted columns) and every
// entry summed in the order of the left factor's row with separately rounded products
// and sums.
#pragma once

#include <utility>

#include "common.hpp"

namespace amge {

// C = A B on the current device (stream: a hipStream_t, null for the default stream;
// opts: its alloc / dealloc hooks, when set, provide the device memory, else hipMalloc).
// A product with a row of more than device_product_max_row() distinct columns runs on
// the host instead (same result); so does every product with AMGE_HOST_PRODUCTS=1.
Csr spgemm_on_device(const Csr& A, const Csr& B, void* stream, const amge_opts* opts = nullptr);

// L (A R), the intermediate kept on the device (Galerkin: P^T (A P)).
Csr triple_on_device(const Csr& L, const Csr& A, const Csr& R, void* stream, const amge_opts* opts = nullptr);

// (X Y, (X Y) Z), the intermediate kept on the device (D^T A and D^T A D).
std::pair<Csr, Csr> chain_on_device(const Csr& X, const Csr& Y, const Csr& Z, void* stream,
                                    const amge_opts* opts = nullptr);

// Largest number of distinct columns in a row that a device product handles.
int device_product_max_row();

// Whether set-up products run on the device (default) or on the host
// (AMGE_HOST_PRODUCTS=1); read per call.
bool device_products();

}  // namespace amge
