// Launch shape and block mapping shared by the device kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

namespace amge {
namespace dev {

constexpr int BLOCK = 256;
constexpr int WAVES = BLOCK / 64;   // slices per block
constexpr int NRED = 1024;          // blocks (and partial sums) of the streaming reductions
constexpr int NXCD = 8;

// Blocks are dispatched round-robin over the XCDs; give XCD k a contiguous range.
__device__ __forceinline__ int xcd_block(int b, int G) {
    const int xcd = b % NXCD, idx = b / NXCD;
    const int per = G / NXCD, rem = G % NXCD;
    return xcd * per + min(xcd, rem) + idx;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace dev
}  // namespace amge
