// l1-scaled symmetric block Gauss-Seidel smoother on the batched path (n x NC blocks):
// launches of the sweep and residual bodies of kernels_bgs.hpp, solo or recorded for
// grouped launches.  Included by one translation unit per vector type BGS_T, so that the
// kernel instances of the two types compile in parallel.
#ifndef BGS_T
#error "define BGS_T (float or double) before including this file"
#endif
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "block_gs.hpp"
#include "kernels_bgs.hpp"

namespace amge {

namespace {

template <class T> const T* vals(const DBgs& g);
template <> const double* vals<double>(const DBgs& g) { return g.v64; }
template <> const float* vals<float>(const DBgs& g) { return g.v32; }
template <class T> const T* dinvs(const DBgs& g);
template <> const double* dinvs<double>(const DBgs& g) { return g.dinv64; }
template <> const float* dinvs<float>(const DBgs& g) { return g.dinv32; }
template <class T> const T* mids(const DBgs& g);
template <> const double* mids<double>(const DBgs& g) { return g.mid64; }
template <> const float* mids<float>(const DBgs& g) { return g.mid32; }

}  // namespace

namespace {

// Shape of the batched launches for W active columns (a power of two): V columns per
// lane, P lanes per row.  32 bytes per lane (8 FP32 or 4 FP64 columns), or one column per
// wave when fewer columns are active.  FP32 with 32 columns or more: the four waves of a
// workgroup share a block (P = 4) and a row's four 32-byte groups sit in neighbouring
// lanes, so each vector access of a wave touches 16 cache lines where one row per lane
// touches 64.  FP64 keeps one row per lane at every width: with four lanes per row its
// batched V-cycles differed between widths at the rounding level, from run to run.
template <class T, class F>
void bgs_shape(int W, F&& f) {
    constexpr int S = (int)sizeof(T);
    using one = std::integral_constant<int, 1>;
    using four = std::integral_constant<int, 4>;
    using vec = std::integral_constant<int, 32 / S>;
    if constexpr (S == 4) {
        if (W * S >= 128) {
            f(vec{}, four{});
            return;
        }
    }
    if (W * S >= 32) f(vec{}, one{});
    else f(one{}, one{});
}

template <class T, int V, int P, bool C16, bool ZERO, int NIN>
void go_mm(const DBgs& g, int W, int NC, const T* X, const T* B, T* Y, const int* stop, hipStream_t s) {
    const int L = W / (P * V);   // groups of P x V columns
    const int64_t waves = (int64_t)g.nblk * L * P;
    launch<dev::BgsMM<T, V, P, C16, ZERO, NIN>>((unsigned)((waves + dev::WAVES - 1) / dev::WAVES), s, g.nblk, g.n,
                                                L, NC, (const dev::BgsBlock*)g.blk, (const uint32_t*)g.meta,
                                                (const int*)g.ci, (const uint16_t*)g.c16, vals<T>(g), dinvs<T>(g),
                                                mids<T>(g), X, B, Y, stop);
}

template <class T, int V, int P, bool C16, bool ZERO>
void go_mm_nin(const DBgs& g, int W, int NC, const T* X, const T* B, T* Y, const int* stop, hipStream_t s) {
    // register bounds of the batched bodies: 8, 16, 32 or 64 (fewer instances)
    if (g.nin <= 8) go_mm<T, V, P, C16, ZERO, 8>(g, W, NC, X, B, Y, stop, s);
    else if (g.nin <= 16) go_mm<T, V, P, C16, ZERO, 16>(g, W, NC, X, B, Y, stop, s);
    else if (g.nin <= 32) go_mm<T, V, P, C16, ZERO, 32>(g, W, NC, X, B, Y, stop, s);
    else go_mm<T, V, P, C16, ZERO, 64>(g, W, NC, X, B, Y, stop, s);
}

template <class T, int V, int P>
void go_mm_v(const DBgs& g, bool zero, int W, int NC, const T* X, const T* B, T* Y, const int* stop,
             hipStream_t s) {
    const bool c16 = g.c16 != nullptr;
    if (zero) {
        if (c16) go_mm_nin<T, V, P, true, true>(g, W, NC, X, B, Y, stop, s);
        else go_mm_nin<T, V, P, false, true>(g, W, NC, X, B, Y, stop, s);
    } else {
        if (c16) go_mm_nin<T, V, P, true, false>(g, W, NC, X, B, Y, stop, s);
        else go_mm_nin<T, V, P, false, false>(g, W, NC, X, B, Y, stop, s);
    }
}

template <class T, int V, int P, class TV>
void go_resid_mm(const DBgs& g, const TV* av, int W, int NC, const T* X, const T* B, T* Y, const int* stop,
                 hipStream_t s) {
    const int L = W / (P * V);   // groups of P x V columns
    const int64_t waves = (int64_t)g.nblk * L * P;
    const unsigned grid = (unsigned)((waves + dev::WAVES - 1) / dev::WAVES);
    if (g.c16)
        launch<dev::BgsResidMM<T, V, P, true, TV>>(grid, s, g.nblk, g.n, L, NC, (const dev::BgsBlock*)g.blk,
                                                   (const uint32_t*)g.meta, (const int*)g.ci, (const uint16_t*)g.c16,
                                                   av, X, B, Y, stop);
    else
        launch<dev::BgsResidMM<T, V, P, false, TV>>(grid, s, g.nblk, g.n, L, NC, (const dev::BgsBlock*)g.blk,
                                                    (const uint32_t*)g.meta, (const int*)g.ci, (const uint16_t*)g.c16,
                                                    av, X, B, Y, stop);
}

template <class T, class TV>
void go_resid_mm_v(const DBgs& g, const TV* av, int W, int NC, const T* X, const T* B, T* Y, const int* stop,
                   hipStream_t s) {
    bgs_shape<T>(W, [&](auto v, auto p) {
        go_resid_mm<T, decltype(v)::value, decltype(p)::value, TV>(g, av, W, NC, X, B, Y, stop, s);
    });
}

}  // namespace

template <class T>
void bgs_mm_launch(const DBgs& g, bool zero, int W, int NC, const T* X, const T* B, T* Y, const int* stop,
                   hipStream_t s) {
    if (g.nblk == 0) return;
    bgs_shape<T>(W, [&](auto v, auto p) {
        go_mm_v<T, decltype(v)::value, decltype(p)::value>(g, zero, W, NC, X, B, Y, stop, s);
    });
}

template <class T>
void bgs_resid_mm_launch(const DBgs& g, bool v64, int W, int NC, const T* X, const T* B, T* Y, const int* stop,
                         hipStream_t s) {
    if (g.nblk == 0) return;
    if (v64 && !std::is_same<T, double>::value) go_resid_mm_v<T, double>(g, g.v64, W, NC, X, B, Y, stop, s);
    else go_resid_mm_v<T, T>(g, vals<T>(g), W, NC, X, B, Y, stop, s);
}

template void bgs_mm_launch<BGS_T>(const DBgs&, bool, int, int, const BGS_T*, const BGS_T*, BGS_T*, const int*,
                                   hipStream_t);
template void bgs_resid_mm_launch<BGS_T>(const DBgs&, bool, int, int, const BGS_T*, const BGS_T*, BGS_T*,
                                         const int*, hipStream_t);

}  // namespace amge
