// l1-scaled symmetric block Gauss-Seidel smoother on the batched path (n x NC blocks):
// launches of the sweep and residual bodies of kernels_bgs.hpp, solo or recorded for
// grouped launches.  Included by one translation unit per launch shape (BGS_SHAPE_T,
// BGS_SHAPE_V, BGS_SHAPE_P defined: the kernel instances of that shape), so that the
// shapes compile in parallel, and once without them (the launchers, which pick a shape
// from the active width).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "block_gs.hpp"

namespace amge {

// The kernel launches of one shape (V columns per lane, P lanes per row): the sweep
// (zero: from x = 0) and the residual (v64: FP64 values with FP32 blocks).
template <class T, int V, int P>
void bgs_mm_shape(const DBgs& g, bool zero, int W, int NC, const T* X, const T* B, T* Y, const int* stop,
                  hipStream_t s);
template <class T, int V, int P>
void bgs_resid_mm_shape(const DBgs& g, bool v64, int W, int NC, const T* X, const T* B, T* Y, const int* stop,
                        hipStream_t s);

#ifdef BGS_SHAPE_T

}  // namespace amge

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

}  // namespace

template <class T, int V, int P>
void bgs_mm_shape(const DBgs& g, bool zero, int W, int NC, const T* X, const T* B, T* Y, const int* stop,
                  hipStream_t s) {
    go_mm_v<T, V, P>(g, zero, W, NC, X, B, Y, stop, s);
}

template <class T, int V, int P>
void bgs_resid_mm_shape(const DBgs& g, bool v64, int W, int NC, const T* X, const T* B, T* Y, const int* stop,
                        hipStream_t s) {
    if constexpr (std::is_same<T, double>::value) go_resid_mm<T, V, P, T>(g, vals<T>(g), W, NC, X, B, Y, stop, s);
    else if (v64) go_resid_mm<T, V, P, double>(g, g.v64, W, NC, X, B, Y, stop, s);
    else go_resid_mm<T, V, P, T>(g, vals<T>(g), W, NC, X, B, Y, stop, s);
}

template void bgs_mm_shape<BGS_SHAPE_T, BGS_SHAPE_V, BGS_SHAPE_P>(const DBgs&, bool, int, int, const BGS_SHAPE_T*,
                                                                 const BGS_SHAPE_T*, BGS_SHAPE_T*, const int*,
                                                                 hipStream_t);
template void bgs_resid_mm_shape<BGS_SHAPE_T, BGS_SHAPE_V, BGS_SHAPE_P>(const DBgs&, bool, int, int,
                                                                       const BGS_SHAPE_T*, const BGS_SHAPE_T*,
                                                                       BGS_SHAPE_T*, const int*, hipStream_t);

#else

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

}  // namespace

template <class T>
void bgs_mm_launch(const DBgs& g, bool zero, int W, int NC, const T* X, const T* B, T* Y, const int* stop,
                   hipStream_t s) {
    if (g.nblk == 0) return;
    bgs_shape<T>(W, [&](auto v, auto p) {
        bgs_mm_shape<T, decltype(v)::value, decltype(p)::value>(g, zero, W, NC, X, B, Y, stop, s);
    });
}

template <class T>
void bgs_resid_mm_launch(const DBgs& g, bool v64, int W, int NC, const T* X, const T* B, T* Y, const int* stop,
                         hipStream_t s) {
    if (g.nblk == 0) return;
    bgs_shape<T>(W, [&](auto v, auto p) {
        bgs_resid_mm_shape<T, decltype(v)::value, decltype(p)::value>(g, v64, W, NC, X, B, Y, stop, s);
    });
}

template void bgs_mm_launch<float>(const DBgs&, bool, int, int, const float*, const float*, float*, const int*,
                                   hipStream_t);
template void bgs_mm_launch<double>(const DBgs&, bool, int, int, const double*, const double*, double*, const int*,
                                    hipStream_t);
template void bgs_resid_mm_launch<float>(const DBgs&, bool, int, int, const float*, const float*, float*, const int*,
                                         hipStream_t);
template void bgs_resid_mm_launch<double>(const DBgs&, bool, int, int, const double*, const double*, double*,
                                          const int*, hipStream_t);

#endif

}  // namespace amge
