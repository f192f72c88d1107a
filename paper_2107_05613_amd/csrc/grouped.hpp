// Solo and grouped launches of the batched kernels.
//
// Every batched kernel body is a device function of a grid object G (its block index and
// block count) and of its operands.  A solo launch runs the body with the hardware grid;
// a grouped launch runs the bodies of several independent operand sets (the same level
// operator of several resident hierarchies) in one launch: block b of the grouped grid
// belongs to the member m with start[m] <= b < start[m + 1] and runs the body with that
// member's operands, block index b - start[m] and block count start[m + 1] - start[m].
// Every member therefore computes exactly what its solo launch computes (the same
// blocks with the same indices), in any grouping.
//
// The host side: launch<Op>(grid, stream, operands...) launches the body of Op solo, or,
// while a LaunchRecorder is installed on the calling thread, appends the launch to it
// instead.  The serving engine records one PCG iteration of each hierarchy of an
// ensemble, merges the records (group_launches) and captures the merged launches as one
// graph.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <vector>

namespace amge {
namespace dev {

struct HwGrid {
    __device__ __forceinline__ unsigned bid() const { return blockIdx.x; }
    __device__ __forceinline__ unsigned nb() const { return gridDim.x; }
};

struct SubGrid {
    unsigned b, n;
    __device__ __forceinline__ unsigned bid() const { return b; }
    __device__ __forceinline__ unsigned nb() const { return n; }
};

// The operands of one launch as a trivially copyable aggregate.
template <class... P> struct ArgPack;
template <> struct ArgPack<> {
    template <class Op, class G, class... D>
    __device__ __forceinline__ void call(G g, D... d) const { Op::run(g, d...); }
};
template <class H, class... R> struct ArgPack<H, R...> {
    H h;
    ArgPack<R...> r;
    template <class Op, class G, class... D>
    __device__ __forceinline__ void call(G g, D... d) const { r.template call<Op>(g, d..., h); }
};

inline ArgPack<> make_argpack() { return {}; }
template <class H, class... R>
ArgPack<H, R...> make_argpack(H h, R... r) { return ArgPack<H, R...>{h, make_argpack(r...)}; }

// Kernel arguments of a grouped launch (passed by value, read with scalar loads).
constexpr int GROUP_ARG_BYTES = 2048;
template <class... P>
struct GroupArgs {
    static constexpr int MAXM_FIT = (int)((GROUP_ARG_BYTES - 4 - 4 * 17) / sizeof(ArgPack<P...>));
    static constexpr int MAXM = MAXM_FIT < 1 ? 1 : (MAXM_FIT > 16 ? 16 : MAXM_FIT);
    int nmem;
    unsigned start[MAXM + 1];   // first block of each member; start[nmem..MAXM] = total
    ArgPack<P...> a[MAXM];
};

template <class Op, class... P>
__global__ void __launch_bounds__(Op::block) k_one(P... a) { Op::run(HwGrid{}, a...); }

template <class Op, class... P>
__global__ void __launch_bounds__(Op::block) k_group(GroupArgs<P...> ga) {
    using GA = GroupArgs<P...>;
    const unsigned b = blockIdx.x;
    int m = 0;   // start[] is nondecreasing: m = number of later members whose range begins at or before b
#pragma unroll
    for (int i = 1; i < GA::MAXM; ++i) m += (i < ga.nmem && b >= ga.start[i]) ? 1 : 0;
    ga.a[m].template call<Op>(SubGrid{b - ga.start[m], ga.start[m + 1] - ga.start[m]});
}

}  // namespace dev

// One recorded launch.
struct LaunchRec {
    const void* key;                   // identifies the body and its operand types
    unsigned grid;
    std::vector<unsigned char> args;   // ArgPack of the operands
    int (*emit)(const LaunchRec* const* ops, int n, hipStream_t s);   // returns the launches issued
};

struct LaunchRecorder {
    std::vector<LaunchRec> ops;
};

// Recorder of the calling thread (null: launches run at once).
LaunchRecorder*& launch_recorder();

// Installs a recorder on the calling thread for its lifetime.
struct RecordLaunches {
    LaunchRecorder* prev;
    explicit RecordLaunches(LaunchRecorder* r) : prev(launch_recorder()) { launch_recorder() = r; }
    ~RecordLaunches() { launch_recorder() = prev; }
    RecordLaunches(const RecordLaunches&) = delete;
    RecordLaunches& operator=(const RecordLaunches&) = delete;
};

template <class Op, class... P>
int emit_group(const LaunchRec* const* ops, int n, hipStream_t s) {
    using GA = dev::GroupArgs<P...>;
    static_assert(sizeof(GA) <= dev::GROUP_ARG_BYTES, "grouped launch arguments too large");
    int launches = 0;
    for (int i0 = 0; i0 < n; i0 += GA::MAXM) {
        const int m = n - i0 < GA::MAXM ? n - i0 : GA::MAXM;
        GA ga;
        memset(&ga, 0, sizeof(ga));
        ga.nmem = m;
        unsigned total = 0;
        for (int j = 0; j < m; ++j) {
            ga.start[j] = total;
            total += ops[i0 + j]->grid;
            memcpy(&ga.a[j], ops[i0 + j]->args.data(), sizeof(dev::ArgPack<P...>));
        }
        for (int j = m; j <= GA::MAXM; ++j) ga.start[j] = total;
        dev::k_group<Op, P...><<<total, Op::block, 0, s>>>(ga);
        ++launches;
    }
    return launches;
}

template <class Op, class... P, class... A>
void launch_sig(void (*)(dev::HwGrid, P...), unsigned grid, hipStream_t s, A... a) {
    if (!grid) return;
    if (LaunchRecorder* r = launch_recorder()) {
        const dev::ArgPack<P...> pk = dev::make_argpack(P(a)...);
        LaunchRec rec;
        rec.key = reinterpret_cast<const void*>(&emit_group<Op, P...>);
        rec.grid = grid;
        rec.args.resize(sizeof(pk));
        memcpy(rec.args.data(), &pk, sizeof(pk));
        rec.emit = &emit_group<Op, P...>;
        r->ops.push_back(std::move(rec));
        return;
    }
    dev::k_one<Op, P...><<<grid, Op::block, 0, s>>>(P(a)...);
}

// Launches (or records) the body of Op on `grid` blocks of Op::block threads.
template <class Op, class... A>
void launch(unsigned grid, hipStream_t s, A... a) {
    launch_sig<Op>(static_cast<typename Op::sig>(nullptr), grid, s, a...);
}

// Merges the recorded launch sequences of independent members into grouped launches:
// each member's launches keep their order, a grouped launch takes the next launch of
// every member whose next launch has the same body and operand types.  Greedy: the body
// that is next for the most members, ties to the member with the most launches left.
// Returns the number of grouped launches issued on s.
int group_launches(const std::vector<LaunchRecorder>& members, hipStream_t s);

}  // namespace amge
