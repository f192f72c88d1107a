// Serving engine: many resident hierarchies and a stream of single right-hand-side
// solve requests.
//
// Each hierarchy added to a server runs the batched PCG (one column per request) on its
// own stream, replaying its captured iteration graph in chunks.  Between chunks the
// host reads the per-column states (pinned memory, no stall of the other hierarchies),
// copies finished columns out, and loads queued requests into the freed columns while
// the other columns stay in flight: continuous batching at the granularity of a PCG
// iteration.  Different hierarchies advance concurrently on their own streams.
//
// Hierarchies added as grouped join one of the server's ensembles instead: one PCG
// iteration of every member of an ensemble is captured as a single graph in which the
// same level operator of the members runs as one grouped launch (grouped.hpp), so small
// hierarchies, whose iterations are chains of short launches, share their launches.
// Each ensemble runs its chunks on its own stream (ensembles advance concurrently, like
// solo hierarchies); every member computes exactly what it computes alone.
//
// Admission: a hierarchy is made resident only if its device footprint fits the
// hierarchy budget; a request is admitted when its hierarchy has a free column and the
// work footprint of all admitted requests (their share of the batched work blocks)
// stays within the in-flight budget.  Requests are admitted in arrival order; one that
// does not fit the in-flight budget blocks those behind it, one whose hierarchy is full
// does not.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <memory>
#include <thread>
#include <vector>

#include "common.hpp"
#include "hierarchy.hpp"

namespace amge {
namespace dev {

constexpr int SBLOCK = 256;

// Loads one right-hand side (n contiguous values) into column c as a fresh column.
__global__ void __launch_bounds__(SBLOCK)
k_serve_insert(int64_t n, int lg, int c, const double* __restrict__ b, double* __restrict__ R, double* __restrict__ X,
               double* __restrict__ P, ColState* __restrict__ cs, BatchStatus* __restrict__ bs, double rtol, int maxit,
               int stop_l2) {
    for (int64_t i = (int64_t)blockIdx.x * SBLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * SBLOCK) {
        const int64_t t = (i << lg) + c;
        R[t] = b[i];
        X[t] = 0.0;
        P[t] = 0.0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ColState s = {};
        s.rtol = rtol;
        s.maxit = maxit;
        s.stop_l2 = stop_l2;
        s.fresh = 1;
        cs[c] = s;
        bs->all_done = 0;
    }
}

// x = column c of X.
__global__ void __launch_bounds__(SBLOCK)
k_serve_extract(int64_t n, int lg, int c, const double* __restrict__ X, double* __restrict__ x) {
    for (int64_t i = (int64_t)blockIdx.x * SBLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * SBLOCK)
        x[i] = X[(i << lg) + c];
}

// Column c idle (a cancelled request leaves it).
__global__ void k_serve_cancel(int c, ColState* __restrict__ cs) {
    if (threadIdx.x == 0) {
        ColState s = {};
        s.done = 1;
        cs[c] = s;
    }
}

// Every column idle.
__global__ void k_serve_reset(int NC, ColState* __restrict__ cs, BatchStatus* __restrict__ bs) {
    const int c = threadIdx.x;
    if (c < NC) {
        ColState s = {};
        s.done = 1;
        cs[c] = s;
    }
    if (c == 0) {
        bs->it = 0;
        bs->all_done = 1;
        bs->any_breakdown = 0;
    }
}

}  // namespace dev

namespace {

unsigned sgrid(int64_t n) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + dev::SBLOCK - 1) / dev::SBLOCK, 2048));
}

struct Request {
    int64_t tag = 0;
    int hid = 0;
    const double* b = nullptr;
    double* x = nullptr;
    double rtol = 0;
    int maxit = 0, stop_l2 = 0;
    hipEvent_t ready = nullptr;   // recorded on the caller's stream at submission
    bool cancel = false;          // cancelled while its chunk was in flight
    amge_completion done{};
};

// One resident hierarchy and its columns.
struct Group {
    const amge_hierarchy* hier = nullptr;   // the resident hierarchy
    std::unique_ptr<amge_ctx> ctx;          // the server's context of it (max_rhs columns)
    amge_hierarchy* H = nullptr;            // the context's execution state
    bool grouped = false;          // member of an ensemble
    hipStream_t stream = nullptr;  // where its inserts, chunks and copy-outs run
    size_t footprint = 0;          // device bytes of the hierarchy
    size_t col_bytes = 0;          // work bytes of one column
    std::vector<int> slot;         // column -> index into the server's request table, -1 free
    dev::ColState* cs_host = nullptr;   // pinned copy of the column states after a chunk
    hipEvent_t ev_chunk = nullptr, ev_extract = nullptr;
    bool chunk_busy = false;
    std::vector<int> extracting;   // requests whose copy-out is in flight
    int active = 0;                // columns holding a request
    // cost model of one PCG iteration on W columns: fixed + W * per_col milliseconds
    // (launch overhead, matrix bytes, vector bytes at a nominal bandwidth); mat_ms is
    // the matrix part of fixed_ms
    double fixed_ms = 0, per_col_ms = 0, mat_ms = 0;
    double chunk_ms = 0;           // estimate for the chunk in flight
    uint64_t turn = 0;             // when the group last finished a chunk (scheduling order)
};

// A set of grouped hierarchies: one captured graph (per iteration parity) runs an
// iteration of all of them (on all their columns), recaptured when a member joins.
constexpr int MAX_ENSEMBLES = 16;
struct Ensemble {
    std::vector<Group*> members;
    hipStream_t stream = nullptr;
    hipGraphExec_t exec[2] = {};   // by iteration parity (which z block is new)
    int par = 0;                   // parity of the next iteration
    bool stale = false;            // a member joined since the capture
    bool busy = false;             // a chunk is in flight
    hipEvent_t ev_chunk = nullptr;
    double chunk_ms = 0;
    uint64_t turn = 0;
    int launches = 0, solo_launches = 0;   // kernels per iteration: grouped, and run alone
};

// Nominal figures of the scheduling cost model.
constexpr double SCHED_BW_BYTES_PER_MS = 3.0e9;   // 3 TB/s
constexpr double SCHED_LAUNCH_MS = 0.003;          // per kernel of an iteration
constexpr double SCHED_CHUNK_MS = 2.0;             // target length of a chunk
constexpr double SCHED_QUEUE_MS = 8.0;             // estimated work allowed in flight

}  // namespace
}  // namespace amge

using namespace amge;

struct amge_server {
    size_t hierarchy_budget = 0, inflight_budget = 0;
    size_t resident = 0, inflight = 0;
    int chunk = 2;                    // upper bound on iterations per chunk
    double queued_ms = 0;             // estimated GPU time of the chunks in flight
    uint64_t clock = 0;               // scheduling turns
    std::vector<std::unique_ptr<Group>> groups;
    std::vector<std::unique_ptr<Ensemble>> ens;
    std::vector<Request> reqs;        // request table (indices stay valid)
    std::vector<int> free_reqs;       // reusable entries of the table
    std::deque<int> queue;            // submitted, not admitted, in arrival order
    std::deque<amge_completion> done; // finished, not yet returned
    std::vector<hipEvent_t> event_pool;

    ~amge_server() {
        for (auto& e : ens) {
            if (e->stream) (void)hipStreamSynchronize(e->stream);
            for (hipGraphExec_t x : e->exec)
                if (x) (void)hipGraphExecDestroy(x);
            if (e->ev_chunk) (void)hipEventDestroy(e->ev_chunk);
            if (e->stream) (void)hipStreamDestroy(e->stream);
        }
        for (auto& g : groups) {
            (void)hipStreamSynchronize(g->H->gstream);
            if (g->cs_host) (void)hipHostFree(g->cs_host);
            if (g->ev_chunk) (void)hipEventDestroy(g->ev_chunk);
            if (g->ev_extract) (void)hipEventDestroy(g->ev_extract);
        }
        for (Request& r : reqs)
            if (r.ready) event_pool.push_back(r.ready);
        for (hipEvent_t e : event_pool) (void)hipEventDestroy(e);
    }

    hipEvent_t take_event() {
        if (!event_pool.empty()) {
            hipEvent_t e = event_pool.back();
            event_pool.pop_back();
            return e;
        }
        hipEvent_t e;
        HIPCHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        return e;
    }

    int new_request() {
        if (!free_reqs.empty()) {
            int i = free_reqs.back();
            free_reqs.pop_back();
            return i;
        }
        reqs.emplace_back();
        return (int)reqs.size() - 1;
    }

    void release(int i) {
        if (reqs[i].ready) event_pool.push_back(reqs[i].ready);
        reqs[i] = Request{};
        free_reqs.push_back(i);
    }

    // Completion of copy-outs: report every request of a finished extraction.
    bool reap_extractions(Group& g) {
        if (g.extracting.empty()) return false;
        hipError_t e = hipEventQuery(g.ev_extract);
        if (e == hipErrorNotReady) return false;
        HIPCHECK(e);
        for (int i : g.extracting) {
            done.push_back(reqs[i].done);
            release(i);
        }
        g.extracting.clear();
        return true;
    }

    // A chunk has finished: copy finished columns out and free them.
    bool reap_chunk(Group& g) {
        if (!g.chunk_busy || g.grouped) return false;
        hipError_t e = hipEventQuery(g.ev_chunk);
        if (e == hipErrorNotReady) return false;
        HIPCHECK(e);
        queued_ms -= g.chunk_ms;
        if (queued_ms < 1e-9) queued_ms = 0;
        g.turn = ++clock;
        collect(g);
        return true;
    }

    bool reap_ensemble(Ensemble& en) {
        if (!en.busy) return false;
        hipError_t e = hipEventQuery(en.ev_chunk);
        if (e == hipErrorNotReady) return false;
        HIPCHECK(e);
        en.busy = false;
        queued_ms -= en.chunk_ms;
        if (queued_ms < 1e-9) queued_ms = 0;
        en.turn = ++clock;
        for (Group* g : en.members) collect(*g);
        return true;
    }

    // Frees column c of an idle group and reports its request as cancelled (x is not
    // written); the column is marked idle on the device before anything later on the
    // group's stream.
    void drop_column(Group& g, int c) {
        const int i = g.slot[c];
        dev::k_serve_cancel<<<1, 64, 0, g.stream>>>(c, g.H->cs);
        HIPCHECK(hipGetLastError());
        Request& r = reqs[i];
        amge_completion d{};
        d.tag = r.tag;
        d.hierarchy = r.hid;
        d.status = AMGE_CANCELLED;
        d.iters = g.cs_host[c].iters;
        d.relres = g.cs_host[c].relres;
        done.push_back(d);
        release(i);
        g.slot[c] = -1;
        g.active -= 1;
        inflight -= g.col_bytes;
    }

    // Cancels every queued or in-flight request with this tag (see amge_server_cancel).
    int cancel(int64_t tag) {
        int n = 0;
        for (auto it = queue.begin(); it != queue.end();) {
            if (reqs[*it].tag != tag) {
                ++it;
                continue;
            }
            amge_completion d{};
            d.tag = tag;
            d.hierarchy = reqs[*it].hid;
            d.status = AMGE_CANCELLED;
            done.push_back(d);
            release(*it);
            it = queue.erase(it);
            ++n;
        }
        for (auto& gp : groups) {
            Group& g = *gp;
            for (int c = 0; c < (int)g.slot.size(); ++c) {
                const int i = g.slot[c];
                if (i < 0 || reqs[i].tag != tag || reqs[i].cancel) continue;
                if (g.chunk_busy) reqs[i].cancel = true;   // dropped when the chunk ends
                else drop_column(g, c);
                ++n;
            }
        }
        return n;
    }

    // After a chunk: report finished columns, copy them out and free them; drop the
    // columns of requests cancelled meanwhile.
    void collect(Group& g) {
        g.chunk_busy = false;
        amge_hierarchy* H = g.H;
        const int64_t n = H->lv[0].n;
        bool any = false;
        for (int c = 0; c < H->NC; ++c) {
            const int i = g.slot[c];
            if (i < 0) continue;
            if (reqs[i].cancel) {
                drop_column(g, c);
                continue;
            }
            const dev::ColState& s = g.cs_host[c];
            if (!s.done) continue;
            Request& r = reqs[i];
            r.done.tag = r.tag;
            r.done.hierarchy = r.hid;
            r.done.iters = s.iters;
            r.done.relres = s.relres;
            r.done.status = s.nonfinite ? AMGE_ERR_NONFINITE
                            : s.breakdown ? AMGE_ERR_BREAKDOWN
                            : (r.rtol > 0 && !(s.relres <= r.rtol)) ? AMGE_NOT_CONVERGED
                                                                     : AMGE_OK;
            dev::k_serve_extract<<<sgrid(n), dev::SBLOCK, 0, g.stream>>>(n, H->lgNC, c, H->bX, r.x);
            g.extracting.push_back(i);
            g.slot[c] = -1;
            g.active -= 1;
            inflight -= g.col_bytes;
            any = true;
        }
        if (any) {
            HIPCHECK(hipGetLastError());
            HIPCHECK(hipEventRecord(g.ev_extract, g.stream));
        }
    }

    // Loads queued requests into free columns of idle groups.
    bool admit() {
        bool any = false;
        for (auto it = queue.begin(); it != queue.end();) {
            Request& r = reqs[*it];
            Group& g = *groups[r.hid];
            if (inflight_budget && inflight + g.col_bytes > inflight_budget) break;   // keeps arrival order
            if (g.chunk_busy || g.active == g.H->NC) {
                ++it;
                continue;
            }
            int c = 0;
            while (g.slot[c] >= 0) ++c;
            amge_hierarchy* H = g.H;
            const int64_t n = H->lv[0].n;
            HIPCHECK(hipStreamWaitEvent(g.stream, r.ready, 0));
            dev::k_serve_insert<<<sgrid(n), dev::SBLOCK, 0, g.stream>>>(n, H->lgNC, c, r.b, H->bR, H->bX, H->bP,
                                                                         H->cs, H->bs, r.rtol, r.maxit, r.stop_l2);
            HIPCHECK(hipGetLastError());
            g.slot[c] = *it;
            g.active += 1;
            inflight += g.col_bytes;
            it = queue.erase(it);
            any = true;
        }
        return any;
    }

    // Starts chunks of iterations on idle groups that hold requests, in the order in which
    // they last finished one (every group gets its turn), while the estimated GPU time of
    // the chunks in flight stays within SCHED_QUEUE_MS (at least one chunk always runs).
    // Hardware queues run kernels in order, so bounding the queued work bounds how long a
    // new chunk of a small hierarchy waits behind the chunks of large ones.  A chunk has as
    // many iterations as fit SCHED_CHUNK_MS (at least one, at most `chunk`).
    bool launch() {
        struct Cand {
            Group* g;      // a solo hierarchy, or
            Ensemble* e;   // an ensemble
            uint64_t turn;
        };
        std::vector<Cand> cand;
        for (auto& gp : groups)
            if (!gp->grouped && !gp->chunk_busy && gp->active > 0) cand.push_back({gp.get(), nullptr, gp->turn});
        for (auto& ep : ens)
            if (!ep->busy)
                for (Group* g : ep->members)
                    if (g->active > 0) {
                        cand.push_back({nullptr, ep.get(), ep->turn});
                        break;
                    }
        std::sort(cand.begin(), cand.end(), [](const Cand& a, const Cand& b) { return a.turn < b.turn; });
        bool any = false;
        for (const Cand& cd : cand) {
            if (cd.e) {
                if (!launch_ensemble(*cd.e)) break;
                any = true;
                continue;
            }
            Group& g = *cd.g;
            amge_hierarchy* H = g.H;
            // active width: the columns up to the highest occupied one (requests take the
            // lowest free column)
            int hi = 0;
            for (int c = 0; c < H->NC; ++c)
                if (g.slot[c] >= 0) hi = c + 1;
            int W = 1;
            while (W < hi) W *= 2;
            const double it_ms = g.fixed_ms + W * g.per_col_ms;
            const int k = std::max(1, std::min(chunk, (int)(SCHED_CHUNK_MS / it_ms)));
            const double est = k * it_ms;
            if (queued_ms > 0 && queued_ms + est > SCHED_QUEUE_MS) break;
            for (int i = 0; i < k; ++i) {
                HIPCHECK(hipGraphLaunch(capture_iteration(H, W, H->bpar), H->gstream));
                H->bpar ^= 1;
            }
            HIPCHECK(hipMemcpyAsync(g.cs_host, H->cs, sizeof(dev::ColState) * H->NC, hipMemcpyDeviceToHost,
                                    H->gstream));
            HIPCHECK(hipEventRecord(g.ev_chunk, H->gstream));
            g.chunk_busy = true;
            g.chunk_ms = est;
            queued_ms += est;
            any = true;
        }
        return any;
    }

    // A chunk of an ensemble (all members, all columns); false if the queue is full.
    bool launch_ensemble(Ensemble& en) {
        if (en.stale || !en.exec[0]) {
            std::vector<amge_hierarchy*> hs;
            for (Group* g : en.members) hs.push_back(g->H);
            for (int p = 0; p < 2; ++p) {
                hipGraphExecDestroy_if(en.exec[p]);
                en.exec[p] = capture_grouped_iteration(hs, p, en.stream, &en.launches, &en.solo_launches);
            }
            en.stale = false;
        }
        // members without requests return from every kernel at once
        double it_ms = en.launches * SCHED_LAUNCH_MS;
        for (Group* g : en.members)
            if (g->active > 0) it_ms += g->mat_ms + g->H->NC * g->per_col_ms;
        const int k = std::max(1, std::min(chunk, (int)(SCHED_CHUNK_MS / it_ms)));
        const double est = k * it_ms;
        if (queued_ms > 0 && queued_ms + est > SCHED_QUEUE_MS) return false;
        for (int i = 0; i < k; ++i) {
            HIPCHECK(hipGraphLaunch(en.exec[en.par], en.stream));
            en.par ^= 1;
        }
        for (Group* g : en.members) {
            HIPCHECK(hipMemcpyAsync(g->cs_host, g->H->cs, sizeof(dev::ColState) * g->H->NC, hipMemcpyDeviceToHost,
                                    en.stream));
            g->chunk_busy = true;
        }
        HIPCHECK(hipEventRecord(en.ev_chunk, en.stream));
        en.busy = true;
        en.chunk_ms = est;
        queued_ms += est;
        return true;
    }

    static void hipGraphExecDestroy_if(hipGraphExec_t& ex) {
        if (ex) (void)hipGraphExecDestroy(ex);
        ex = nullptr;
    }

    bool busy() const {
        if (!queue.empty()) return true;
        for (auto& e : ens)
            if (e->busy) return true;
        for (auto& g : groups)
            if (g->chunk_busy || g->active || !g->extracting.empty()) return true;
        return false;
    }
};

namespace {
template <class F>
amge_status sguard(F&& f) {
    try {
        return f();
    } catch (const Error& e) {
        set_last_error(e.what());
        return e.code;
    } catch (const std::bad_alloc&) {
        set_last_error("host allocation failed");
        return AMGE_ERR_OOM;
    } catch (const std::exception& e) {
        set_last_error(e.what());
        return AMGE_ERR_ARG;
    }
}
}  // namespace

extern "C" amge_status amge_server_create(size_t hierarchy_budget, size_t inflight_budget, int32_t chunk,
                                          amge_server** out) {
    return sguard([&]() -> amge_status {
        if (!out) fail(AMGE_ERR_ARG, "null output pointer");
        if (chunk < 1) fail(AMGE_ERR_ARG, "chunk must be >= 1");
        auto S = std::make_unique<amge_server>();
        S->hierarchy_budget = hierarchy_budget;
        S->inflight_budget = inflight_budget;
        S->chunk = chunk;
        *out = S.release();
        return AMGE_OK;
    });
}

extern "C" void amge_server_destroy(amge_server* s) { delete s; }

namespace {
amge_status server_add(amge_server* s, amge_hierarchy* hier, int32_t* id, int ensemble) {
    const bool grouped = ensemble >= 0;
    return sguard([&]() -> amge_status {
        if (ensemble >= MAX_ENSEMBLES) fail(AMGE_ERR_ARG, "ensemble index out of range");
        if (!s || !hier || !id) fail(AMGE_ERR_ARG, "null argument");
        if (hier->parent) fail(AMGE_ERR_ARG, "not a hierarchy");
        if (hier->opts.max_rhs < 2) fail(AMGE_ERR_ARG, "hierarchy needs max_rhs >= 2 to serve");
        for (auto& g : s->groups)
            if (g->hier == hier) fail(AMGE_ERR_ARG, "hierarchy already added");
        const size_t need = hier->bytes + make_ctx(hier, hier->opts.max_rhs, true)->st.bytes;
        if (s->hierarchy_budget && s->resident + need > s->hierarchy_budget)
            fail(AMGE_ERR_BUSY, "hierarchy does not fit the device memory budget");
        auto g = std::make_unique<Group>();
        g->hier = hier;
        g->ctx = make_ctx(hier, hier->opts.max_rhs);
        amge_hierarchy* h = &g->ctx->st;
        g->H = h;
        g->footprint = hier->bytes + h->bytes;
        // one column of the work blocks: six FP64 PCG blocks and the V-cycle's level blocks
        size_t cb = 6 * sizeof(double) * (size_t)h->lv[0].n;
        const size_t vs = (h->opts.precond_bits == 32 && h->lv.size() > 1) ? sizeof(float) : sizeof(double);
        for (const DLevel& L : h->lv) cb += vs * (5 * (size_t)L.n + 4 * (size_t)L.m);
        g->col_bytes = cb;
        g->slot.assign(h->NC, -1);
        {
            // cost model: V-cycle bytes on one and two columns (amge_vcycle_bytes), the FP64
            // product with A_1 and about twelve FP64 vector streams of the PCG updates
            const int bits = h->opts.precond_bits == 32 && h->lv.size() > 1 ? 32 : 64;
            double b1 = 0, b2 = 0;
            if (amge_vcycle_bytes(hier, bits, 1, &b1) != AMGE_OK || amge_vcycle_bytes(hier, bits, 2, &b2) != AMGE_OK)
                fail(AMGE_ERR_ARG, "cost model");
            const double n1 = h->lv[0].n;
            const double col = (b2 - b1) + 12 * 8 * n1;
            const double mat = (b1 - (b2 - b1)) + 12.0 * (double)h->lv[0].A.nnz;
            const int kernels = 16 * ((int)h->lv.size() - 1) + 8;
            g->mat_ms = std::max(0.0, mat) / SCHED_BW_BYTES_PER_MS;
            g->fixed_ms = kernels * SCHED_LAUNCH_MS + g->mat_ms;
            g->per_col_ms = col / SCHED_BW_BYTES_PER_MS;
        }
        HIPCHECK(hipHostMalloc((void**)&g->cs_host, sizeof(dev::ColState) * h->NC, hipHostMallocDefault));
        HIPCHECK(hipEventCreateWithFlags(&g->ev_chunk, hipEventDisableTiming));
        HIPCHECK(hipEventCreateWithFlags(&g->ev_extract, hipEventDisableTiming));
        if (grouped) {
            while ((int)s->ens.size() <= ensemble) s->ens.push_back(std::make_unique<Ensemble>());
            Ensemble& en = *s->ens[ensemble];
            if (!en.stream) {
                HIPCHECK(hipStreamCreateWithFlags(&en.stream, hipStreamNonBlocking));
                HIPCHECK(hipEventCreateWithFlags(&en.ev_chunk, hipEventDisableTiming));
            }
            g->grouped = true;
            g->stream = en.stream;
        } else {
            g->stream = h->gstream;
            for (int W = 1; W <= h->NC; W *= 2)
                for (int p = 0; p < 2; ++p) capture_iteration(h, W, p);
        }
        dev::k_serve_reset<<<1, 64, 0, h->gstream>>>(h->NC, h->cs, h->bs);
        HIPCHECK(hipGetLastError());
        HIPCHECK(hipStreamSynchronize(h->gstream));
        s->resident += g->footprint;
        *id = (int32_t)s->groups.size();
        if (grouped) {
            s->ens[ensemble]->members.push_back(g.get());
            s->ens[ensemble]->stale = true;
        }
        s->groups.push_back(std::move(g));
        return AMGE_OK;
    });
}
}  // namespace

extern "C" amge_status amge_server_add(amge_server* s, amge_hierarchy* h, int32_t* id) {
    return server_add(s, h, id, -1);
}

extern "C" amge_status amge_server_add_grouped(amge_server* s, amge_hierarchy* h, int32_t ensemble, int32_t* id) {
    if (ensemble < 0) {
        set_last_error("ensemble index must be >= 0");
        return AMGE_ERR_ARG;
    }
    return server_add(s, h, id, ensemble);
}

extern "C" amge_status amge_server_ensemble(const amge_server* s, int32_t* members, int32_t* launches,
                                            int32_t* solo_launches) {
    return sguard([&]() -> amge_status {
        if (!s) fail(AMGE_ERR_ARG, "null argument");
        int32_t m = 0, k = 0, k1 = 0;
        for (auto& e : s->ens) {
            m += (int32_t)e->members.size();
            k += e->launches;
            k1 += e->solo_launches;
        }
        if (members) *members = m;
        if (launches) *launches = k;
        if (solo_launches) *solo_launches = k1;
        return AMGE_OK;
    });
}

extern "C" amge_status amge_server_request_bytes(const amge_server* s, int32_t id, size_t* bytes) {
    return sguard([&]() -> amge_status {
        if (!s || !bytes) fail(AMGE_ERR_ARG, "null argument");
        if (id < 0 || id >= (int32_t)s->groups.size()) fail(AMGE_ERR_ARG, "unknown hierarchy id");
        *bytes = s->groups[id]->col_bytes;
        return AMGE_OK;
    });
}

extern "C" amge_status amge_server_submit(amge_server* s, int32_t id, const double* b, double* x, double rtol,
                                          int32_t maxit, int32_t stop_norm, int64_t tag, void* stream) {
    return sguard([&]() -> amge_status {
        if (!s || !b || !x) fail(AMGE_ERR_ARG, "null argument");
        if (id < 0 || id >= (int32_t)s->groups.size()) fail(AMGE_ERR_ARG, "unknown hierarchy id");
        if (maxit < 1) fail(AMGE_ERR_ARG, "maxit must be >= 1");
        if (s->inflight_budget && s->groups[id]->col_bytes > s->inflight_budget)
            fail(AMGE_ERR_BUSY, "request work footprint exceeds the in-flight budget");
        const int i = s->new_request();
        Request& r = s->reqs[i];
        r.tag = tag;
        r.hid = id;
        r.b = b;
        r.x = x;
        r.rtol = rtol;
        r.maxit = maxit;
        r.stop_l2 = stop_norm ? 1 : 0;
        r.ready = s->take_event();
        HIPCHECK(hipEventRecord(r.ready, (hipStream_t)stream));
        s->queue.push_back(i);
        return AMGE_OK;
    });
}

extern "C" amge_status amge_server_progress(amge_server* s, int32_t wait, amge_completion* out, int32_t cap,
                                            int32_t* nout) {
    return sguard([&]() -> amge_status {
        if (!s || !nout || (cap > 0 && !out)) fail(AMGE_ERR_ARG, "null argument");
        *nout = 0;
        while (true) {
            bool moved = false;
            for (auto& g : s->groups) {
                moved |= s->reap_extractions(*g);
                moved |= s->reap_chunk(*g);
            }
            for (auto& e : s->ens) moved |= s->reap_ensemble(*e);
            moved |= s->admit();
            moved |= s->launch();
            if (!s->done.empty() || !wait || !s->busy()) break;
            if (!moved) std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
        int k = 0;
        while (k < cap && !s->done.empty()) {
            out[k++] = s->done.front();
            s->done.pop_front();
        }
        *nout = k;
        return AMGE_OK;
    });
}

extern "C" amge_status amge_server_cancel(amge_server* s, int64_t tag, int32_t* count) {
    return sguard([&]() -> amge_status {
        if (!s) fail(AMGE_ERR_ARG, "null argument");
        const int n = s->cancel(tag);
        if (count) *count = n;
        return AMGE_OK;
    });
}

extern "C" amge_status amge_server_stats(const amge_server* s, int32_t* queued, int32_t* inflight,
                                         size_t* inflight_bytes, size_t* resident_bytes) {
    return sguard([&]() -> amge_status {
        if (!s) fail(AMGE_ERR_ARG, "null argument");
        int act = 0;
        for (auto& g : s->groups) act += g->active + (int)g->extracting.size();
        if (queued) *queued = (int32_t)s->queue.size();
        if (inflight) *inflight = act;
        if (inflight_bytes) *inflight_bytes = s->inflight;
        if (resident_bytes) *resident_bytes = s->resident;
        return AMGE_OK;
    });
}
