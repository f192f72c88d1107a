"""Serving driver: a seeded Poisson stream of solve requests over resident hierarchies.

The engine itself (admission, continuous batching, per-hierarchy streams and graphs,
ensembles of hierarchies sharing grouped launches) is native (amge_server_* in the
library); this module builds the resident hierarchies of a request mix, feeds requests
at their arrival times and records latencies.
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np

from . import amge
from . import workloads as W


@dataclasses.dataclass
class Mix:
    """Resident hierarchies and device right-hand sides of a request stream."""
    requests: list            # dicts from workloads.serving_requests (arrival times at rate 1)
    keys: list                # (kind, n, coef_seed) per hierarchy
    hierarchies: list         # amge.Hierarchy per key
    hid_of: list              # request -> index into keys
    rhs: list                 # device FP64 right-hand side per request
    x: list                   # device FP64 solution per request
    build_s: float = 0.0
    setup_s: float = 0.0


def build_mix(num=256, seed=0, sizes=(16, 24, 32, 48, 64), coef_pool=2, slots=8, precond_bits=0,
              nu_primary=2, nu_aux=2, tail_rows=2048, extension="l2", smoother="l1jacobi"):
    """Hierarchies for every (kind, n, coefficient seed) of the stream (coefficients as the
    jump workload: per 4^3-hex block 10^U(-3,3)), and one right-hand side per request
    (seed = request id).  precond_bits 0 lets every hierarchy pick its V-cycle precision
    by trial solves at set-up; smoother: the point smoother ("l1jacobi" or "l1blockgs")."""
    import torch
    reqs = W.serving_requests(num, seed, sizes, coef_pool, rate=1.0)
    keys = sorted({(r["kind"], r["n"], r["coef_seed"]) for r in reqs})
    hs, tb, ts = [], 0.0, 0.0
    for kind, n, cs in keys:
        w = W.Workload(f"{kind}_n{n}_c{cs}", kind, n, W.default_levels(n), "blocks", coef_seed=cs)
        a, b = W.coefficients(w)
        t0 = time.perf_counter()
        prod = amge.build_problem(kind, n, w.levels, a, b, extension=extension, device=True)
        t1 = time.perf_counter()
        hs.append(amge.Hierarchy(prod, precond_bits=precond_bits, max_rhs=slots, nu_primary=nu_primary,
                                 nu_aux=nu_aux, tail_rows=tail_rows(n) if callable(tail_rows) else tail_rows,
                                 smoother=smoother))
        tb += t1 - t0
        ts += time.perf_counter() - t1
    index = {k: i for i, k in enumerate(keys)}
    hid_of = [index[(r["kind"], r["n"], r["coef_seed"])] for r in reqs]
    rhs, xs = [], []
    for r, h in zip(reqs, hid_of):
        n1 = hs[h].rows[0]
        rhs.append(torch.from_numpy(W.rhs(n1, r["rhs_seed"])[:, 0]).cuda())
        xs.append(torch.zeros(n1, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    return Mix(reqs, keys, hs, hid_of, rhs, xs, tb, ts)


def make_server(mix, hierarchy_budget=0, inflight_budget=0, chunk=8, grouped_max_n=0, ensembles=1):
    """Server with every hierarchy of the mix resident; those with n <= grouped_max_n
    join one of `ensembles` ensembles in turn (their iterations share grouped launches)."""
    srv = amge.Server(hierarchy_budget, inflight_budget, chunk)
    ids, k = [], 0
    for h, key in zip(mix.hierarchies, mix.keys):
        if key[1] <= grouped_max_n:
            ids.append(srv.add(h, grouped=True, ensemble=k % ensembles))
            k += 1
        else:
            ids.append(srv.add(h))
    return srv, ids


def run(srv, ids, mix, arrivals=None, order=None, rtol=1e-8, maxit=1000, poll_sleep=20e-6):
    """Feeds the requests of `order` (default: all) to the server at their arrival times
    (seconds from the start; None: all at once, a closed batch) and waits for all of them.

    Returns per request: completion record and latency (completion time - arrival time),
    plus the makespan."""
    import torch
    order = list(range(len(mix.requests))) if order is None else list(order)
    arr = np.zeros(len(order)) if arrivals is None else np.asarray(arrivals, dtype=np.float64)
    idx = np.argsort(arr, kind="stable")
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nxt, done = 0, {}
    done_t = {}
    while len(done) < len(order):
        now = time.perf_counter() - t0
        while nxt < len(order) and arr[idx[nxt]] <= now:
            j = order[idx[nxt]]
            srv.submit(ids[mix.hid_of[j]], mix.rhs[j], mix.x[j], tag=j, rtol=rtol, maxit=maxit, stream=stream)
            nxt += 1
        got = srv.progress(wait=False)
        tnow = time.perf_counter() - t0
        for tag, hid, status, iters, relres in got:
            done[tag] = (status, iters, relres)
            done_t[tag] = tnow
        if not got:
            st = srv.stats()
            if st["queued"] == 0 and st["inflight"] == 0 and nxt < len(order):
                # idle until the next arrival
                time.sleep(max(0.0, min(arr[idx[nxt]] - (time.perf_counter() - t0), 1e-3)))
            else:
                time.sleep(poll_sleep)
    makespan = max(done_t.values()) if done_t else 0.0
    pos = {j: k for k, j in enumerate(order)}
    lat = {j: done_t[j] - arr[pos[j]] for j in order}
    return done, lat, makespan


def run_closed(srv, ids, mix, concurrency, rtol=1e-8, maxit=1000, poll_sleep=20e-6):
    """Closed loop: `concurrency` requests outstanding at all times; each completion
    submits the next request of the stream.  Returns completions, latencies (completion
    - submission) and the makespan."""
    import torch
    order = list(range(len(mix.requests)))
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sub_t, done, done_t = {}, {}, {}
    nxt = 0

    def submit_one():
        nonlocal nxt
        j = order[nxt]
        srv.submit(ids[mix.hid_of[j]], mix.rhs[j], mix.x[j], tag=j, rtol=rtol, maxit=maxit, stream=stream)
        sub_t[j] = time.perf_counter() - t0
        nxt += 1

    while nxt < min(concurrency, len(order)):
        submit_one()
    while len(done) < len(order):
        got = srv.progress(wait=False)
        tnow = time.perf_counter() - t0
        for tag, hid, status, iters, relres in got:
            done[tag] = (status, iters, relres)
            done_t[tag] = tnow
            if nxt < len(order):
                submit_one()
        if not got:
            time.sleep(poll_sleep)
    makespan = max(done_t.values()) if done_t else 0.0
    lat = {j: done_t[j] - sub_t[j] for j in order}
    return done, lat, makespan


def latency_stats(lat):
    v = np.sort(np.asarray(list(lat.values())))
    return {"p50_ms": 1e3 * float(np.percentile(v, 50)), "p99_ms": 1e3 * float(np.percentile(v, 99)),
            "max_ms": 1e3 * float(v[-1]), "mean_ms": 1e3 * float(v.mean())}
