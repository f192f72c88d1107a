"""Benchmark of the AMGe solve phase on one MI355X.

One step = one complete PCG solve (FP32 V-cycle preconditioner inside FP64 inexact
PCG, stopped at relative residual 1e-8 in the preconditioner norm) of the H(curl)
system on the 64^3 x 6 Kuhn mesh with the 5-level hierarchy, starting from the
right-hand side already resident in HBM.  The hybrid smoother's point smoother is the
l1-scaled symmetric block Gauss-Seidel of the paper's experiments (64-row blocks; the
other point smoothers are timed beside it, --smoother picks the headline's).  The same solve with an all-FP64 V-cycle
("plain FP64 PCG") is timed beside it, and the V-cycle's achieved bandwidth is
reported from its algorithmic bytes.

Beside it, in the same JSON line: the roofline of the dominant kernel family (fine-level
A sweeps and residual, HIP events on their launch stream) with a measured device-copy
bandwidth for reference, the batched solve of the 48^3 H(div) workload with 32
right-hand sides, the serving mix (burst, closed loop, open loop) with a solo vs
grouped-launch comparison on small hierarchies, and the oracle timed on one host core.

Prints one JSON line (rank 0).  Options: --gpus N (only 1 is supported), --steps K,
--warmup W, --workload NAME, --no-cpu-baseline, --batched-workload NAME ("" to skip),
--serving-requests N (0 to skip), --smoother NAME, --grouped-ab-only CONFIG (one configuration of the
small-hierarchy serving burst alone, for kernel traces), --copy-calibration (a 1 GiB
device copy first: the reference kernel of the HBM counter runs).
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "solves/s + V-cycle HBM GB/s, FP32-precond vs FP64 PCG at rel-res 1e-8"
PEAK_HBM_GBPS = 8000.0
SMOOTHER_NAMES = {"l1blockgs": "l1-scaled symmetric block Gauss-Seidel (64-row blocks)",
                  "l1jacobi": "l1-Jacobi", "symgs": "symmetric Gauss-Seidel in colour order"}
ROOFLINE_KERNELS = {
    "l1blockgs": ("fine-level A_1 kernels on the block layout (block Gauss-Seidel sweeps, the first from zero "
                  "reading the in-block entries only, and the residual; FP32 values, 16-bit codes)"),
    "l1jacobi": "fine-level A_1 sliced-ELL kernels (l1-Jacobi sweeps + residual, FP32, 16-bit column offsets)",
    "symgs": "fine-level A_1 sliced-ELL residual (the colour sweeps are separate launches)"}


TRAFFIC_SOURCES = {
    "l1blockgs": ("paper_2107_05613_amd/csrc/kernels_base.hpp", "paper_2107_05613_amd/csrc/kernels_bgs.hpp",
                  "paper_2107_05613_amd/csrc/block_gs.hpp", "paper_2107_05613_amd/csrc/block_gs.hip"),
    "l1jacobi": ("paper_2107_05613_amd/csrc/kernels_base.hpp", "paper_2107_05613_amd/csrc/kernels.hpp",
                 "paper_2107_05613_amd/csrc/sell_layout.hpp", "paper_2107_05613_amd/csrc/sell_layout.cpp"),
}


def traffic_hash(smoother):
    """Hash of the sources of the dominant kernel family and its matrix layout."""
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES.get(smoother, ()):
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(smoother):
    """HBM bytes per launch of the dominant kernel family from the committed rocprofv3
    counter runs (profiles/hbm_traffic.json), or None if they were taken with another
    smoother or the kernel source or its matrix layout changed since."""
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "hbm_traffic.json")))
    except (OSError, ValueError):
        return None
    if rec.get("smoother") != smoother or smoother not in TRAFFIC_SOURCES:
        return None
    if traffic_hash(smoother) != rec.get("source_hash"):
        return None
    return rec["traffic_bytes_per_launch"]


def _oracle_sample(H, ml, rhs, iters):
    """Seconds per PCG iteration of the oracle: `iters` fixed iterations timed (they cost
    iters + 1 V-cycles and iters A-products)."""
    from oracle.solve import pcg
    t0 = time.perf_counter()
    pcg(H.A[0], rhs, ml, fixed_iters=iters)
    return (time.perf_counter() - t0) / (iters + 1)


def cpu_baseline_worker(workloads, budget_s: float, outdir: str, smoother: str = "l1jacobi"):
    """Oracle leg (separate process, one thread per process).  Per workload: the oracle
    hierarchy is built (not timed); its FP64 PCG solve to the workload's rtol gives the
    reference solution (saved to outdir for the GPU results' errors); a bounded number
    of PCG iterations is timed on one core; then one forked process per host core (the
    hierarchy shared copy-on-write) times the same iterations concurrently, for the
    aggregate throughput.  Prints a JSON dict."""
    import multiprocessing as mp
    import numpy as np
    from paper_2107_05613_amd import workloads as W
    from oracle.hierarchy import build_hierarchy
    from oracle.solve import Multilevel, pcg
    cores = len(os.sched_getaffinity(0))
    res = {}
    for name in workloads:
        w = W.WORKLOADS[name]
        a, b = W.coefficients(w)
        t0 = time.perf_counter()
        H = build_hierarchy(w.kind, w.n, w.levels, a, b, check_targets=False)
        ml = Multilevel.from_hierarchy(H, smoother=smoother)
        t_build = time.perf_counter() - t0
        rhs = W.rhs(H.A[0].shape[0], w.rhs_seed)[:, 0]
        t0 = time.perf_counter()
        x, ito, hist = pcg(H.A[0], rhs, ml, rtol=w.rtol)
        t_solve = time.perf_counter() - t0
        np.save(os.path.join(outdir, f"{name}.npy"), x)
        s1 = t_solve / (2 * ito + 1) * 2          # first estimate of seconds per iteration
        iters = max(1, min(200, int(budget_s / max(s1, 1e-4))))
        s_iter = _oracle_sample(H, ml, rhs, iters)
        # all cores: the same sample in one forked process per core, started together
        it_n = max(1, iters // 2)
        ctx = mp.get_context("fork")
        q = ctx.Queue()
        procs = [ctx.Process(target=lambda: q.put(_oracle_sample(H, ml, rhs, it_n))) for _ in range(cores)]
        t0 = time.perf_counter()
        for p in procs:
            p.start()
        per = [q.get() for _ in procs]
        for p in procs:
            p.join()
        wall = time.perf_counter() - t0
        res[name] = {"t_build_s": t_build, "oracle_iters": ito, "oracle_relres": hist[-1],
                     "t_solve_s": t_solve, "sample_iters": iters, "s_per_iter": s_iter,
                     "allcore_iters": it_n, "allcore_s_per_iter": per, "allcore_wall_s": wall}
        print(f"[oracle] {name}: build {t_build:.1f}s, {ito} iterations in {t_solve:.1f}s, "
              f"{1e3 * s_iter:.0f} ms/iteration on 1 core, {cores} cores {wall:.1f}s", file=sys.stderr, flush=True)
    res["cores"] = cores
    print(json.dumps(res), flush=True)


def run_cpu_baseline(workloads, budget_s=20.0, smoother="l1jacobi"):
    """Runs cpu_baseline_worker in a subprocess (BLAS and OpenMP pinned to one thread per
    process); returns (its JSON, directory of the oracle's reference solutions)."""
    import tempfile
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "NUMEXPR_NUM_THREADS"):
        env[k] = "1"
    outdir = tempfile.mkdtemp(prefix="amge_oracle_")
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-baseline-worker", "--workload", ",".join(workloads),
           "--cpu-budget", str(budget_s), "--oracle-dir", outdir, "--smoother", smoother]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, text=True, env=env, timeout=1500)
    if r.returncode != 0:
        return {"error": f"oracle worker exited with {r.returncode}"}, outdir
    return json.loads(r.stdout.strip().splitlines()[-1]), outdir


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def baseline_entry(res, iters_needed):
    """cpu_baseline object for one workload: 1-core solves/s (the sample scaled to
    iters_needed iterations per solve) and the all-core aggregate."""
    per_solve = res["s_per_iter"] * (iters_needed + 1)
    agg = sum(1.0 / (s * (iters_needed + 1)) for s in res["allcore_s_per_iter"])
    return {"value": 1.0 / per_solve, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "allcore": {"value": agg, "unit": "solves/s", "cores": len(res["allcore_s_per_iter"]),
                        "processes": "one forked oracle process per core, all timing the same sample at once"},
            "cpu_model": cpu_model(),
            "sample": (f"FP64 oracle (scipy CSR, 1 thread per process) PCG on its own hierarchy of the same "
                       f"workload and rhs: {res['sample_iters']} iterations timed on 1 core "
                       f"({res['sample_iters'] * res['s_per_iter']:.1f} s) and {res['allcore_iters']} per process on "
                       f"all cores ({res['allcore_wall_s']:.1f} s), scaled to {iters_needed} iterations per solve; "
                       f"hierarchy build {res['t_build_s']:.0f} s not timed (with the smoother's set-up)")}


def batched_smoother(args):
    """Point smoother of the batched and serving legs: the headline's, except the
    colour-order Gauss-Seidel (single-column only), which falls back to l1-Jacobi."""
    return args.smoother if args.smoother != "symgs" else "l1jacobi"


def run_batched(args, amge, W):
    """Block solve of the multi-right-hand-side workload: all columns in one batched
    FP32-preconditioned PCG call, against the same columns solved one at a time on the
    same hierarchy; plus the batched V-cycle's bandwidth from its algorithmic bytes."""
    import torch
    w = W.WORKLOADS[args.batched_workload]
    a, b = W.coefficients(w)
    t0 = time.perf_counter()
    prod = amge.build_problem(w.kind, w.n, w.levels, a, b)
    t_build = time.perf_counter() - t0
    sm = batched_smoother(args)
    t0 = time.perf_counter()
    H = amge.Hierarchy(prod, precond_bits=32, max_rhs=w.nrhs, smoother=sm)
    t_setup = time.perf_counter() - t0
    n1, k = H.rows[0], w.nrhs
    B = torch.from_numpy(W.rhs(n1, w.rhs_seed, k)).cuda().reshape(-1)
    X = torch.zeros_like(B)
    print(f"[bench] {w.name}: n1={n1} x {k} columns, build {t_build:.1f}s setup {t_setup:.1f}s",
          file=sys.stderr, flush=True)

    def block_solve():
        st, its, rrs = H.pcg(B, X, rtol=w.rtol, maxit=1000, nrhs=k)
        if st != 0:
            raise RuntimeError("batched solve did not converge")
        return its, rrs

    for _ in range(args.warmup):
        block_solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        its, rrs = block_solve()
    torch.cuda.synchronize()
    dt_b = (time.perf_counter() - t0) / args.steps
    # the same columns one at a time (a few of them), same hierarchy and precision
    ncol = min(k, 4)
    cols = [B.view(n1, k)[:, j].contiguous() for j in range(ncol)]
    x1 = torch.zeros(n1, dtype=torch.float64, device="cuda")
    H.pcg(cols[0], x1, rtol=w.rtol, maxit=1000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it1 = []
    for c in cols:
        st, it, _ = H.pcg(c, x1, rtol=w.rtol, maxit=1000)
        it1.append(it[0])
    torch.cuda.synchronize()
    dt_1 = (time.perf_counter() - t0) / ncol
    # batched V-cycle bandwidth (FP32)
    Z = torch.empty_like(B)
    for _ in range(3):
        H.vcycle(B, Z, nrhs=k)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record()
    for _ in range(reps):
        H.vcycle(B, Z, nrhs=k)
    e1.record()
    torch.cuda.synchronize()
    vms = e0.elapsed_time(e1) / reps
    by = H.vcycle_bytes(32, nrhs=k)
    H.close()
    # the same block with the all-FP64 V-cycle (plain FP64 PCG)
    H64 = amge.Hierarchy(prod, precond_bits=64, max_rhs=w.nrhs, smoother=sm)
    X.zero_()
    st, its64, _ = H64.pcg(B, X, rtol=w.rtol, maxit=1000, nrhs=k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(max(1, args.steps // 2)):
        st, its64, _ = H64.pcg(B, X, rtol=w.rtol, maxit=1000, nrhs=k)
    torch.cuda.synchronize()
    dt_64 = (time.perf_counter() - t0) / max(1, args.steps // 2)
    H64.close()
    print(f"[bench] batched: {k / dt_b:.1f} solves/s ({1e3 * dt_b:.1f} ms per block, iterations "
          f"{min(its)}..{max(its)}); FP64 block {k / dt_64:.1f} solves/s; one at a time {1 / dt_1:.1f} solves/s; "
          f"V-cycle {vms:.2f} ms", file=sys.stderr, flush=True)
    return {
        "workload": (f"{w.name}: H({w.kind}) on {w.n}^3x6 Kuhn tets, {w.levels}-level AMGe, {k} right-hand "
                     f"sides (uniform[-1,1] seed {w.rhs_seed}) in one call, FP32 V-cycle in per-column FP64 "
                     f"PCG to rel-res {w.rtol:g}, smoother {SMOOTHER_NAMES[sm]}"),
        "fine_dofs": n1,
        "solves_per_s": k / dt_b,
        "ms_per_block": 1e3 * dt_b,
        "iters": [min(its), max(its)],
        "single_column_solves_per_s": 1.0 / dt_1,
        "single_column_iters": it1,
        "batching_speedup": dt_1 * k / dt_b,
        "fp64_block_solves_per_s": k / dt_64,
        "fp64_block_iters": [min(its64), max(its64)],
        "speedup_fp32_vs_fp64_block": dt_64 / dt_b,
        "vcycle": {"ms": vms, "algorithmic_bytes": by, "GBps": by / (vms * 1e-3) / 1e9,
                   "ms_per_column": vms / k},
        "setup_s": {"build": t_build, "device_setup": t_setup},
    }


def run_small_configs(names, steps, smoother):
    """The two small configurations, each solved with the FP32 and the FP64 V-cycle on the
    library's own hierarchy: iterations, time per solve (host clock around complete
    solves), and the solutions (kept for their errors against the oracle)."""
    import torch
    from paper_2107_05613_amd import amge
    from paper_2107_05613_amd import workloads as W
    out, sols = {}, {}
    for name in names:
        w = W.WORKLOADS[name]
        a, b = W.coefficients(w)
        prod = amge.build_problem(w.kind, w.n, w.levels, a, b)
        rhs = None
        r = {"workload": (f"H({w.kind}) on {w.n}^3x6 Kuhn tets, {w.levels} levels, coefficients {w.coef}, "
                          f"rhs uniform[-1,1] seed {w.rhs_seed}, rtol {w.rtol:g}, smoother {smoother}")}
        for bits in (32, 64):
            H = amge.Hierarchy(prod, precond_bits=bits, smoother=smoother)
            if rhs is None:
                rhs = torch.from_numpy(W.rhs(H.rows[0], w.rhs_seed)[:, 0]).cuda()
                r["level_rows"] = H.rows
                r["kappa"] = H.precision_info()[0]
            x = torch.zeros_like(rhs)
            for _ in range(2):
                st, it, rr = H.pcg(rhs, x, rtol=w.rtol, maxit=2000)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                st, it, rr = H.pcg(rhs, x, rtol=w.rtol, maxit=2000)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            r[f"fp{bits}"] = {"iters": it[0], "relres": rr[0], "status": st, "ms_per_solve": 1e3 * dt,
                              "solves_per_s": 1.0 / dt}
            sols[(name, bits)] = x.cpu().numpy()
            H.close()
        out[name] = r
        print(f"[bench] {name}: FP32-preconditioned {r['fp32']['iters']} iterations {r['fp32']['ms_per_solve']:.2f} "
              f"ms, FP64 {r['fp64']['iters']} iterations {r['fp64']['ms_per_solve']:.2f} ms", file=sys.stderr,
              flush=True)
    return out, sols


def run_options(steps, smoother):
    """Coefficient-aware extensions and essential boundary conditions (the library's
    builder options) on the 32^3 H(div) jump workload and on two of the serving mix's
    48^3 jump hierarchies: FP64 PCG iterations to rtol 1e-8 and time per solve, with the
    headline's point smoother."""
    import torch
    from paper_2107_05613_amd import amge
    from paper_2107_05613_amd import workloads as W
    cases = [W.WORKLOADS["div_n32_l4_jumps"],
             W.Workload("curl_n48_c0", "curl", 48, W.default_levels(48), "blocks", coef_seed=0),
             W.Workload("div_n48_c0", "div", 48, W.default_levels(48), "blocks", coef_seed=0)]
    out = {}
    for w in cases:
        a, b = W.coefficients(w)
        r = {}
        for ext in ("l2", "coefficient"):
            for bc in ("natural", "essential"):
                prod = amge.build_problem(w.kind, w.n, w.levels, a, b, extension=ext, bc=bc)
                H = amge.Hierarchy(prod, precond_bits=64, smoother=smoother)
                rhs = torch.from_numpy(W.rhs(H.rows[0], w.rhs_seed)[:, 0]).cuda()
                x = torch.zeros_like(rhs)
                st, it, rr = H.pcg(rhs, x, rtol=1e-8, maxit=2000)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(max(1, steps // 5)):
                    H.pcg(rhs, x, rtol=1e-8, maxit=2000)
                torch.cuda.synchronize()
                dt = (time.perf_counter() - t0) / max(1, steps // 5)
                r[f"{ext}/{bc}"] = {"iters": it[0], "status": st, "dofs": H.rows[0], "ms_per_solve": 1e3 * dt}
                H.close()
        out[w.name] = r
        out["smoother"] = smoother
        print(f"[bench] options {w.name}: " + ", ".join(f"{k} {v['iters']}" for k, v in r.items()),
              file=sys.stderr, flush=True)
    return out


def run_smoother(w, prod, rhs, steps, smoother):
    """The same solve with another point smoother in the hybrid smoother: iterations, time
    per solve and V-cycle time, FP32 and FP64 V-cycles."""
    import torch
    from paper_2107_05613_amd import amge
    out = {}
    for bits in (32, 64):
        t0 = time.perf_counter()
        H = amge.Hierarchy(prod, precond_bits=bits, smoother=smoother)
        t_setup = time.perf_counter() - t0
        x = torch.zeros_like(rhs)
        for _ in range(2):
            st, it, rr = H.pcg(rhs, x, rtol=w.rtol, maxit=1000)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            st, it, rr = H.pcg(rhs, x, rtol=w.rtol, maxit=1000)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        z = torch.empty_like(rhs)
        H.vcycle(rhs, z)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            H.vcycle(rhs, z)
        e1.record()
        torch.cuda.synchronize()
        out[f"fp{bits}"] = {"iters": it[0], "status": st, "ms_per_solve": 1e3 * dt, "solves_per_s": 1.0 / dt,
                            "vcycle_ms": e0.elapsed_time(e1) / 10, "setup_s": t_setup}
        H.close()
    print(f"[bench] smoother {smoother}: FP32 {out['fp32']['iters']} iterations "
          f"{out['fp32']['ms_per_solve']:.2f} ms, FP64 {out['fp64']['iters']} iterations "
          f"{out['fp64']['ms_per_solve']:.2f} ms", file=sys.stderr, flush=True)
    return out


def cold_sweep(H, rhs, x, reps=10):
    """Average time of the fine-level FP32 sweep of the point smoother launched alone
    (amge_level_apply SWEEP: a block Gauss-Seidel sweep from x, or an l1-Jacobi sweep; HIP
    events on its stream), warm (launched back to back, its matrix partly
    served by the last-level cache) and cold (after a 2 GiB device copy that evicts the
    256 MB last-level cache, so the matrix streams from HBM)."""
    import torch
    from paper_2107_05613_amd import amge
    out = torch.empty_like(rhs)
    src = torch.ones(1 << 29, dtype=torch.float32, device="cuda")   # 2 GiB
    dst = torch.empty_like(src)
    res = {}
    for name, flush in (("warm", False), ("cold", True)):
        H.level_apply(0, amge.OP_SWEEP, rhs, out, x2=x, precision=32)
        torch.cuda.synchronize()
        H.timing_enable(True)
        for _ in range(reps):
            if flush:
                dst.copy_(src)
            H.level_apply(0, amge.OP_SWEEP, rhs, out, x2=x, precision=32)
        torch.cuda.synchronize()
        ms, n, by = H.timing_read()
        H.timing_enable(False)
        res[name] = (ms / max(n, 1), by / max(n, 1))
    del src, dst
    torch.cuda.empty_cache()
    return res


def _by_class(mix, lat, order=None):
    """p50/p99 latency per size class n."""
    from paper_2107_05613_amd import serve
    out = {}
    for n in sorted({r["n"] for r in mix.requests}):
        sub = {j: v for j, v in lat.items() if mix.requests[j]["n"] == n}
        if sub:
            st = serve.latency_stats(sub)
            out[str(n)] = {"requests": len(sub), "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"]}
    return out


def run_serving(args):
    """Serving mix: seeded requests over 20 resident hierarchies (H(curl)/H(div),
    n in {16,24,32,48,64}, two coefficient-jump fields each), 8 columns per hierarchy,
    V-cycle precision chosen per hierarchy at set-up (trial solves).  All requests at once
    (burst), a closed loop with two outstanding requests per hierarchy (capacity), Poisson
    arrivals at 0.8 x and 0.4 x that capacity (open loop: p50/p99 overall and per size
    class); and the burst again with every hierarchy in FP64 (the FP32 ones rebuilt)."""
    import numpy as np
    import torch
    from paper_2107_05613_amd import amge, serve
    from paper_2107_05613_amd import workloads as W
    t0 = time.perf_counter()
    mix = serve.build_mix(num=args.serving_requests, seed=0, slots=args.serving_slots, precond_bits=0,
                          extension=args.serving_extension, smoother=batched_smoother(args))
    print(f"[bench] serving: {len(mix.keys)} hierarchies built in {time.perf_counter() - t0:.1f}s "
          f"(build {mix.build_s:.1f}s, device setup {mix.setup_s:.1f}s)", file=sys.stderr, flush=True)
    srv, ids = serve.make_server(mix, chunk=8)
    resident = srv.stats()["resident_bytes"]
    prec = [h.precision_info() for h in mix.hierarchies]
    fp32_keys = [k for k, (_, b) in zip(mix.keys, prec) if b == 32]
    resid64_keys = [k for k, (_, b), h in zip(mix.keys, prec, mix.hierarchies) if b == 32 and h.resid_bits() == 64]
    # warm-up: one request per hierarchy
    first = {}
    for j, h in enumerate(mix.hid_of):
        first.setdefault(h, j)
    serve.run(srv, ids, mix, order=list(first.values()))
    # burst: every request at t = 0 (columns as full as the stream allows)
    done, lat, makespan = serve.run(srv, ids, mix)
    burst = len(done) / makespan
    burst_by = _by_class(mix, lat)
    bad = sum(1 for v in done.values() if v[0] != 0)
    print(f"[bench] serving burst: {burst:.1f} solves/s ({makespan:.2f}s for {len(done)}; "
          f"{len(fp32_keys)} of {len(prec)} hierarchies FP32)", file=sys.stderr, flush=True)
    # closed loop: two requests per resident hierarchy outstanding on average
    conc = 2 * len(mix.keys)
    donec, latc, makespanc = serve.run_closed(srv, ids, mix, conc)
    capacity = len(donec) / makespanc
    bad += sum(1 for v in donec.values() if v[0] != 0)
    print(f"[bench] serving closed loop ({conc} outstanding): {capacity:.1f} solves/s", file=sys.stderr, flush=True)
    open_loop = {}
    iters = []
    for frac, num in ((0.8, len(mix.requests)), (0.4, len(mix.requests) // 2)):
        rate = frac * capacity
        order = list(range(num))
        arrivals = np.array([mix.requests[j]["t_arrive"] for j in order]) / rate
        d2, l2, mk2 = serve.run(srv, ids, mix, arrivals=arrivals, order=order)
        st = serve.latency_stats(l2)
        bad += sum(1 for v in d2.values() if v[0] != 0)
        iters += [v[1] for v in d2.values()]
        open_loop[f"{frac}x_capacity"] = {"arrival_rate_per_s": rate, "requests": num,
                                           "solves_per_s": len(d2) / mk2, **st, "by_size": _by_class(mix, l2)}
        print(f"[bench] serving open loop at {rate:.1f}/s: p50 {st['p50_ms']:.1f} ms p99 {st['p99_ms']:.1f} ms",
              file=sys.stderr, flush=True)
    srv.close()
    # the burst with every hierarchy in FP64: rebuild the FP32 ones
    fp64 = list(mix.hierarchies)
    rebuilt = []
    for i, (key, (_, b)) in enumerate(zip(mix.keys, prec)):
        if b == 32:
            kind, n, cs = key
            w = W.Workload(f"{kind}_n{n}_c{cs}", kind, n, W.default_levels(n), "blocks", coef_seed=cs)
            a, be = W.coefficients(w)
            fp64[i] = amge.Hierarchy(amge.build_problem(kind, n, w.levels, a, be, extension=args.serving_extension,
                                                        device=True), precond_bits=64, max_rhs=args.serving_slots,
                                     smoother=batched_smoother(args))
            rebuilt.append(fp64[i])
    mix64 = serve.Mix(mix.requests, mix.keys, fp64, mix.hid_of, mix.rhs, mix.x)
    srv64, ids64 = serve.make_server(mix64, chunk=8)
    serve.run(srv64, ids64, mix64, order=list(first.values()))
    d64, l64, mk64 = serve.run(srv64, ids64, mix64)
    burst64 = len(d64) / mk64
    bad += sum(1 for v in d64.values() if v[0] != 0)
    srv64.close()
    for H in rebuilt:
        H.close()
    print(f"[bench] serving burst, all FP64: {burst64:.1f} solves/s", file=sys.stderr, flush=True)
    mix_desc = {"requests": mix.requests, "keys": len(mix.keys),
                "setup_s": {"build": mix.build_s, "device_setup": mix.setup_s}}
    del mix, mix64
    torch.cuda.synchronize()
    grouped = run_grouped_ab()
    out = {
        "workload": (f"{len(mix_desc['requests'])} seeded requests, H(curl)/H(div) on n^3x6 Kuhn tets with n in "
                     f"{{16,24,32,48,64}} drawn uniformly, per-4^3-block coefficient jumps 10^U(-3,3) from a pool "
                     f"of 2 seeds per (type, n): {mix_desc['keys']} resident hierarchies, {args.serving_slots} PCG "
                     f"columns each; "
                     f"V-cycle precision per hierarchy from trial solves at set-up, per-column FP64 PCG "
                     f"to rel-res 1e-8; local extensions: {args.serving_extension}; smoother "
                     f"{SMOOTHER_NAMES[batched_smoother(args)]}"),
        "precision": {"fp32_hierarchies": len(fp32_keys), "fp64_hierarchies": len(prec) - len(fp32_keys),
                      "fp32": [f"{k[0]} n={k[1]} seed {k[2]}" for k in fp32_keys],
                      "fp32_with_fp64_fine_residual": [f"{k[0]} n={k[1]} seed {k[2]}" for k in resid64_keys],
                      "kappa_range": [min(k for k, b in prec), max(k for k, b in prec)]},
        "resident_bytes": resident,
        "burst": {"solves_per_s": burst, "makespan_s": makespan, **serve.latency_stats(lat), "by_size": burst_by},
        "burst_all_fp64": {"solves_per_s": burst64, "makespan_s": mk64, **serve.latency_stats(l64)},
        "closed_loop": {"outstanding": conc, "solves_per_s": capacity, **serve.latency_stats(latc)},
        "open_loop": open_loop,
        "iters": [int(min(iters)), int(max(iters))],
        "failed_requests": bad,
        "setup_s": mix_desc["setup_s"],
        "persistent_launches": ("not built: a grid-wide barrier of a cooperative kernel measured 27 us at 256 "
                                "workgroups (110 us at 1024), against 1.7-2.1 us for a dependent launch in a HIP "
                                "graph, so a persistent kernel stepping through the V-cycle's operators would be "
                                "slower than the grouped and solo launches"),
        "grouped_launches": grouped,
    }
    return out


def stream_reference(nbytes=1 << 30, reps=10):
    """Bandwidth this GPU reaches on a plain stream: a 1 GiB device copy (torch, read +
    write bytes, HIP events on torch's stream)."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    out = {}
    for name, fn, moved in (("copy", lambda: dst.copy_(src), 2 * nbytes),):
        for _ in range(3):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name] = moved / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return out


GROUPED_CONFIGS = (("solo", 0, 1), ("grouped", 16, 1), ("grouped_4_ensembles", 16, 4))


def run_grouped_ab(only=None):
    """Solo streams vs grouped launches (one ensemble, and four ensembles on their own
    streams) on 16 resident 16^3 hierarchies (both types, 8 coefficient fields), 128
    requests at once, 8 columns each.  only: run that configuration alone."""
    from paper_2107_05613_amd import serve
    mix = serve.build_mix(num=128, seed=0, sizes=(16,), coef_pool=8, slots=8, precond_bits=0)
    first = {}
    for j, h in enumerate(mix.hid_of):
        first.setdefault(h, j)
    out = {"workload": f"{len(mix.requests)} requests at once on {len(mix.keys)} resident 16^3 hierarchies "
                       f"(H(curl)/H(div), 8 coefficient-jump fields each), 8 columns each"}
    for name, gmax, ens in GROUPED_CONFIGS:
        if only and name != only:
            continue
        srv, ids = serve.make_server(mix, chunk=8, grouped_max_n=gmax, ensembles=ens)
        serve.run(srv, ids, mix, order=list(first.values()))
        done, lat, mk = serve.run(srv, ids, mix)
        members, launches, solo_launches = srv.ensemble()
        srv.close()
        r = {"solves_per_s": len(done) / mk, **serve.latency_stats(lat),
             "failed_requests": sum(1 for v in done.values() if v[0] != 0)}
        if gmax:
            r.update(members=members, kernels_per_iteration=launches, kernels_alone=solo_launches)
        out[name] = r
        print(f"[bench] {name} small-hierarchy burst: {r['solves_per_s']:.1f} solves/s", file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="curl_n64_l5")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batched-workload", default="div_n48_l5_rhs32",
                    help="multi-right-hand-side workload timed beside the main one ('' to skip)")
    ap.add_argument("--serving-requests", type=int, default=256,
                    help="requests of the serving mix run beside the main workload (0 to skip)")
    ap.add_argument("--serving-extension", choices=("l2", "coefficient"), default="coefficient",
                    help="extension of the serving hierarchies' local problems (remark closing section 3.3): "
                         "coefficient-weighted (default) or unweighted L2")
    ap.add_argument("--serving-slots", type=int, default=8, help="PCG columns per serving hierarchy")
    ap.add_argument("--cpu-baseline-worker", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--oracle-dir", default=None)
    ap.add_argument("--smoother", choices=("l1blockgs", "l1jacobi", "symgs"), default="l1blockgs",
                    help="point smoother of the headline solve (section 4.1): l1-scaled symmetric block "
                         "Gauss-Seidel (default), l1-Jacobi, or symmetric Gauss-Seidel in colour order")
    ap.add_argument("--no-gs", action="store_true", help="skip the solves with the other point smoothers")
    ap.add_argument("--no-options", action="store_true",
                    help="skip the extension / boundary-condition option comparison")
    ap.add_argument("--small-configs", default="curl_n8_l2,div_n32_l4_jumps",
                    help="comma-separated small configurations timed beside the main one ('' to skip)")
    ap.add_argument("--grouped-ab-only", choices=[c[0] for c in GROUPED_CONFIGS],
                    help="run only that configuration of the small-hierarchy serving burst and print its JSON "
                         "(for kernel traces)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 1 GiB device copy first (reference kernel for HBM counters)")
    args = ap.parse_args()

    if args.cpu_baseline_worker:
        cpu_baseline_worker(args.workload.split(","), args.cpu_budget, args.oracle_dir, args.smoother)
        return 0
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one MI355X: the solve phase is not sharded across GPUs "
              "(run with --gpus 1)", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    from paper_2107_05613_amd import amge
    from paper_2107_05613_amd import workloads as W

    if args.grouped_ab_only:
        print(json.dumps(run_grouped_ab(only=args.grouped_ab_only)), flush=True)
        return 0

    w = W.WORKLOADS[args.workload]
    a, b = W.coefficients(w)
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    torch.zeros(1, device="cuda")
    torch.cuda.synchronize()
    # set-up: the level matrices built with the GPU steps of the builder (Galerkin products
    # on the device), the host-only build timed beside it; then the device hierarchies
    t0 = time.perf_counter()
    prod = amge.build_problem(w.kind, w.n, w.levels, a, b, device=True)
    t_build = time.perf_counter() - t0
    t0 = time.perf_counter()
    amge.build_problem(w.kind, w.n, w.levels, a, b)
    t_build_host = time.perf_counter() - t0
    t0 = time.perf_counter()
    H32 = amge.Hierarchy(prod, precond_bits=32, smoother=args.smoother)
    torch.cuda.synchronize()
    t_setup32 = time.perf_counter() - t0
    H64 = amge.Hierarchy(prod, precond_bits=64, smoother=args.smoother)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    n1 = H32.rows[0]
    rhs = torch.from_numpy(W.rhs(n1, w.rhs_seed)[:, 0]).cuda()
    x32 = torch.zeros_like(rhs)
    x64 = torch.zeros_like(rhs)
    print(f"[bench] {w.name}: n1={n1} levels={H32.rows} build {t_build:.1f}s setup {t_setup:.1f}s",
          file=sys.stderr, flush=True)

    def solve(H, x):
        st, it, rr = H.pcg(rhs, x, rtol=w.rtol, maxit=1000)
        if st != 0:
            raise RuntimeError("solve did not converge")
        return it[0], rr[0]

    # ---- FP32-preconditioned PCG (the product path: graph-captured iterations)
    for _ in range(args.warmup):
        solve(H32, x32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        it32, rr32 = solve(H32, x32)
    torch.cuda.synchronize()
    dt32 = time.perf_counter() - t0
    print(f"[bench] fp32-precond: {it32} iters, {1e3 * dt32 / args.steps:.2f} ms/solve", file=sys.stderr, flush=True)
    # ---- dominant kernel family: fine-level A launches of the same solves, bracketed by
    # HIP events on their launch stream (timing on launches the iterations directly)
    H32.timing_enable(True)
    for _ in range(max(1, min(args.steps, 3))):
        solve(H32, x32)
    torch.cuda.synchronize()
    k_ms, k_launches, k_bytes = H32.timing_read()
    H32.timing_enable(False)
    sweep = cold_sweep(H32, rhs, x32)

    # ---- plain FP64 PCG on the same hierarchy
    for _ in range(max(1, args.warmup)):
        solve(H64, x64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        it64, rr64 = solve(H64, x64)
    torch.cuda.synchronize()
    dt64 = time.perf_counter() - t0
    print(f"[bench] fp64: {it64} iters, {1e3 * dt64 / args.steps:.2f} ms/solve", file=sys.stderr, flush=True)

    # ---- V-cycle bandwidth (FP32 and FP64), device time by events on the launch stream
    z = torch.empty_like(rhs)
    vc = {}
    for bits, H in ((32, H32), (64, H64)):
        for _ in range(3):
            H.vcycle(rhs, z)
        reps = 20
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            H.vcycle(rhs, z)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        by = H.vcycle_bytes(bits, nrhs=1)
        vc[bits] = (ms, by, by / (ms * 1e-3) / 1e9)
    err = float(torch.linalg.norm(x32 - x64) / torch.linalg.norm(x64))

    sol = {(w.name, 32): x32.cpu().numpy(), (w.name, 64): x64.cpu().numpy()}
    lv0 = prod[0][0]
    del H64
    others = {sm: run_smoother(w, prod, rhs, args.steps, sm)
              for sm in ("l1jacobi", "symgs", "l1blockgs") if sm != args.smoother} if not args.no_gs else None
    stream_ref = stream_reference()
    small_names = [c for c in args.small_configs.split(",") if c]
    small, small_sol = run_small_configs(small_names, args.steps, args.smoother) if small_names else ({}, {})
    sol.update(small_sol)
    options = run_options(args.steps, args.smoother) if not args.no_options else None
    batched = run_batched(args, amge, W) if args.batched_workload else None
    serving = run_serving(args) if args.serving_requests > 0 else None

    value = args.steps / dt32
    k_avg_ms = k_ms / max(k_launches, 1)
    k_gbps = (k_bytes / max(k_launches, 1)) / (k_avg_ms * 1e-3) / 1e9 if k_launches else 0.0
    # byte model of the scope table (32-bit column indices, one FP32 value per entry,
    # rows + 1 row pointers, four vector streams of the sweep: x, b, d, y)
    model_bytes = 8.0 * lv0.nnz + 4.0 * (n1 + 1) + 16.0 * n1

    def gbps(by, ms):
        return by / (ms * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt32 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"{w.name}: H({w.kind}) lowest-order "
                         f"{'Nedelec' if w.kind == 'curl' else 'Raviart-Thomas'} on {w.n}^3x6 Kuhn tets, "
                         f"{w.levels}-level AMGe (2x2x2 agglomerates), hybrid smoother 2+2 sweeps with "
                         f"{SMOOTHER_NAMES[args.smoother]}, "
                         f"FP32 V-cycle in FP64 inexact PCG to rel-res {w.rtol:g} (preconditioner norm)"),
            "fine_dofs": n1,
            "level_rows": H32.rows,
            "rhs": f"uniform[-1,1] seed {w.rhs_seed}",
            "coefficients": w.coef,
        },
        "dtype_detail": "V-cycle values and accumulation FP32; outer PCG, dots and coarsest Cholesky FP64",
        "iters_fp32_precond": it32,
        "iters_fp64": it64,
        "relres_fp32_precond": rr32,
        "fp64_solves_per_s": args.steps / dt64,
        "speedup_fp32_vs_fp64": (args.steps / dt32) / (args.steps / dt64),
        "solution_rel_diff_fp32_vs_fp64": err,
        "vcycle": {
            "fp32": {"ms": vc[32][0], "algorithmic_bytes": vc[32][1], "GBps": vc[32][2]},
            "fp64": {"ms": vc[64][0], "algorithmic_bytes": vc[64][1], "GBps": vc[64][2]},
        },
        "roofline": {
            "bound": "hbm",
            "kernel": ROOFLINE_KERNELS[args.smoother],
            "achieved": k_gbps,
            "peak": PEAK_HBM_GBPS,
            "unit": "GB/s",
            "frac": k_gbps / PEAK_HBM_GBPS,
            "traffic": measured_traffic(args.smoother),
            "avg_launch_us": 1e3 * k_avg_ms,
            "bytes_per_launch": k_bytes / max(k_launches, 1),
            "launches": k_launches,
            "model_bytes_per_launch": model_bytes,
            "frac_model": gbps(model_bytes, k_avg_ms) / PEAK_HBM_GBPS,
            "sweep_alone": {
                name: {"avg_launch_us": 1e3 * ms_, "achieved": gbps(by_, ms_), "frac": gbps(by_, ms_) / PEAK_HBM_GBPS,
                       "frac_model": gbps(model_bytes, ms_) / PEAK_HBM_GBPS}
                for name, (ms_, by_) in sweep.items()},
            "cold_note": ("sweep_alone.cold: the same FP32 sweep launched after a 2 GiB device copy that evicts "
                          "the 256 MB last-level cache (its matrix streams from HBM); warm: launched back to back"),
            "stream_reference_GBps": stream_ref,
        },
        "smoother": args.smoother,
        "other_smoothers": others,
        "configs": small,
        "extension_and_boundary_options": options,
        "setup_s": {"build": t_build, "build_host_only": t_build_host, "device_setup": t_setup,
                    "device_setup_fp32_hierarchy": t_setup32,
                    "note": ("build: level matrices with the builder's GPU steps (AMGE_BUILD_DEVICE); "
                             "device_setup: the FP32- and FP64-V-cycle hierarchies (layouts filled on the "
                             "device, set-up products on the device, tuning)")},
        "batched": batched,
        "serving": serving,
    }
    if not args.no_cpu_baseline:
        import shutil
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        ores, odir = run_cpu_baseline([args.workload] + small_names, args.cpu_budget, args.smoother)
        if "error" in ores:
            out["cpu_baseline"] = ores
        else:
            out["cpu_baseline"] = baseline_entry(ores[args.workload], it64)
            out["cpu_baseline"]["host_cores_available"] = ores["cores"]

            def err_vs_oracle(name, bits):
                xo = np.load(os.path.join(odir, f"{name}.npy"))
                return float(np.linalg.norm(sol[(name, bits)] - xo) / np.linalg.norm(xo))
            out["solution_rel_err_vs_oracle"] = {"fp32_precond": err_vs_oracle(args.workload, 32),
                                                 "fp64": err_vs_oracle(args.workload, 64),
                                                 "oracle_iters": ores[args.workload]["oracle_iters"]}
            for name in small_names:
                r = out["configs"][name]
                r["oracle_iters"] = ores[name]["oracle_iters"]
                for bits in (32, 64):
                    r[f"fp{bits}"]["rel_err_vs_oracle"] = err_vs_oracle(name, bits)
                r["cpu_baseline"] = baseline_entry(ores[name], ores[name]["oracle_iters"])
        shutil.rmtree(odir, ignore_errors=True)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
