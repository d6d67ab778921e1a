#!/usr/bin/env python3
"""Benchmark: adaptive sampled betweenness (time to epsilon) on one MI355X.

One step = one whole adaptive run through the C ABI (kad_run): vertex-diameter rule,
pilot samples, computeDelta, then batches of sampled shortest paths (balanced
bidirectional BFS, uniform path, interior hits) with the stopping rule checked every
interval, on a graph already resident in HBM.

Workload (default): undirected Chung-Lu graph, n = 1,000,000, power-law exponent 2.3,
mean degree 20 (2.0e7 arcs), uint32 CSR; all-nodes task, epsilon = 0.005, delta = 0.1,
seed 1, 65,536 samples per sampler launch.

Other workloads (--workload):
  er2000    the same run on G(2000, 8/1999)'s largest component, epsilon 0.01;
  dcl4m     directed Chung-Lu, n = 4,000,000, out/in exponents 2.5/2.1, mean degree 15,
            top-k with k = 50, epsilon 0.0002 (the paper's top-k setting), launch shape
            autotuned before the timed steps;
  batch256  256 Chung-Lu graphs (seed 1000+i; n log-uniform in [1e3, 1e5], half directed,
            exponents in [2.1, 2.8], mean degree 4..30), epsilon 0.01, delta 0.1, seed 1:
            one step = all 256 adaptive runs through the multi-query engine
            (kad_run_batch); the same 256 runs one after another through kad_run are
            timed beside it, and the results are checked identical.
  exponent  Theorem 2 / Fig. 2: arcs visited per sampled path with the balanced search and
            with the forward BFS from s, on the appendix's random-graph models (Chung-Lu,
            configuration model, Norros-Reittu, generalized random graph; --models) with
            power-law exponents --betas at mean degree --mean-degree, n in --sizes; fits
            arcs ~ n^alpha per model, exponent and search (value = mean balanced alpha).
  serve     the serving workload: 33 resident graphs (er2000, cl1m, 30 Chung-Lu graphs of
            1e4..1e6 nodes, the 2000x2000 grid with 5% of edges deleted), a Poisson stream
            of --queries queries at --rate per second (seed 7), each on a uniformly drawn
            graph, all-nodes or top-k (k in {10, 100}) with epsilon uniform in
            [0.002, 0.02], delta 0.1, through kad_server_*.  Latency = submit to result,
            measured by the server.  Queries still running --drain seconds after the
            last arrival are canceled and counted with their age as a lower bound.

Prints one JSON line.  value = sampled shortest paths per second over the timed steps
(pilot + main-phase samples that enter the result; samples computed past the stopping
point of the last batch are not counted).  roofline = the sampler kernel's algorithmic
bytes per launch over its event-timed average launch duration, against 8 TB/s.
cpu_baseline = the CPU oracle beside it: for cl1m and er2000 its whole adaptive run on the
same graph and parameters (time to epsilon, paths/s, and whether its result equals the
GPU's), plus its one-thread sampling rate; for the other workloads its sampling rate on
a bounded prefix of sample ids.  time_to_epsilon_cold_s = a graph registered anew and its
first run (vertex diameter included) on the warm context.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD_TEXT = {"cl1m": "undirected Chung-Lu, beta 2.3, mean degree 20",
                 "er2000": "G(2000, 8/1999) seed 1, largest component",
                 "dcl4m": "directed Chung-Lu, out beta 2.5, in beta 2.1, mean degree 15",
                 "grid2000": "2000x2000 grid, 5% of edges deleted"}
def measured_traffic(workload, kernel="sampler_kernel"):
    """Bytes per dispatch of `kernel` below the L2 (FETCH_SIZE + WRITE_SIZE, scaled by a
    plain copy) from the committed counter passes, if they were taken on this workload with
    the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles",
                        f"{kernel.replace('_kernel', '')}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    from paper_1604_08553_amd.profiling import kernel_source_sha256
    rec = json.load(open(path))
    if rec.get("kernel_source_sha256") != kernel_source_sha256():
        return None
    return rec.get("l2_egress_bytes_per_dispatch", rec.get("hbm_bytes_per_dispatch"))


def algorithmic_bytes(arcs, nodes, hits):
    """Bytes the method must touch: 4 B neighbour id + 1 bit visited probe per scanned
    arc, 26 B per reached node (8 B row bounds, 16 B path count, 2 B level), 4 B per hit."""
    return 4.125 * arcs + 26.0 * nodes + 4.0 * hits


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def host_threads():
    return int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1


def cpu_baseline_run(csr, kw, gpu, one_thread_samples):
    """The oracle's whole adaptive run on the same graph and parameters (all host threads):
    its time to epsilon and sampling rate, and whether its result equals the GPU's; plus the
    oracle's sampling rate on one thread over a prefix of main-phase ids."""
    import numpy as np
    import oracle
    threads = host_threads()
    okw = {k: v for k, v in kw.items() if k != "kernel_batch"}
    t0 = time.perf_counter()
    r = oracle.run(csr, threads=threads, **okw)
    dt = time.perf_counter() - t0
    parity = bool(r["tau"] == gpu["tau"] and r["stop_rule"] == gpu["stop_reason"]
                  and r["arcs"] == gpu["arcs_scanned"]
                  and np.array_equal(r["count"], gpu["count"])
                  and np.array_equal(r["lower"], gpu["lower"])
                  and np.array_equal(r["upper"], gpu["upper"]))
    paths = r["alpha"] + r["tau"]
    t1 = time.perf_counter()
    S = oracle.sample_paths(csr, kw["seed"], 1, 0, one_thread_samples, threads=1)
    dt1 = time.perf_counter() - t1
    return {"value": paths / dt, "unit": "sampled shortest paths/s", "cores": threads,
            "kind": "oracle", "cpu_model": cpu_model(),
            "time_to_epsilon_s": dt, "gteps": (r["arcs"] + r["pilot_arcs"]) / dt / 1e9,
            "parity": parity, "tau": int(r["tau"]),
            "one_thread": {"value": one_thread_samples / dt1, "unit": "sampled shortest paths/s",
                           "gteps": float(S.arcs.sum()) / dt1 / 1e9,
                           "sample": f"main-phase ids 0..{one_thread_samples - 1}"},
            "sample": f"the oracle's whole adaptive run on the same graph and parameters "
                      f"(vertex diameter, pilot, computeDelta, {paths} samples; {dt:.1f} s), "
                      "all host threads; result compared with the GPU's"}


def cpu_baseline(csr, samples, seed):
    """The oracle's sampling rate over main-phase ids [0, samples) (all host threads)."""
    import oracle
    threads = host_threads()
    t0 = time.perf_counter()
    S = oracle.sample_paths(csr, seed, 1, 0, samples, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": samples / dt, "unit": "sampled shortest paths/s", "cores": threads,
            "kind": "oracle", "cpu_model": cpu_model(), "gteps": float(S.arcs.sum()) / dt / 1e9,
            "sample": f"oracle sample_paths: main-phase ids 0..{samples - 1}, seed {seed}, "
                      f"same graph ({dt:.1f} s)"}


def cpu_baseline_family(csrs, kw, gpu_results, stride=16):
    """The oracle's whole adaptive runs on every stride-th query of a batch (all host
    threads, one after another): their sampling rate and time to epsilon, scaled to the
    whole batch by sampled paths, and whether each result equals the GPU's."""
    import numpy as np
    import oracle
    threads = host_threads()
    picks = list(range(0, len(csrs), stride))
    t0 = time.perf_counter()
    paths, parity = 0, True
    for i in picks:
        r = oracle.run(csrs[i], threads=threads, **kw)
        g = gpu_results[i]
        paths += r["alpha"] + r["tau"]
        parity &= bool(r["tau"] == g["tau"] and np.array_equal(r["count"], g["count"])
                       and np.array_equal(r["lower"], g["lower"])
                       and np.array_equal(r["upper"], g["upper"]))
    dt = time.perf_counter() - t0
    total = sum(r["alpha"] + r["tau"] for r in gpu_results)
    return {"value": paths / dt, "unit": "sampled shortest paths/s", "cores": threads,
            "kind": "oracle", "cpu_model": cpu_model(), "parity": parity,
            "time_to_epsilon_whole_batch_s_estimate": dt * total / max(paths, 1),
            "sample": f"the oracle's whole runs of queries {picks[0]}, {picks[0] + stride}, ... "
                      f"({len(picks)} of {len(csrs)}; {paths} samples, {dt:.1f} s), all host "
                      "threads, results compared with the GPU's; the whole-batch time is "
                      "scaled by sampled paths"}


def cpu_baseline_serve(csrs, Gs, ctx, stream, grid_id, kad, per_graph=2000, grid_samples=4):
    """The oracle's sampling rate over the resident graphs: on each, main-phase ids
    0..per_graph-1 under the seed of the graph's first query (grid_samples ids on the grid,
    whose samples reach about 1.35M nodes with counts of hundreds of bits), all host
    threads; the GPU's paths for the same ids (kad_sample_paths) compared with them."""
    import numpy as np
    import oracle
    threads = host_threads()
    seeds = {}
    for q in stream:
        seeds.setdefault(q["graph"], q["seed"])
    total, arcs, dt, parity = 0, 0, 0.0, True
    for i, g in csrs.items():
        cnt = grid_samples if i == grid_id else per_graph
        seed = seeds.get(i, 1)
        t0 = time.perf_counter()
        S = oracle.sample_paths(g, seed, 1, 0, cnt, threads=threads)
        dt += time.perf_counter() - t0
        total += cnt
        arcs += int(S.arcs.sum())
        A = kad.sample_paths(ctx, Gs[i], seed, 1, 0, cnt)
        parity &= bool((A["flags"] == 0).all() and np.array_equal(A["s"], S.s)
                       and np.array_equal(A["t"], S.t) and np.array_equal(A["arcs"], S.arcs)
                       and np.array_equal(A["path_off"], S.path_off)
                       and np.array_equal(A["nodes"], S.nodes))
    return {"value": total / dt, "unit": "sampled shortest paths/s", "cores": threads,
            "kind": "oracle", "cpu_model": cpu_model(), "gteps": arcs / dt / 1e9,
            "parity": parity,
            "sample": f"oracle sample_paths on each of the {len(csrs)} resident graphs: main-phase "
                      f"ids 0..{per_graph - 1} under the seed of its first query ({grid_samples} "
                      f"on the grid); {total} samples, {dt:.1f} s, all host threads; the GPU's "
                      "paths for the same ids compared"}


def _same_result(a, b):
    import numpy as np
    return (a["tau"] == b["tau"] and a["stop_reason"] == b["stop_reason"]
            and np.array_equal(a["count"], b["count"]) and np.array_equal(a["lower"], b["lower"])
            and np.array_equal(a["upper"], b["upper"]))


def bench_batch(args, torch, gg, kad):
    """256-graph family: engine (one step = one kad_run_batch of all queries) against
    the same queries run one after another with kad_run, in its default launch mode
    (recorded batch chains) and on the plain single-graph path."""
    ngraphs = 256
    t0 = time.perf_counter()
    csrs = [gg.batch_graph(i) for i in range(ngraphs)]
    print(f"[bench] {ngraphs} graphs: {sum(g.n for g in csrs)} nodes, "
          f"{sum(g.arcs for g in csrs)} arcs ({time.perf_counter() - t0:.1f} s)",
          file=sys.stderr, flush=True)
    ctx = kad.Context(0)
    Gs = [kad.Graph(ctx, g) for g in csrs]
    eps = args.epsilon
    kw = dict(epsilon=eps, delta=args.delta, seed=args.seed)
    params = [dict(kw) for _ in Gs]
    for w in range(args.warmup):
        kad.run_batch(ctx, Gs, params)
        for mode in ("graph", "plain"):
            ctx.set_exec(mode)
            for G in Gs:
                kad.run(ctx, G, **kw)
        ctx.set_exec("graph")
        print(f"[bench] warmup {w} done", file=sys.stderr, flush=True)
    # sequential single runs: recorded batch chains, then the plain single-graph path
    seq = {}
    for mode in ("graph", "plain"):
        ctx.set_exec(mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(args.steps):
            runs_m = [kad.run(ctx, G, **kw) for G in Gs]
        torch.cuda.synchronize()
        seq[mode] = ((time.perf_counter() - t0) / args.steps, runs_m)
        print(f"[bench] sequential kad_run ({mode}): {seq[mode][0]:.3f} s per pass",
              file=sys.stderr, flush=True)
    ctx.set_exec("graph")
    seq_s, single = seq["graph"]
    plain_s, plain = seq["plain"]
    # the engine: ticks launched call by call, then replayed as recorded chains (default)
    ctx.set_exec("stream")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        batch_s = kad.run_batch(ctx, Gs, params)
    torch.cuda.synchronize()
    engine_stream_s = (time.perf_counter() - t0) / args.steps
    ctx.set_exec("graph")
    r0 = ctx.exec_info()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        batch = kad.run_batch(ctx, Gs, params)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    step_s = elapsed / args.steps
    r1 = ctx.exec_info()
    print(f"[bench] kad_run_batch call by call: {engine_stream_s:.3f} s; replayed: {step_s:.3f} s",
          file=sys.stderr, flush=True)
    # the engine's sampler launches timed by events, in one further step
    ctx.set_timing(True)
    t1 = time.perf_counter()
    kad.run_batch(ctx, Gs, params)
    torch.cuda.synchronize()
    timed_elapsed = time.perf_counter() - t1
    tm = ctx.timing()
    ctx.set_timing(False)
    print(f"[bench] kad_run_batch: {step_s:.3f} s per step", file=sys.stderr, flush=True)
    identical = all(_same_result(a, b) for a, b in zip(batch, single)) and \
        all(_same_result(a, b) for a, b in zip(plain, single)) and \
        all(_same_result(a, b) for a, b in zip(batch_s, single))
    paths = sum(r["alpha"] + r["tau"] for r in batch)
    arcs = sum(r["arcs_scanned"] + r["pilot_arcs_scanned"] for r in batch)
    alg = algorithmic_bytes(tm["arcs"], tm["nodes"], tm["hits"])
    avg_launch_s = tm["seconds"] / max(tm["launches"], 1)
    achieved = alg / max(tm["launches"], 1) / avg_launch_s / 1e9 if avg_launch_s > 0 else 0.0
    out = {
        "metric": "sampled shortest paths/sec",
        "value": paths / step_s,
        "unit": "paths/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u128", "data": "synthetic",
        "config": {"workload": f"{ngraphs} Chung-Lu graphs (seed 1000+i, n log-uniform in "
                               f"[1e3,1e5], half directed), all-nodes, epsilon={eps}, "
                               f"delta={args.delta}, seed {args.seed}, one multi-query engine "
                               "run"},
        "gteps": arcs / step_s / 1e9,
        "time_to_epsilon_s": step_s,
        "sequential_time_to_epsilon_s": seq_s,
        "speedup_vs_sequential": seq_s / step_s,
        "plain_sequential_time_to_epsilon_s": plain_s,
        "speedup_vs_plain": plain_s / step_s,
        "engine_call_by_call_time_to_epsilon_s": engine_stream_s,
        "chain_replays_per_step": (r1["replays"] - r0["replays"]) / args.steps,
        "results_identical_to_single_runs": identical,
        "sampler": {"note": "one further engine step with event timing",
                    "launches": tm["launches"], "samples": tm["samples"],
                    "avg_launch_ms": avg_launch_s * 1e3,
                    "gteps_in_kernel": tm["arcs"] / max(tm["seconds"], 1e-12) / 1e9,
                    "busy_fraction": tm["seconds"] / timed_elapsed},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "sampler_kernel (multi-segment)"},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_family(csrs, kw, batch)
        print(f"[bench] cpu baseline: {out['cpu_baseline']['value']:.0f} paths/s, parity "
              f"{out['cpu_baseline']['parity']}", file=sys.stderr, flush=True)
    for G in Gs:
        G.close()
    ctx.close()
    print(json.dumps(out), flush=True)


def time_modes(ctx, G, kw, ref, torch, kad, reps=3):
    """Warm time to epsilon of one call in each of kad_run's launch modes -- recorded
    batch chains, call by call, and the plain single-graph path -- after one untimed call,
    and whether each result equals the headline's."""
    import numpy as np
    ref = {k: (np.copy(v) if hasattr(v, "shape") else v) for k, v in ref.items()}
    out = {}
    for mode in ("graph", "stream", "plain"):
        ctx.set_exec(mode)
        r = kad.run(ctx, G, **kw)
        same = (r["tau"] == ref["tau"] and r["arcs_scanned"] == ref["arcs_scanned"]
                and all(np.array_equal(r[k], ref[k]) for k in ("count", "lower", "upper")))
        arrays = {k: r[k] for k in ("count", "bc", "lower", "upper")}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            kad.run(ctx, G, out=arrays, **kw)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / reps
        out[mode] = {"time_to_epsilon_s": t, "identical": bool(same)}
        print(f"[bench] exec {mode}: {t * 1e3:.2f} ms per call, identical={same}",
              file=sys.stderr, flush=True)
    ctx.set_exec("graph")
    out["graph_vs_plain_speedup"] = out["plain"]["time_to_epsilon_s"] / out["graph"]["time_to_epsilon_s"]
    out["graph_vs_stream_speedup"] = out["stream"]["time_to_epsilon_s"] / out["graph"]["time_to_epsilon_s"]
    return out


def _pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if len(xs) else None


def bench_serve(args, torch, gg, kad):
    """Serving: Poisson query stream through kad_server_* over resident graphs."""
    grid_id = gg.SERVE_GRAPHS - 1
    ids = [i for i in range(gg.SERVE_GRAPHS) if not (args.exclude_grid and i == grid_id)]
    t0 = time.perf_counter()
    csrs = {i: gg.serve_graph(i) for i in ids}
    print(f"[bench] {len(csrs)} graphs, {sum(g.n for g in csrs.values())} nodes, "
          f"{sum(g.arcs for g in csrs.values())} arcs ({time.perf_counter() - t0:.1f} s)",
          file=sys.stderr, flush=True)
    ctx = kad.Context(0)
    Gs = {i: kad.Graph(ctx, g) for i, g in csrs.items()}
    stream = [q for q in gg.serve_queries(args.queries, rate=args.rate, seed=7,
                                          graphs=gg.SERVE_GRAPHS) if q["graph"] in Gs]
    # warm-up: one light query per graph (vertex diameters, slot state, counter pools)
    t0 = time.perf_counter()
    with kad.Server(ctx) as srv:
        ts = [srv.submit(G, epsilon=0.1, delta=0.1, seed=99) for G in Gs.values()]
        for t in ts:
            srv.wait(t)
    print(f"[bench] warm-up {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)

    srv = kad.Server(ctx)
    pending = {}   # ticket -> (query, host submit time)
    done = []      # (query, result)
    canceled = []  # (query, age at cancel)

    def collect():
        for t in list(pending):
            try:
                r = srv.poll(t)
            except kad.KadError as e:
                q, ts_ = pending.pop(t)
                canceled.append((q, time.perf_counter() - ts_, e.status))
                continue
            if r is not None:
                done.append((pending.pop(t)[0], r))

    start = time.perf_counter()
    next_report = start + 10.0
    for q in stream:
        while True:
            now = time.perf_counter()
            if now >= start + q["t"]:
                break
            collect()
            time.sleep(min(0.002, start + q["t"] - now))
        kw = dict(epsilon=q["epsilon"], delta=q["delta"], seed=q["seed"])
        if q["mode"] == "topk":
            kw.update(mode="topk", k=q["k"])
        t = srv.submit(Gs[q["graph"]], **kw)
        pending[t] = (q, time.perf_counter())
        if time.perf_counter() > next_report:
            print(f"[bench] t={time.perf_counter() - start:.0f} s submitted {len(done) + len(pending) + len(canceled)}"
                  f" done {len(done)}", file=sys.stderr, flush=True)
            next_report += 10.0
    last_arrival = time.perf_counter()
    while pending and time.perf_counter() < last_arrival + args.drain:
        collect()
        time.sleep(0.005)
        if time.perf_counter() > next_report:
            print(f"[bench] draining: {len(pending)} running", file=sys.stderr, flush=True)
            next_report += 10.0
    cut = time.perf_counter()
    unfinished = [(q, cut - ts_) for t, (q, ts_) in pending.items()]
    srv.cancel()
    settle = time.perf_counter() + 120.0  # canceled queries finish once their launches drain
    while pending and time.perf_counter() < settle:
        for t in list(pending):
            try:
                if srv.poll(t) is not None:
                    pending.pop(t)
            except kad.KadError:
                pending.pop(t)
        if pending:
            time.sleep(0.05)
            if time.perf_counter() > next_report:
                print(f"[bench] canceling: {len(pending)} left", file=sys.stderr, flush=True)
                next_report += 10.0
    st = srv.stats()
    print("[bench] closing the server (waits for launches in flight)", file=sys.stderr, flush=True)
    srv.close()
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_serve(csrs, Gs, ctx, stream, grid_id, kad)
        print(f"[bench] cpu baseline: {cpu['value']:.0f} paths/s, parity {cpu['parity']}",
              file=sys.stderr, flush=True)
    elapsed = cut - start
    lat = [r["seconds"] for _, r in done]
    lower = lat + [age for _, age in unfinished]
    paths = sum(r["alpha"] + r["tau"] for _, r in done)

    def cls(pred):
        xs = [r["seconds"] for q, r in done if pred(q)]
        ys = [age for q, age in unfinished if pred(q)]
        return {"completed": len(xs), "unfinished": len(ys), "p50_s": _pct(xs + ys, 50),
                "p99_s": _pct(xs + ys, 99)}

    p99 = _pct(lower, 99)
    out = {
        "metric": "p99 query latency",
        "value": p99,
        "unit": "s",
        "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": elapsed * 1e3,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "u128", "data": "synthetic",
        "config": {"workload": f"serving: {len(Gs)} resident graphs, {len(stream)} queries at "
                               f"{args.rate}/s (Poisson, seed 7), all-nodes or top-k k in "
                               "{10,100}, epsilon U[0.002,0.02], delta 0.1"
                               + (", grid excluded" if args.exclude_grid else "")},
        "p50_s": _pct(lower, 50), "p99_s": p99, "mean_s": float(sum(lower) / max(len(lower), 1)),
        "p99_is_lower_bound": bool(unfinished) and p99 is not None and p99 >= min(a for _, a in unfinished),
        "completed": len(done), "unfinished_at_cutoff": len(unfinished),
        "cutoff_s": elapsed, "queries_per_s": len(done) / elapsed,
        "sampled_paths_per_s": paths / elapsed,
        "server": st,
        "by_class": {"all_nodes": cls(lambda q: q["mode"] == "all"),
                     "topk": cls(lambda q: q["mode"] == "topk"),
                     "grid": cls(lambda q: q["graph"] == grid_id),
                     "not_grid": cls(lambda q: q["graph"] != grid_id)},
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu

    def phases(rs):
        """Mean seconds per phase of a query: queued, pilot (admission to the pilot's counts),
        computeDelta, main phase, outputs (stopping to the result)."""
        if not rs:
            return None
        keys = ("setup", "pilot", "delta", "main")
        m = {k: sum(r[f"seconds_{k}"] for r in rs) / len(rs) for k in keys}
        m["outputs"] = sum(r["seconds"] - sum(r[f"seconds_{k}"] for k in keys) for r in rs) / len(rs)
        return m
    ng = sorted((r for q, r in done if q["graph"] != grid_id), key=lambda r: r["seconds"])
    out["not_grid_phases_s"] = {"all": phases(ng), "slowest_5pct": phases(ng[-max(1, len(ng) // 20):])}
    for q, age in sorted(unfinished, key=lambda x: -x[1])[:12]:
        print(f"[bench] unfinished: graph {q['graph']} (n={csrs[q['graph']].n}) {q['mode']} "
              f"k={q['k']} eps={q['epsilon']:.4f} age {age:.1f} s", file=sys.stderr, flush=True)
    slow = sorted(done, key=lambda x: -x[1]["seconds"])[:8]
    for q, r in slow:
        print(f"[bench] slowest: graph {q['graph']} (n={csrs[q['graph']].n}) {q['mode']} "
              f"k={q['k']} eps={q['epsilon']:.4f} {r['seconds']:.2f} s tau={r['tau']} "
              f"omega={r['omega']} queued {r['seconds_setup']:.2f} pilot {r['seconds_pilot']:.2f} "
              f"delta {r['seconds_delta']:.2f} main {r['seconds_main']:.2f} s", file=sys.stderr,
              flush=True)
    for G in Gs.values():
        G.close()
    ctx.close()
    print(json.dumps(out), flush=True)


def _gen_model(spec):
    import graphgen as gg
    model, n, beta, mean, seed = spec
    g = gg.random_model(model, n, beta, mean, seed)
    return spec, g


def bench_wide(args, torch, gg, kad):
    """The wide-count kernel on the 2000x2000 grid with 5% of edges deleted, where every
    sample needs path counts of hundreds to thousands of bits: hit counts of a fixed range
    of main-phase ids, timed end to end, then the same call with event timing for the
    kernel's own launch time and roofline."""
    g = gg.workload("grid2000")
    ctx = kad.Context(0)
    G = kad.Graph(ctx, g)
    N = args.wide_samples
    t0 = time.perf_counter()
    # warm-up: the timed call itself (slots, arenas, vertex diameter), so that every wide
    # dispatch of the run has one shape and a counter pass's mean per dispatch is the
    # timed launch's
    kad.hit_counts(ctx, G, args.seed, 1, 1000, N)
    print(f"[bench] warm-up {N} samples {time.perf_counter() - t0:.2f} s, layout "
          f"{ctx.wide_info()}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        counts, arcs = kad.hit_counts(ctx, G, args.seed, 1, 1000, N)
    torch.cuda.synchronize()
    step_s = (time.perf_counter() - t0) / args.steps
    ctx.set_timing(True)
    kad.hit_counts(ctx, G, args.seed, 1, 1000, N)
    tm = ctx.timing()
    ctx.set_timing(False)
    alg = algorithmic_bytes(tm["arcs"], tm["nodes"], tm["hits"])
    avg_launch_s = tm["seconds"] / max(tm["launches"], 1)
    achieved = alg / max(tm["launches"], 1) / avg_launch_s / 1e9 if avg_launch_s > 0 else 0.0
    run_info = None
    if args.grid_run_eps > 0:  # one whole adaptive run (all nodes) on the grid
        t0 = time.perf_counter()
        r = kad.run(ctx, G, epsilon=args.grid_run_eps, delta=args.delta, seed=args.seed)
        run_info = {"epsilon": args.grid_run_eps, "delta": args.delta,
                    "time_to_epsilon_s": time.perf_counter() - t0, "tau": r["tau"],
                    "omega": r["omega"], "vd": r["vd"],
                    "stop": "rule" if r["stop_reason"] else "omega"}
        print(f"[bench] grid2000 run at epsilon {args.grid_run_eps}: {run_info}", file=sys.stderr,
              flush=True)
    hbm = measured_traffic("grid2000", "wide_kernel")
    traffic = hbm / avg_launch_s / 1e9 if hbm and avg_launch_s > 0 else None
    out = {
        "metric": "sampled shortest paths/sec",
        "value": N / step_s,
        "unit": "paths/s",
        "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "multi-limb u64", "data": "synthetic",
        "config": {"workload": f"{WORKLOAD_TEXT['grid2000']}: n={g.n}, {g.arcs} arcs; hit counts "
                               f"of main-phase ids 1000..{1000 + N - 1}, seed {args.seed}"},
        "wide_layout": ctx.wide_info(),
        "run": run_info,
        "gteps": arcs / step_s / 1e9,
        "per_sample": {"arcs": tm["arcs"] / max(tm["samples"], 1),
                       "nodes": tm["nodes"] / max(tm["samples"], 1)},
        "sampler": {"note": "one further call with event timing", "launches": tm["launches"],
                    "samples": tm["samples"], "avg_launch_ms": avg_launch_s * 1e3},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": "wide_kernel",
                     "alg_bytes_per_launch": alg / max(tm["launches"], 1),
                     "l2_egress_bytes_per_launch": hbm,
                     "note": "algorithmic bytes by the sampler's per-arc and per-node figures; "
                             "the multi-limb counts add to them"},
    }
    G.close()
    ctx.close()
    print(json.dumps(out), flush=True)


def bench_exponent(args, torch, gg, kad):
    """Theorem 2 and Fig. 2: arcs visited per sampled path, balanced bidirectional search
    against the forward BFS from s, on the appendix's random-graph models as n grows."""
    import numpy as np
    from concurrent.futures import ProcessPoolExecutor
    models = args.models.split(",")
    betas = [float(b) for b in args.betas.split(",")]
    sizes = [int(float(x)) for x in args.sizes.split(",")]
    specs = [(m, n, b, args.mean_degree, 77 + i) for m in models for b in betas
             for i, n in enumerate(sizes)]
    t0 = time.perf_counter()
    workers = min(len(specs), max(1, min(16, host_threads())))
    graphs = {}
    with ProcessPoolExecutor(max_workers=workers) as ex:
        for spec, g in ex.map(_gen_model, specs):
            graphs[spec] = g
            print(f"[bench] generated {g.name}: n={g.n} arcs={g.arcs}", file=sys.stderr, flush=True)
    gen_s = time.perf_counter() - t0
    ctx = kad.Context(0)
    rows = []
    for spec in specs:
        g = graphs.pop(spec)
        G = kad.Graph(ctx, g)
        row = {"model": spec[0], "beta": spec[2], "n": g.n, "arcs": g.arcs}
        for search in ("balanced", "forward"):
            G.set_search(search)
            A = kad.sample_paths(ctx, G, 1, 1, 0, args.exp_samples)
            arcs = A["arcs"].astype(np.float64)
            conn = np.diff(A["path_off"].astype(np.int64)) > 0
            row[search] = {"arcs_per_sample": float(arcs.mean()),
                           "arcs_per_connected_sample": float(arcs[conn].mean()) if conn.any() else None,
                           "connected": float(conn.mean()),
                           # the paper's Fig. 2 exponent: log(m_avg) / log(m)
                           "alpha_fig2": float(np.log(arcs.mean()) / np.log(g.arcs))}
        print(f"[bench] {g.name}: balanced {row['balanced']['arcs_per_sample']:.0f}, forward "
              f"{row['forward']['arcs_per_sample']:.0f} arcs/sample", file=sys.stderr, flush=True)
        rows.append(row)
        G.close()
    ctx.close()
    fits = []
    for m in models:
        for b in betas:
            rs = [r for r in rows if r["model"] == m and r["beta"] == b]
            x = np.log([r["n"] for r in rs])
            fit = {"model": m, "beta": b,
                   "theorem2": 0.5 if b >= 3 else (4 - b) / 2}
            for search in ("balanced", "forward"):
                y = np.log([r[search]["arcs_per_sample"] for r in rs])
                fit[f"alpha_{search}"] = float(np.polyfit(x, y, 1)[0])
            fits.append(fit)
    out = {"metric": "exponent alpha of arcs visited per sampled path (arcs ~ n^alpha)",
           "value": float(np.mean([f["alpha_balanced"] for f in fits])),
           "unit": "exponent", "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": None,
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "u128", "data": "synthetic",
           "config": {"workload": f"random-graph models {models}, beta {betas}, mean degree "
                                  f"{args.mean_degree}, n in {sizes}, {args.exp_samples} "
                                  "samples each, balanced and forward search"},
           "generation_s": gen_s, "fits": fits, "rows": rows}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed runs (default 10; 3 for dcl4m)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cl1m")
    ap.add_argument("--epsilon", type=float, default=None,
                    help="default 0.005 (0.01 for er2000, 0.0002 for dcl4m)")
    ap.add_argument("--mode", default=None, choices=["all", "topk"],
                    help="default all (topk for dcl4m)")
    ap.add_argument("--k", type=int, default=50, help="top-k: k")
    ap.add_argument("--autotune", action="store_true",
                    help="autotune the sampler launch shape before timing (always for dcl4m)")
    ap.add_argument("--launch", default=None, metavar="BLOCK,SMALL",
                    help="sampler launch shape to use instead of the autotuner's")
    ap.add_argument("--delta", type=float, default=0.1)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--kernel-batch", type=int, default=65536)
    ap.add_argument("--check-interval", type=int, default=0)
    ap.add_argument("--exec", default="graph", choices=["graph", "stream", "plain"],
                    help="kad_run launch mode of the timed steps")
    ap.add_argument("--table", type=int, default=0,
                    help="sampler slot layout (kad_ctx_set_table): 0 library choice, 1 one "
                         "record per node, 6..24 hash tables of 2^k records")
    ap.add_argument("--no-modes", action="store_true",
                    help="skip timing the call in every launch mode")
    ap.add_argument("--cpu-samples", type=int, default=150000,
                    help="oracle sampling-rate baseline: main-phase ids (--no-cpu-full-run)")
    ap.add_argument("--cpu-full-run", dest="cpu_full_run", action="store_true", default=None,
                    help="baseline = the oracle's whole adaptive run (default for cl1m, er2000)")
    ap.add_argument("--no-cpu-full-run", dest="cpu_full_run", action="store_false")
    ap.add_argument("--cpu-one-thread", type=int, default=4000,
                    help="main-phase ids the one-thread oracle rate is measured on")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--queries", type=int, default=1000, help="serve: queries in the stream")
    ap.add_argument("--rate", type=float, default=20.0, help="serve: arrivals per second")
    ap.add_argument("--drain", type=float, default=30.0,
                    help="serve: seconds after the last arrival before running queries are canceled")
    ap.add_argument("--exclude-grid", action="store_true",
                    help="serve: leave the 2000x2000 grid (and its queries) out")
    ap.add_argument("--models", default="cl,cm,nr,grg", help="exponent: random-graph models")
    ap.add_argument("--betas", default="2.5,3.5", help="exponent: power-law exponents")
    ap.add_argument("--sizes", default="1e4,3e4,1e5,3e5,1e6", help="exponent: node counts")
    ap.add_argument("--mean-degree", type=float, default=10.0, help="exponent: mean degree")
    ap.add_argument("--exp-samples", type=int, default=1024, help="exponent: samples per graph")
    ap.add_argument("--wide-samples", type=int, default=1000,
                    help="grid2000: samples per call of the wide-count kernel")
    ap.add_argument("--grid-run-eps", type=float, default=0.02,
                    help="grid2000: epsilon of one whole run after the timed calls (0: none)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (scale for HBM counters)")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = {"dcl4m": 3, "grid2000": 2}.get(args.workload, 10)
    if args.epsilon is None:
        args.epsilon = {"er2000": 0.01, "dcl4m": 0.0002}.get(args.workload, 0.005)
    if args.mode is None:
        args.mode = "topk" if args.workload == "dcl4m" else "all"
    if args.workload == "dcl4m" and not args.launch:
        args.autotune = True
    if args.cpu_full_run is None:
        args.cpu_full_run = args.workload in ("cl1m", "er2000")
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(samples would shard across GPUs with one all-reduce of the counters per "
              "check interval; not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    import graphgen as gg
    import paper_1604_08553_amd as kad

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calibrate_copy:
        nbytes = args.calibrate_copy << 20
        x = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "device copy", "bytes_read": nbytes,
                          "bytes_written": nbytes}), flush=True)
        return
    if args.workload == "batch256":
        return bench_batch(args, torch, gg, kad)
    if args.workload == "serve":
        return bench_serve(args, torch, gg, kad)
    if args.workload == "exponent":
        return bench_exponent(args, torch, gg, kad)
    if args.workload == "grid2000":
        return bench_wide(args, torch, gg, kad)
    t0 = time.perf_counter()
    csr = gg.workload(args.workload)
    gen_s = time.perf_counter() - t0
    print(f"[bench] graph {csr.name}: n={csr.n} arcs={csr.arcs} ({gen_s:.1f} s)", file=sys.stderr,
          flush=True)
    t0 = time.perf_counter()
    ctx = kad.Context(0)
    ctx_create_s = time.perf_counter() - t0
    if args.table:
        ctx.set_table(args.table)
    G = kad.Graph(ctx, csr)
    tuned = None
    if args.launch:
        block, small = (int(x) for x in args.launch.split(","))
        G.set_launch(block, small)
        tuned = {"block": block, "small_expansion": small, "seconds": None}
    elif args.autotune:
        tuned = G.autotune(args.kernel_batch)
        print(f"[bench] autotune: {tuned}", file=sys.stderr, flush=True)
    kw = dict(epsilon=args.epsilon, delta=args.delta, seed=args.seed,
              kernel_batch=args.kernel_batch, check_interval=args.check_interval)
    if args.mode == "topk":
        kw.update(mode="topk", k=args.k)
    arrays = None  # result arrays, allocated by the warmup and reused by every step
    first_call_s = None
    for w in range(args.warmup):
        r = kad.run(ctx, G, out=arrays, **kw)
        arrays = {k: r[k] for k in ("count", "bc", "lower", "upper")}
        if first_call_s is None:
            first_call_s = r["seconds"]
        print(f"[bench] warmup {w}: tau={r['tau']} {r['seconds']:.3f} s", file=sys.stderr, flush=True)

    ctx.set_exec(args.exec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = []
    for s in range(args.steps):
        r = kad.run(ctx, G, out=arrays, **kw)
        arrays = {k: r[k] for k in ("count", "bc", "lower", "upper")}
        if first_call_s is None:
            first_call_s = r["seconds"]
        runs.append(r)
        print(f"[bench] step {s}: tau={r['tau']} omega={r['omega']} stop={r['stop_reason']} "
              f"{r['seconds']:.3f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    exec_info = ctx.exec_info()
    # the sampler's own launch time: the same call again with every sampler launch timed
    # by HIP events on its stream (timing launches call by call)
    ctx.set_timing(True)
    timed_steps = max(1, min(args.steps, 5))
    for s in range(timed_steps):
        rt = kad.run(ctx, G, out=arrays, **kw)
        assert rt["tau"] == runs[0]["tau"]
    tm = ctx.timing()
    ctx.set_timing(False)
    print(f"[bench] event-timed pass: {tm['launches']} launches, {tm['seconds']:.4f} s",
          file=sys.stderr, flush=True)

    paths = sum(r["alpha"] + r["tau"] for r in runs)
    arcs = sum(r["arcs_scanned"] + r["pilot_arcs_scanned"] for r in runs)
    r0 = runs[0]
    alg = algorithmic_bytes(tm["arcs"], tm["nodes"], tm["hits"])
    per_launch_bytes = alg / max(tm["launches"], 1)
    avg_launch_s = tm["seconds"] / max(tm["launches"], 1)
    achieved = per_launch_bytes / avg_launch_s / 1e9 if avg_launch_s > 0 else 0.0
    hbm = measured_traffic(args.workload)
    traffic = hbm / avg_launch_s / 1e9 if hbm and avg_launch_s > 0 else None

    out = {
        "metric": "sampled shortest paths/sec",
        "value": paths / elapsed,
        "unit": "paths/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u128",
        "data": "synthetic",
        "config": {
            "workload": f"{WORKLOAD_TEXT.get(args.workload, args.workload)}: n={csr.n}, "
                        f"{csr.arcs} arcs; "
                        + (f"top-k k={args.k}" if args.mode == "topk" else "all-nodes")
                        + f", epsilon={args.epsilon}, delta={args.delta}, seed {args.seed}, "
                        f"{args.kernel_batch} samples per sampler launch",
            "launch_shape": tuned,
            "graph_sha256": csr.sha256(),
        },
        "gteps": arcs / elapsed / 1e9,
        "time_to_epsilon_s": elapsed / args.steps,
        "tau": r0["tau"], "omega": r0["omega"], "alpha": r0["alpha"], "vd": r0["vd"],
        "check_interval": r0["interval"], "stop": "rule" if r0["stop_reason"] else "omega",
        "phases_s": dict({k: sum(r[f"seconds_{k}"] for r in runs) / len(runs)
                          for k in ("setup", "pilot", "delta", "main")},
                         outputs=sum(r["seconds"] - sum(r[f"seconds_{k}"] for k in
                                                        ("setup", "pilot", "delta", "main"))
                                     for r in runs) / len(runs),
                         note="outputs: the final counts copied to the host (n x 8 bytes) "
                              "and the per-node intervals computed there in binary64"),
        "exec": {"mode": args.exec, "chains_recorded": exec_info["records"],
                 "chain_replays": exec_info["replays"]},
        "slot_layout": ctx.table_info(),
        "sampler": {"note": f"from {timed_steps} further calls with event timing",
                    "launches": tm["launches"], "samples": tm["samples"],
                    "avg_launch_ms": avg_launch_s * 1e3,
                    "arcs_per_sample": tm["arcs"] / max(tm["samples"], 1),
                    "nodes_per_sample": tm["nodes"] / max(tm["samples"], 1),
                    "gteps_in_kernel": tm["arcs"] / max(tm["seconds"], 1e-12) / 1e9},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "sampler_kernel",
                     "alg_bytes_per_launch": per_launch_bytes,
                     "l2_egress_bytes_per_launch": hbm},
    }
    if not args.no_modes:
        out["exec_modes"] = time_modes(ctx, G, kw, runs[0], torch, kad)
    # cold time to epsilon: a graph registered anew (upload, validation, transpose) and its
    # first run (vertex diameter, buffers) on the warm context
    G.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    G2 = kad.Graph(ctx, csr)
    t_graph = time.perf_counter() - t0
    if tuned:
        G2.set_launch(tuned["block"], tuned["small_expansion"])
    rc = kad.run(ctx, G2, out=arrays, **kw)
    t_cold = time.perf_counter() - t0
    out["time_to_epsilon_cold_s"] = t_cold
    out["cold"] = {"graph_create_s": t_graph, "first_run_s": rc["seconds"],
                   "first_run_setup_s": rc["seconds_setup"],
                   "context_create_s": ctx_create_s, "first_call_on_new_context_s": first_call_s,
                   "note": "time_to_epsilon_cold_s = graph_create_s + first_run_s (vertex "
                           "diameter computed); first_call_on_new_context_s also allocates "
                           "and clears the sampler slots"}
    assert rc["tau"] == r0["tau"] and rc["stop_reason"] == r0["stop_reason"]
    G2.close()
    ctx.close()
    if not args.no_cpu_baseline:
        if args.cpu_full_run:
            out["cpu_baseline"] = cpu_baseline_run(csr, kw, rc, args.cpu_one_thread)
        else:
            out["cpu_baseline"] = cpu_baseline(csr, args.cpu_samples, args.seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
