#!/usr/bin/env python3
"""Benchmark of the Louvain local-moving hot path on one MI355X.

Workload: R-MAT scale 24, edge factor 16 (a=0.57, b=0.19, c=0.19), symmetrised,
self-loops and duplicates removed, unit weights (16.8M vertices, ~521M CSR
entries).  One step = multi-level Louvain (local moving, renumbering and
aggregation at every level; final labels and per-level statistics copied to
the host) followed by LPA (max 20 sweeps; labels copied to the host) on the
same device-resident graph.  The graph is created (copied to HBM) before
timing.

The timed steps run the production path (each level's sweeps captured as
hipGraphs, degree classes on concurrent streams).

Printed JSON line (one):
  value       local-move GTEPS of Louvain in the timed steps: sum over levels
              and sweeps of the level's CSR entries / summed local-moving time
              (HIP events around each level's sweep loop)
  roofline    the dominant move kernel, from one instrumented step after the
              timed region (kernels one at a time, HIP events around each on
              the library's stream): compulsory bytes per launch (8 per CSR
              entry + 36 per vertex of its class) / average launch duration;
              traffic from the stored rocprofv3 counters.  Beside it the
              local-moving phase as a whole: level0_frac and all_levels_frac
              = compulsory bytes of the sweeps (8E + 36n per sweep of a level
              with n vertices and E entries) / the timed steps' sweep time /
              8 TB/s, with the per-level figures in `levels`
  cpu_baseline  the CPU oracle, unmodified, timed on this host: one warm-up
              and five timed repetitions (median and mean) of level-0 sweeps
              over the full graph, and per-phase (local moving, renumbering,
              aggregation) Louvain runs of the small SBM configuration and a
              sample of the batch graphs on all host threads and on one
  parity      every level of the timed runs equals the oracle's per-level
              digests (tests/golden/rmat24_seed2_digests.json): sizes, Q_int,
              per-sweep move counts, SHA-256 of the final labels; the GPU's
              first-sweep partition equals the oracle's, bit for bit
  workloads   the small SBM (4,096 vertices) and the 10 M-vertex LFR graph:
              time per step and local-move rate
  batch       4,096 mixed graphs in one packed handle vs one graph per call
  serving     a Poisson trace of Louvain jobs: continuous batching vs FIFO one
              graph per call, throughput and p50/p99 latency
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "local-move GTEPS + %HBM roofline at exact partitions; batched p50/p99 latency"
HBM_PEAK_GBS = 8000.0
GOLDEN = os.path.join(ROOT, "tests", "golden", "rmat24_seed2_digests.json")
GOLDEN_LFR = os.path.join(ROOT, "tests", "golden", "lfr10m_seed3_digests.json")
# the paper's own local-moving times (context, not the target): Section V-B,
# strong scaling on com-livejournal (3,997,962 vertices, 34,681,189 edges)
PAPER_CONTEXT = {
    "local_move_s": {"2_threads": 16.8, "128_threads": 2.4},
    "louvain_total_s": {"2_threads": 25.6, "128_threads": 5.6},
    "hardware": "2 x AMD EPYC 7763 (128 cores), 512 GB, Chapel/Arachne",
    "workload": "com-livejournal, 3,997,962 vertices, 34,681,189 edges, all levels",
    "source": "Section V-B (strong scaling) and Section IV-B (setup)",
    "note": "different graph and hardware; quoted as context only",
}


def sha256_i32(*arrays) -> str:
    import hashlib

    import numpy as np

    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a, dtype="<i4").tobytes())
    return h.hexdigest()


def level_roofline(runs, peak_gbs=HBM_PEAK_GBS):
    """Compulsory-bytes roofline of local moving per level of the timed steps:
    a sweep over a level with n vertices and E entries touches 8E + 36n bytes
    (indices and weights; offsets, label, degree and volume read, label and
    volume written per vertex), sweep time from the HIP events around each
    level's sweeps, averaged over the steps."""
    K = len(runs)
    levels = []
    for lvl, lv in enumerate(runs[0][0].levels):
        i = lv.info
        ms = sum(r.levels[lvl].info["sweep_ms"] for r, _ in runs) / K
        b = 8 * i["nnz"] + 36 * i["n"]
        sw = i["sweeps"]
        levels.append({"level": lvl, "n": i["n"], "nnz": i["nnz"], "sweeps": sw,
                       "cached_sweeps": i["cached_sweeps"], "refreshed_entries": i["refreshed_entries"],
                       "sweep_ms": round(ms, 3), "ms_per_sweep": round(ms / max(sw, 1), 4),
                       "bytes_per_sweep": b,
                       "frac": round(b * sw / (ms * 1e-3) / (peak_gbs * 1e9), 4) if ms > 0 else None})
    tot_b = sum(x["bytes_per_sweep"] * x["sweeps"] for x in levels)
    tot_ms = sum(x["sweep_ms"] for x in levels)
    return levels, (tot_b / (tot_ms * 1e-3) / (peak_gbs * 1e9) if tot_ms > 0 else None)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


PMC_FILE = os.path.join(ROOT, "profiles", "pmc_rmat24.txt")


KERNEL_SOURCES = ("lv_device.h", "lv_internal.h", "lv_move.hip")  # where the move kernels are defined


def kernel_source_digest() -> str:
    """Digest of the move kernels' code, to tell whether stored counters still
    describe them: comments and runs of white space are left out, so that a
    change of wording alone keeps the record (the sources hold no comment
    marker inside a string literal)."""
    import hashlib
    import re

    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2507_06471_amd", "csrc")
    for f in KERNEL_SOURCES:
        with open(os.path.join(d, f)) as fh:
            text = fh.read()
        code = re.sub(r"//[^\n]*", "", re.sub(r"/\*.*?\*/", "", text, flags=re.S))
        h.update(f.encode() + b"\0" + " ".join(code.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic(slot: str):
    """HBM bytes per launch of the kernel in `slot` from the stored rocprofv3
    FETCH_SIZE / WRITE_SIZE passes over this workload, each scaled by the
    counter's reading for a plain copy of known size; None if there is no
    record or the kernel sources changed since it was taken."""
    if not os.path.exists(PMC_FILE):
        return None
    with open(PMC_FILE) as fh:
        recs = [dict(kv.split("=", 1) for kv in line.split()) for line in fh if line.strip() and not line.startswith("#")]
    for r in recs:
        if r.get("slot") == slot:
            if r.get("src") != kernel_source_digest():
                return None
            fetch = float(r["fetch_kib"]) / float(r["copy_fetch_factor"])
            write = float(r["write_kib"]) / float(r["copy_write_factor"])
            return round((fetch + write) * 1024.0)
    return None


def prune_leg(args, lvp, dg, runs, phases, K, torch):
    """The same job with active-vertex pruning (LV_PRUNE): only vertices whose
    neighbourhood changed in the last two sweeps are evaluated.  Louvain's
    partition differs from the full sweeps' (its Q is reported beside the
    full one); LPA's must be identical.  Entries per second count every entry
    of every executed sweep, as for the full sweeps, so they are an
    equivalent rate, not bytes read."""
    reps = []
    for _ in range(args.prune_reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = lvp.louvain(dg, level_labels=False, prune=True)
        lp = lvp.lpa(dg, prune=True)
        torch.cuda.synchronize()
        reps.append((time.perf_counter() - t0, r, lp))
    lm = sum(lv.info["sweep_ms"] for _, r, _ in reps for lv in r.levels) / len(reps)
    edges = sum(lv.info["nnz"] * lv.info["sweeps"] for lv in reps[0][1].levels)
    lpa_ms = sum(lp.info["sweep_ms"] for _, _, lp in reps) / len(reps)
    r, lp = reps[0][1], reps[0][2]
    full_r, full_lp = runs[0]
    lpa_same = full_lp.moves == lp.moves and bool((full_lp.labels == lp.labels).all())
    if not lpa_same:
        print("pruned LPA differs from full LPA", file=sys.stderr, flush=True)
        sys.exit(1)
    out = {"local_move_ms": round(lm, 3),
           "local_move_speedup": round(phases["local_move_ms"] / K / lm, 3) if lm > 0 else None,
           "equiv_gteps": round(edges / (lm * 1e-3) / 1e9, 3) if lm > 0 else None,
           "ms_per_step": round(sum(t for t, _, _ in reps) / len(reps) * 1e3, 3),
           "levels": len(r.accepted), "sweeps_per_level": [lv.info["sweeps"] for lv in r.levels],
           "q": r.q, "q_full_sweeps": full_r.q,
           "lpa_ms": round(lpa_ms, 3), "lpa_speedup": round(phases["lpa_ms"] / K / lpa_ms, 3) if lpa_ms > 0 else None,
           "lpa_equal_to_full": lpa_same}
    log(f"pruned: {out}")
    return out


def async_leg(args, lvp, dg, runs, phases, K, torch):
    """The same job with asynchronous sweeps (LV_ASYNC, Alg. 1 and 2 as
    written: labels and volumes updated in place during a sweep).  Results
    depend on scheduling; Q is reported beside the synchronous sweeps' Q and
    the reported Q_int is checked against the modularity of the labels."""
    reps = []
    for _ in range(args.async_reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = lvp.louvain(dg, level_labels=False, asynchronous=True)
        lp = lvp.lpa(dg, asynchronous=True)
        torch.cuda.synchronize()
        reps.append((time.perf_counter() - t0, r, lp))
    for _, r, _ in reps:
        qi, m, _ = lvp.modularity(dg, r.final_labels)
        if (qi, m) != (r.q_int, r.M):
            print("asynchronous run: reported modularity differs from its labels'", file=sys.stderr, flush=True)
            sys.exit(1)
    lm = sum(lv.info["sweep_ms"] for _, r, _ in reps for lv in r.levels) / len(reps)
    edges = sum(lv.info["nnz"] * lv.info["sweeps"] for lv in reps[0][1].levels)
    lpa_ms = sum(lp.info["sweep_ms"] for _, _, lp in reps) / len(reps)
    r0, lp0 = reps[0][1], reps[0][2]
    out = {"local_move_ms": round(lm, 3), "gteps": round(edges / (lm * 1e-3) / 1e9, 3) if lm > 0 else None,
           "ms_per_step": round(sum(t for t, _, _ in reps) / len(reps) * 1e3, 3),
           "levels": len(r0.accepted), "sweeps_per_level": [lv.info["sweeps"] for lv in r0.levels],
           "q": [r.q for _, r, _ in reps], "q_full_sweeps": runs[0][0].q,
           "lpa_ms": round(lpa_ms, 3), "lpa_sweeps": lp0.info["sweeps"],
           "lpa_q": lp0.info["q_end"] / float(dg.volume) ** 2}
    log(f"asynchronous: {out}")
    return out


def edges_leg(args, lvp, graphgen, g, np, torch):
    """The step before the path: the benchmark graph built on the device from
    its raw R-MAT samples (loops dropped, repeated pairs merged to weight 1),
    timed from device-resident edge arrays to a ready handle (sort, merge,
    CSR, degrees, degree-ordered storage).  The built CSR must equal the
    generator's."""
    t = time.time()
    u, v = graphgen.rmat_edges(args.scale, args.edge_factor, seed=args.seed)
    du, dv = torch.from_numpy(u).cuda(), torch.from_numpy(v).cuda()
    del u, v
    torch.cuda.synchronize()
    log(f"edges: {du.numel()} raw samples resident in {time.time() - t:.1f}s")
    times = []
    for rep in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        eg = lvp.Graph.from_edges(g.n, du, dv, drop_loops=True, simple=True)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        if rep == 0:
            off, idx, _ = eg.csr()
            equal = bool(np.array_equal(off, g.offsets) and np.array_equal(idx, g.indices))
            del off, idx
        eg.close()
    m = int(du.numel())
    del du, dv
    best = min(times)
    out = {"edges": m, "ms": round(best * 1e3, 2), "medges_per_s": round(m / best / 1e6, 1),
           "csr_equal_to_generator": equal, "timed": "device edge arrays -> ready handle, best of 2"}
    log(f"edges: {out}")
    if not equal:
        print("edge-list construction differs from the generator's CSR", file=sys.stderr, flush=True)
        sys.exit(1)
    return out


def batch_leg(args, lvp, graphgen, np, torch):
    """Mixed batch of independent graphs: one packed handle (every graph in the
    same launches, sweeps captured as hipGraphs, autotuned classes) against
    one graph per call on the same GPU, over a sample of the same graphs.
    Both sides start from device-resident graphs and end with every graph's
    final labels and modularity on the host; partitions must be identical."""
    t = time.time()
    gs = graphgen.batch_mix(args.batch_graphs, seed=4)
    V = sum(g.n for g in gs)
    E = sum(g.nnz for g in gs)
    log(f"batch: {len(gs)} graphs, {V} vertices, {E} entries, generated in {time.time() - t:.1f}s")
    t = time.time()
    bg = lvp.Graph.batch(gs, validate=True)
    log(f"batch: packed handle resident in {time.time() - t:.1f}s")
    cfg, est = lvp.autotune(bg)
    log(f"batch: autotuned {cfg} (estimated level-0 {est:.1f} ms)")

    def timed(**kw):
        fp_ = lvp.louvain_final(bg, **kw)  # warm-up
        ts = []
        for _ in range(args.batch_reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fp_ = lvp.louvain_final(bg, **kw)
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts)), fp_

    # the two ways of launching the later sweeps' classes, at default settings
    per_class_s, fp_pc = timed(tuning={"fused": 0})
    fused_s, fp_f = timed(tuning={"fused": 1})
    launch_cmp = {"per_class_launches_ms": round(per_class_s * 1e3, 2), "fused_persistent_ms": round(fused_s * 1e3, 2),
                  "same_partitions": bool(np.array_equal(fp_pc.labels, fp_f.labels))}
    log(f"batch: {launch_cmp}")
    batch_s, fp = timed(autotuned=True)
    # entries processed by local moving, from a timed run's per-level counts
    # (per graph: sum over levels of entries x sweeps)
    detail = lvp.louvain(bg, autotuned=True)
    lm_entries = sum(lv.info["nnz"] * lv.info["sweeps"] for r in detail for lv in r.levels)
    bases = np.concatenate([[0], np.cumsum([g.n for g in gs])])
    # one graph per call over an evenly spaced sample
    step_ = max(1, len(gs) // args.batch_sample)
    sample = list(range(0, len(gs), step_))[:args.batch_sample]
    handles = [lvp.Graph.from_csr(gs[i], validate=True) for i in sample]
    for h in handles[:4]:
        lvp.louvain_final(h)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    singles = [lvp.louvain_final(h) for h in handles]
    single_s = time.perf_counter() - t0
    same = True
    for i, h, fs in zip(sample, handles, singles):
        lo, hi = bases[i], bases[i + 1]
        same &= bool(np.array_equal(fs.labels, fp.labels[lo:hi])) and int(fs.q_int[0]) == int(fp.q_int[i])
        h.close()
    sample_entries = sum(lv.info["nnz"] * lv.info["sweeps"] for i in sample for lv in detail[i].levels)
    bg.close()
    out = {
        "workload": f"{len(gs)} graphs alternating SBM (blocks of 128, 75% of the degree inside) and R-MAT "
                    "(0.57, 0.19, 0.19); n log-uniform in [1024, 65536], mean degree uniform in [8, 32], "
                    "unit weights, seed 4",
        "graphs": len(gs), "vertices": V, "entries": E,
        "batched": {"ms": round(batch_s * 1e3, 2), "graphs_per_s": round(len(gs) / batch_s, 1),
                    "local_move_gteps": round(lm_entries / batch_s / 1e9, 3), "reps": args.batch_reps,
                    "tuning": cfg, "autotune_estimate_ms": round(est, 2), "launch_modes": launch_cmp},
        "one_graph_per_call": {"sample_graphs": len(sample), "ms": round(single_s * 1e3, 2),
                               "graphs_per_s": round(len(sample) / single_s, 1),
                               "local_move_gteps": round(sample_entries / single_s / 1e9, 3)},
        "identical_partitions": same,
    }
    out["speedup_graphs_per_s"] = round(out["batched"]["graphs_per_s"] / out["one_graph_per_call"]["graphs_per_s"], 2)
    log(f"batch: {out}")
    if not same or not launch_cmp["same_partitions"]:
        print("batched partitions differ from one-graph-per-call partitions", file=sys.stderr, flush=True)
        sys.exit(1)
    return out


def serving_leg(args, lvp, graphgen, np, torch):
    """Poisson traces of Louvain jobs replayed in real time, at each load of
    --serve-loads (arrival rate / one-graph-per-call capacity): through a FIFO
    loop that runs one graph per call (create from host memory, Louvain,
    final labels) and through the continuous-batching server.  Latency is
    arrival -> result; every job's partition must equal its graph's result
    alone.  Then both at saturation (jobs submitted at once)."""
    import threading

    t = time.time()
    pool = graphgen.serving_pool(args.serve_pool, seed=5)
    log(f"serving: pool of {len(pool)} graphs (n {min(g.n for g in pool)}..{max(g.n for g in pool)}, "
        f"{sum(g.nnz for g in pool)} entries) generated in {time.time() - t:.1f}s")
    # per-graph service time of one-graph-per-call, and each graph's partition alone
    alone, svc = [], []
    for g in pool:
        with lvp.Graph.from_csr(g) as h:
            lvp.louvain_final(h)
    for g in pool:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with lvp.Graph.from_csr(g) as h:
            fp = lvp.louvain_final(h)
        svc.append(time.perf_counter() - t0)
        alone.append((fp.labels.copy(), int(fp.q_int[0])))
    rng = np.random.default_rng(5)
    J = args.serve_jobs
    which = rng.integers(0, len(pool), size=J)
    mean_svc = float(np.mean([svc[i] for i in which]))
    gaps = rng.exponential(1.0, size=J)  # one trace shape, scaled to each load
    entries = [pool[i].nnz for i in which]

    def summarize(lat, span, same):
        lat = np.asarray(lat) * 1e3
        return {"jobs_per_s": round(J / span, 2), "p50_ms": round(float(np.percentile(lat, 50)), 2),
                "p99_ms": round(float(np.percentile(lat, 99)), 2), "mean_ms": round(float(lat.mean()), 2),
                "span_s": round(span, 2), "identical_partitions": same}

    srv = lvp.Server(max_jobs=args.serve_max_jobs)
    loads = {}
    for load in args.serve_loads:
        rate = load / mean_svc
        arrivals = np.cumsum(gaps / rate)
        log(f"serving: {J} jobs, mean one-per-call service {mean_svc * 1e3:.2f} ms, Poisson rate {rate:.1f}/s "
            f"({load:.0%} of one-per-call capacity)")
        # FIFO, one graph per call
        same = True
        lat = np.zeros(J)
        t0 = time.perf_counter()
        for i in range(J):
            now = time.perf_counter()
            if now < t0 + arrivals[i]:
                time.sleep(t0 + arrivals[i] - now)
            with lvp.Graph.from_csr(pool[which[i]]) as h:
                fp = lvp.louvain_final(h)
            done = time.perf_counter()
            lat[i] = done - (t0 + arrivals[i])
            same &= bool(np.array_equal(fp.labels, alone[which[i]][0])) and int(fp.q_int[0]) == alone[which[i]][1]
            if i % 250 == 0:
                log(f"serving {load:.0%}: fifo job {i}")
        fifo = summarize(lat, time.perf_counter() - t0, same)
        log(f"serving {load:.0%}: one graph per call {fifo}")
        # continuous batching server
        tickets = [0] * J
        submitted = [0.0] * J
        ready = [threading.Event() for _ in range(J)]
        t0 = time.perf_counter()

        def submitter():
            for i in range(J):
                now = time.perf_counter()
                if now < t0 + arrivals[i]:
                    time.sleep(t0 + arrivals[i] - now)
                submitted[i] = time.perf_counter()
                tickets[i] = srv.submit(pool[which[i]])
                ready[i].set()

        th = threading.Thread(target=submitter)
        th.start()
        same = True
        lat = np.zeros(J)
        end = 0.0
        for i in range(J):
            ready[i].wait()
            srv.wait(tickets[i])
            labels, info = srv.result(tickets[i], pool[which[i]].n)
            fin = submitted[i] + info["total_ms"] * 1e-3
            end = max(end, fin)
            lat[i] = fin - (t0 + arrivals[i])
            same &= bool(np.array_equal(labels, alone[which[i]][0])) and int(info["q_int"]) == alone[which[i]][1]
            if i % 250 == 0:
                log(f"serving {load:.0%}: server job {i}")
        th.join()
        batched = summarize(lat, end - t0, same)
        log(f"serving {load:.0%}: continuous batching {batched}")
        loads[f"{load:g}"] = {"rate_per_s": round(rate, 2), "one_graph_per_call": fifo, "continuous_batching": batched,
                              "p50_speedup": round(fifo["p50_ms"] / batched["p50_ms"], 2) if batched["p50_ms"] > 0 else None,
                              "p99_speedup": round(fifo["p99_ms"] / batched["p99_ms"], 2) if batched["p99_ms"] > 0 else None,
                              "throughput_speedup": round(batched["jobs_per_s"] / fifo["jobs_per_s"], 2)}
        if not (fifo["identical_partitions"] and batched["identical_partitions"]):
            print("a served partition differs from the graph's partition alone", file=sys.stderr, flush=True)
            sys.exit(1)
    stats = srv.stats()

    # capacity: the first jobs of the trace all submitted at once
    C = min(J, args.serve_capacity_jobs)
    same = True
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(C):
        with lvp.Graph.from_csr(pool[which[i]]) as h:
            fp = lvp.louvain_final(h)
        same &= bool(np.array_equal(fp.labels, alone[which[i]][0]))
    fifo_cap = C / (time.perf_counter() - t0)
    t0 = time.perf_counter()
    tk = [srv.submit(pool[which[i]]) for i in range(C)]
    for i in range(C):
        srv.wait(tk[i])
        labels, info = srv.result(tk[i], pool[which[i]].n)
        same &= bool(np.array_equal(labels, alone[which[i]][0]))
    srv_cap = C / (time.perf_counter() - t0)
    srv.close()
    log(f"serving: saturated ({C} jobs at once): one per call {fifo_cap:.2f}/s, server {srv_cap:.2f}/s")
    if not same:
        print("a served partition differs from the graph's partition alone", file=sys.stderr, flush=True)
        sys.exit(1)
    first = loads[f"{args.serve_loads[0]:g}"]
    out = {"workload": f"{J} Louvain jobs per trace, Poisson arrivals at {', '.join(f'{x:.0%}' for x in args.serve_loads)} "
                       f"of one-graph-per-call capacity; graphs from a pool of {len(pool)} R-MAT graphs, n log-uniform "
                       "in [1e4, 4e6], edge factor uniform in {8..16}, unit weights, seed 5",
           "mean_entries": round(float(np.mean(entries))), "mean_one_per_call_service_ms": round(mean_svc * 1e3, 2),
           "loads": loads,
           "one_graph_per_call": first["one_graph_per_call"], "continuous_batching": first["continuous_batching"],
           "p99_speedup": first["p99_speedup"], "throughput_speedup": first["throughput_speedup"],
           "saturated": {"jobs": C, "one_graph_per_call_jobs_per_s": round(fifo_cap, 2),
                         "server_jobs_per_s": round(srv_cap, 2), "speedup": round(srv_cap / fifo_cap, 2),
                         "identical_partitions": same},
           "server_stats": {"max_batch": int(stats["max_batch"]), "packed_levels": int(stats["steps"])}}
    return out


def digest_check(r, lp, g, path, name):
    """Every level of a timed run (Louvain result r, LPA result lp, graph g)
    against the oracle's per-level digests in `path` (written by the scripts
    in tests/golden/ from the oracle alone).  Exits on a mismatch."""
    import json

    with open(path) as fh:
        gold = json.load(fh)
    want = gold["louvain"]
    bad = []
    if (g.n, g.nnz) != (gold["n"], gold["nnz"]):
        bad.append("graph size")
    if len(r.levels) != len(want["levels"]):
        bad.append("number of levels")
    for lvl, (a, b) in enumerate(zip(r.levels, want["levels"])):
        i = a.info
        if (i["n"], i["nnz"], i["n_next"], i["q_start"], i["q_end"], bool(i["accepted"])) != \
                (b["n"], b["nnz"], b["n_next"], b["q_start"], b["q_end"], b["accepted"]):
            bad.append(f"level {lvl} sizes or Q_int")
        if a.moves != b["moves"]:
            bad.append(f"level {lvl} moves")
    if (r.M, r.q_int) != (want["M"], want["q_int"]) or sha256_i32(r.final_labels) != want["final_labels_sha256"]:
        bad.append("final labels or Q_int")
    if lp.moves != gold["lpa"]["moves"] or sha256_i32(lp.labels) != gold["lpa"]["labels_sha256"] or \
            lp.info["q_end"] != gold["lpa"]["q_int"]:
        bad.append("LPA")
    out = {"equal": not bad, "levels": len(want["levels"]), "file": os.path.relpath(path, ROOT),
           "checked": "per level n, nnz, n_next, Q_start, Q_end, acceptance, per-sweep moves; final labels "
                      "(SHA-256), Q_int, M; LPA moves, labels (SHA-256) and Q_int"}
    log(f"golden digests ({name}): {out}")
    if bad:
        print(f"{name}: timed run differs from the oracle's digests: {bad}", file=sys.stderr, flush=True)
        sys.exit(1)
    return out


def golden_check(args, r, lp, g):
    """The benchmark graph's timed run against its digests
    (tests/golden/make_rmat24_digests.py); None for other graphs."""
    if (args.scale, args.edge_factor, args.seed) != (24, 16.0, 2) or not os.path.exists(GOLDEN):
        return None
    return digest_check(r, lp, g, GOLDEN, "R-MAT 24")


def cpu_baseline(args, oracle, adj, g, graphgen, np):
    """The CPU oracle as it stands, on this host's cores: one warm-up and
    `cpu_reps` timed repetitions of `cpu_sweeps` level-0 sweeps over the full
    benchmark graph (median and mean), and whole Louvain runs with the paper's
    phases timed apart on the small SBM configuration and a sample of the
    batch graphs, on all threads and on one (one warm-up, five repetitions)."""
    def reps(fn, n):
        fn()
        ts = []
        for _ in range(n):
            t = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t)
        return float(np.median(ts)), float(np.mean(ts))

    threads = oracle.num_threads()
    sweeps = max(1, args.cpu_sweeps)
    med, mean = reps(lambda: oracle.local_move(adj, oracle.LOUVAIN, max_sweeps=sweeps), args.cpu_reps)
    out = {"value": round(sweeps * g.nnz / med / 1e9, 4), "unit": "GTEPS", "cores": threads, "kind": "oracle",
           "host_nproc": os.cpu_count(),
           "sample": f"{sweeps} level-0 synchronous Louvain sweeps of the CPU oracle over the full graph "
                     f"({sweeps * g.nnz} entries per repetition), 1 warm-up + {args.cpu_reps} repetitions, "
                     f"median {med:.2f} s, mean {mean:.2f} s",
           "median_s": round(med, 3), "mean_s": round(mean, 3)}

    def phases(graphs, threads_):
        oracle.set_threads(threads_)
        pts = []

        def run():
            pt = {}
            for x in graphs:
                oracle.louvain(x, phase_times=pt)
            pts.append(pt)
        med_, mean_ = reps(run, 5)
        keys = ("local_move", "renumber", "aggregate", "other")
        ph = {k: round(float(np.median([p[k] for p in pts[1:]])) * 1e3, 3) for k in keys}
        return {"threads": threads_, "ms_median": round(med_ * 1e3, 3), "ms_mean": round(mean_ * 1e3, 3),
                "phase_ms_median": ph}

    sbm = graphgen.sbm(4096, 128, 0.05, 0.0005, seed=1)
    sample = graphgen.batch_mix(args.cpu_batch_sample, seed=4)
    try:
        out["phases"] = {
            "sbm_4096": {"all_threads": phases([sbm], threads), "one_thread": phases([sbm], 1)},
            "batch_sample": {"graphs": len(sample), "entries": int(sum(x.nnz for x in sample)),
                             "all_threads": phases(sample, threads), "one_thread": phases(sample, 1)},
        }
    finally:
        oracle.set_threads(threads)
    log(f"cpu baseline: {out}")
    return out


def workloads_leg(args, lvp, graphgen, np, torch):
    """The other single-graph configurations: the 4,096-vertex SBM (Louvain)
    and the LFR-style graph (Louvain and LPA), each device-resident before
    timing; local-move rate from the levels' sweep events."""
    out = {}

    def run(name, g, lpa, reps, golden=None):
        with lvp.Graph.from_csr(g, validate=False) as dg:
            def step():
                r = lvp.louvain(dg, level_labels=False)
                lp = lvp.lpa(dg) if lpa else None
                return r, lp
            step()
            torch.cuda.synchronize()
            res, t0 = [], time.perf_counter()
            for _ in range(reps):
                res.append(step())
            torch.cuda.synchronize()
            wall = (time.perf_counter() - t0) / reps
        r = res[0][0]
        e = sum(lv.info["nnz"] * lv.info["sweeps"] for rr, _ in res for lv in rr.levels)
        ms = sum(lv.info["sweep_ms"] for rr, _ in res for lv in rr.levels)
        d = {"n": g.n, "nnz": g.nnz, "ms_per_step": round(wall * 1e3, 3), "levels": len(r.accepted), "q": r.q,
             "local_move_ms": round(ms / reps, 3), "local_move_gteps": round(e / (ms * 1e-3) / 1e9, 3) if ms else None,
             "sweeps_per_level": [lv.info["sweeps"] for lv in r.levels],
             "cached_sweeps_per_level": [lv.info["cached_sweeps"] for lv in r.levels],
             "step": "Louvain, all levels" + (" + LPA" if lpa else "")}
        if lpa:
            lms = sum(lp.info["sweep_ms"] for _, lp in res) / reps
            d["lpa_ms"] = round(lms, 3)
            d["lpa_sweeps"] = res[0][1].info["sweeps"]
        if golden and os.path.exists(golden):
            d["golden"] = digest_check(res[0][0], res[0][1], g, golden, name)
        log(f"workload {name}: {d}")
        return d

    out["sbm_4096"] = run("sbm_4096", graphgen.sbm(4096, 128, 0.05, 0.0005, seed=1), False, 20)
    t = time.time()
    g, _ = graphgen.lfr(args.lfr_n, seed=3)
    log(f"LFR n={g.n} nnz={g.nnz} generated in {time.time() - t:.1f}s")
    out["lfr"] = run("lfr", g, True, 3, golden=GOLDEN_LFR if args.lfr_n == 10_000_000 else None)
    out["lfr"]["workload"] = (f"LFR-style, n={g.n}, degree exponent 2.5, mean degree 20, max degree 5,000, "
                              "community sizes 50-20,000 (exponent 1.5), mixing 0.3, weights 1..8, seed 3")
    del g
    return out


def profile_summary(paths, out_dir, command, run_log=None):
    """Summaries for profiles/ from rocprofv3 databases of
    `bench.py --steps 1 --warmup 1 ... --copy-probe-mib 1024` (kernel trace,
    FETCH_SIZE pass, WRITE_SIZE pass, TCC hit/miss pass): per kernel, the
    dispatches of the instrumented step's Louvain (all levels: those between
    the first two of the three marker launches of the copy probe's kernel
    around its Louvain and LPA), averaged; the first launch of that kernel is
    the 1 GiB calibration copy, the next two enclose the timed steps (whose
    GPU idle time is summed).  run_log: the kernel-trace run's output
    (its JSON line gives the graph's entry count, for the probes'
    calibration on the gather pattern).
    Writes <out_dir>/move_kernels_rmat24_kernel_trace.md,
    move_kernels_rmat24_pmc.md and pmc_rmat24.txt (read by the roofline's
    `traffic`)."""
    import re
    import sqlite3

    def short(n):
        n = re.sub(r"^void |lv::\(anonymous namespace\)::|lv::", "", n).split("(")[0]
        return n

    def louvain_dispatches(db, part=0):
        con = sqlite3.connect(db)
        rows = con.execute("select dispatch_id, name, duration from kernels order by start").fetchall()
        marks = [i for i, r in enumerate(rows) if "bitwise_not" in r[1]]
        a, b = marks[-3 - part], marks[-2 - part]
        return con, rows[a + 1:b], rows[:marks[0] + 1]

    def copy_probe(rows):
        return [r for r in rows if "bitwise_not" in r[1]]

    names = {}
    con, sel, _ = louvain_dispatches(paths[0])
    dur = {}
    for d, n, t in sel:
        dur.setdefault(short(n), []).append(t / 1e6)
    counters = {}
    for key, db in zip(("fetch", "write", "hit"), paths[1:]):
        c2, sel2, rows2 = louvain_dispatches(db)
        ids = {d: short(n) for d, n, _ in sel2}
        probe_ids = {d for d, _, _ in copy_probe(rows2)}
        vals, pv = {}, {}
        for d, cn, v in c2.execute("select dispatch_id, counter_name, value from counters_collection"):
            if d in ids:
                vals.setdefault((ids[d], cn), {}).setdefault(d, 0.0)
                vals[(ids[d], cn)][d] += v
            if d in probe_ids:
                pv[cn] = pv.get(cn, 0.0) + v
        counters[key] = (vals, pv)
    gib_kib = (1 << 30) / 1024.0
    fetch_factor = counters["fetch"][1].get("FETCH_SIZE", 0.0) / gib_kib
    write_factor = counters["write"][1].get("WRITE_SIZE", 0.0) / gib_kib

    def avg(key, kern, cn):
        d = counters[key][0].get((kern, cn), {})
        return sum(d.values()) / len(d) if d else None

    src = kernel_source_digest()
    rows_out = []
    for kern, ts in sorted(dur.items(), key=lambda kv: -sum(kv[1])):
        f, w = avg("fetch", kern, "FETCH_SIZE"), avg("write", kern, "WRITE_SIZE")
        h, m = avg("hit", kern, "TCC_HIT_sum"), avg("hit", kern, "TCC_MISS_sum")
        rows_out.append((kern, len(ts), sum(ts) / len(ts), sum(ts), f, w, h, m))
    # the timed step (captured sweeps): GPU busy and idle between its first
    # and last dispatch, from the kernel trace
    con0 = sqlite3.connect(paths[0])
    allk = con0.execute("select name, start, end from kernels order by start").fetchall()
    mk = [i for i, r in enumerate(allk) if "bitwise_not" in r[0]]
    step = allk[mk[1] + 1:mk[2]]  # between the markers around the timed steps
    idle = busy = span = 0.0
    gaps10 = 0
    if step:
        edge = step[0][2]
        busy = (step[0][2] - step[0][1]) / 1e6
        for nme, st, en in step[1:]:
            gap = max(0, st - edge) / 1e6
            idle += gap
            gaps10 += gap > 0.01
            busy += max(0, en - max(st, edge)) / 1e6
            edge = max(edge, en)
        span = (edge - step[0][1]) / 1e6
    # the library's probes, on the same graph: a 16-byte copy of the index
    # array and the pure gather (index stream + one random 8-byte pair per entry)
    nnz = None
    if run_log and os.path.exists(run_log):
        import json
        for line in open(run_log):
            if line.startswith("{") and '"metric"' in line:
                nnz = json.loads(line)["config"]["nnz"]

    def probe_avg(db, name, counter):
        c = sqlite3.connect(db)
        ids = {d for d, n in c.execute("select dispatch_id, name from kernels") if name in n}
        vals = {}
        for d, cn, v in c.execute("select dispatch_id, counter_name, value from counters_collection"):
            if d in ids and cn == counter:
                vals[d] = vals.get(d, 0.0) + v
        return sum(vals.values()) / len(vals) if vals else None

    probes = {}
    for pn in ("k_probe_copy", "k_probe_gather"):
        probes[pn] = (probe_avg(paths[1], pn, "FETCH_SIZE"), probe_avg(paths[2], pn, "WRITE_SIZE"),
                      probe_avg(paths[3], pn, "TCC_HIT_sum"), probe_avg(paths[3], pn, "TCC_MISS_sum"))
    _, sel_lpa, _ = louvain_dispatches(paths[0], part=-1)
    dur_lpa = {}
    for d, n, t in sel_lpa:
        dur_lpa.setdefault(short(n), []).append(t / 1e6)
    os.makedirs(out_dir, exist_ok=True)
    with open(os.path.join(out_dir, "move_kernels_rmat24_kernel_trace.md"), "w") as fh:
        fh.write("# Kernel trace: R-MAT 24, the instrumented step\n\n")
        fh.write("Command (run from the repository root on the GPU host, with `cd /tmp && export TMPDIR=/tmp` for the "
                 "profiler's files):\n\n```\n" + command[0] + "\n```\n\n")
        fh.write("Dispatches between the marker launches around the instrumented step's Louvain (all levels), "
                 "grouped by kernel.  bench.py's roofline takes its dominant kernel's average from HIP events on "
                 "the same calls.  Sum of the dispatches: %.3f ms.\n\n| kernel | dispatches | avg ms | total ms |\n"
                 "|---|---:|---:|---:|\n" % sum(r[3] for r in rows_out))
        for kern, nd, a, t, *_ in rows_out[:40]:
            fh.write(f"| `{kern}` | {nd} | {a:.4f} | {t:.3f} |\n")
        fh.write(f"\nThe timed steps before it (captured sweeps, Louvain and LPA): {span:.2f} ms from the first to "
                 f"the last dispatch, GPU busy {busy:.2f} ms, idle {idle:.2f} ms between dispatches ({gaps10} gaps "
                 f"over 10 us).\n")
        tot = sum(sum(v) for v in dur_lpa.values())
        fh.write("\nLPA of the same step (launched for every sweep up to the limit; after the stopping rule a "
                 "dispatch returns at once): sum of the dispatches %.3f ms.\n\n| kernel | dispatches | avg ms | "
                 "total ms |\n|---|---:|---:|---:|\n" % tot)
        for kern, ts in sorted(dur_lpa.items(), key=lambda kv: -sum(kv[1]))[:20]:
            fh.write(f"| `{kern}` | {len(ts)} | {sum(ts) / len(ts):.4f} | {sum(ts):.3f} |\n")
    with open(os.path.join(out_dir, "move_kernels_rmat24_pmc.md"), "w") as fh:
        fh.write("# HBM counters: R-MAT 24, the instrumented step's Louvain (all levels)\n\nThree rocprofv3 passes, one counter "
                 "group each:\n\n```\n" + "\n".join(command[1:]) + "\n```\n\n")
        fh.write(f"Calibration: the 1 GiB copy probe (torch bitwise_not: 1 GiB read, 1 GiB written) reads "
                 f"FETCH_SIZE = {fetch_factor:.4f} x its bytes read and WRITE_SIZE = {write_factor:.4f} x its bytes "
                 "written (KiB).  Calibrated bytes = FETCH_SIZE / fetch factor + WRITE_SIZE / write factor.  These "
                 "TCC counters see requests from L2 to the memory fabric: a line served by the Infinity Cache (MALL) "
                 "is counted like one from HBM, so 'HBM bytes' here is an upper bound on DRAM traffic.\n\n")
        if nnz:
            fh.write("The library's probes over the same graph's index array (E = %d entries), per dispatch:\n\n"
                     "| probe | requested bytes | FETCH_SIZE / requested read | WRITE_SIZE / requested write | "
                     "L2 hit %% |\n|---|---:|---:|---:|---:|\n" % nnz)
            for pn, rd, wr in (("k_probe_copy", 4 * nnz, 4 * nnz), ("k_probe_gather", 12 * nnz, 0)):
                f_, w_, h_, m_ = probes[pn]
                if f_ is None:
                    continue
                hit = 100.0 * h_ / (h_ + m_) if h_ is not None and m_ and h_ + m_ > 0 else float("nan")
                wtxt = f"{w_ * 1024 / wr:.3f}" if wr and w_ is not None else "-"
                fh.write(f"| `{pn}` | {rd + wr} | {f_ * 1024 / rd:.3f} | {wtxt} | {hit:.1f} |\n")
            fh.write("\nThe copy probe reads the index array once (4E bytes read, 4E written); the gather probe "
                     "streams it and gathers one random 8-byte pair per entry from an n-entry table (12E bytes "
                     "requested).  Its FETCH_SIZE per requested byte, over the copy's, is the line amplification "
                     "of random 8-byte gathers on this graph (the 134 MB table fits in the Infinity Cache, whose "
                     "hits these counters cannot tell from HBM reads).\n\n")
        fh.write("| kernel | dispatches | avg ms | FETCH_SIZE MiB | WRITE_SIZE MiB | calibrated MB | L2 hit % |\n"
                 "|---|---:|---:|---:|---:|---:|---:|\n")
        for kern, nd, a, t, f, w, h, m in rows_out[:40]:
            if f is None or w is None:
                continue
            cal = (f / max(fetch_factor, 1e-9) + w / max(write_factor, 1e-9)) * 1024 / 1e6
            hit = 100.0 * h / (h + m) if h is not None and m and (h + m) > 0 else float("nan")
            fh.write(f"| `{kern}` | {nd} | {a:.4f} | {f / 1024:.2f} | {w / 1024:.2f} | {cal:.1f} | {hit:.1f} |\n")
    with open(os.path.join(out_dir, "pmc_rmat24.txt"), "w") as fh:
        fh.write("# Per-dispatch HBM counters of the move kernels on R-MAT 24 (see move_kernels_rmat24_pmc.md);\n"
                 "# fetch_kib / write_kib: FETCH_SIZE / WRITE_SIZE averaged over the instrumented step's Louvain\n"
                 "# dispatches of the kernel, copy_*_factor: the counter's reading per byte of a plain 1 GiB copy;\n"
                 "# src: digest of the kernels' code (comments and white space left out) when taken.\n")
        for kern, nd, a, t, f, w, h, m in rows_out:
            slot = KERNEL_SLOT_OF(kern)
            if slot is None or f is None or w is None:
                continue
            fh.write(f"slot={slot} kernel={kern.replace(' ', '')} dispatches={nd} fetch_kib={f:.1f} write_kib={w:.1f} "
                     f"copy_fetch_factor={fetch_factor:.4f} copy_write_factor={write_factor:.4f} src={src}\n")


def KERNEL_SLOT_OF(kern):
    """The library's timing-slot name of a profiled kernel symbol (None: not
    a kernel that a slot times alone)."""
    import re

    names = ["l4", "l8", "l32", "l128", "l256", "l512", "l1k", "l2k", "l3k", "l8k"]
    m = re.match(r"k_move_claim<(\d+),", kern)
    if m and 1 <= int(m.group(1)) <= 10:
        return names[int(m.group(1)) - 1]
    m = re.match(r"k_move<(\d+),.*, 0>$", kern)
    if m and 1 <= int(m.group(1)) <= 10:
        return names[int(m.group(1)) - 1] + "/first"
    if kern.startswith("k_hub_scatter"):
        return "hub/scatter"
    if kern.startswith("k_hub_part_claim"):
        return "hub"
    if kern.startswith("k_hub_part<true"):
        return "hub/first"
    if kern.startswith("k_move_fused"):
        return "fused"
    return None


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--profile-summary":
        # bench.py --profile-summary OUT_DIR KT_DB FETCH_DB WRITE_DB HIT_DB CMD_KT CMD_FETCH CMD_WRITE CMD_HIT [KT_LOG]
        a = sys.argv[2:]
        profile_summary(a[1:5], a[0], a[5:9], a[9] if len(a) > 9 else None)
        return
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--scale", type=int, default=24)
    ap.add_argument("--edge-factor", type=float, default=16.0)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--cpu-sweeps", type=int, default=2, help="oracle sweeps per timed cpu_baseline repetition")
    ap.add_argument("--cpu-reps", type=int, default=5, help="timed cpu_baseline repetitions (after one warm-up)")
    ap.add_argument("--cpu-batch-sample", type=int, default=8, help="batch graphs in the per-phase CPU sample")
    ap.add_argument("--no-workloads", action="store_true", help="skip the SBM and LFR legs")
    ap.add_argument("--lfr-n", type=int, default=10_000_000, help="vertices of the LFR leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--batch-graphs", type=int, default=4096, help="graphs in the batch leg (0: skip it)")
    ap.add_argument("--batch-sample", type=int, default=256, help="graphs run one per call for the baseline")
    ap.add_argument("--batch-reps", type=int, default=3)
    ap.add_argument("--serve-jobs", type=int, default=1000, help="jobs in the serving trace (0: skip it)")
    ap.add_argument("--serve-pool", type=int, default=32, help="distinct graphs the jobs draw from")
    ap.add_argument("--serve-loads", type=float, nargs="+", default=[0.8, 0.95],
                    help="arrival rates / one-per-call capacity, one trace each")
    ap.add_argument("--serve-max-jobs", type=int, default=64)
    ap.add_argument("--serve-capacity-jobs", type=int, default=200, help="jobs of the saturated capacity runs")
    ap.add_argument("--prune-reps", type=int, default=2,
                    help="timed steps with active-vertex pruning (LV_PRUNE) after the main steps (0: skip)")
    ap.add_argument("--async-reps", type=int, default=2,
                    help="timed steps with asynchronous sweeps (LV_ASYNC) after the main steps (0: skip)")
    ap.add_argument("--no-edges-leg", action="store_true",
                    help="skip building the graph from its raw R-MAT samples on the device")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB before the steps (PMC calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path (no sharding, no collectives), "
              f"so --gpus {args.gpus} is refused", file=sys.stderr, flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    import graphgen
    import paper_2507_06471_amd as lvp

    torch.cuda.init()
    log(f"device {torch.cuda.get_device_name(0)}; host nproc {os.cpu_count()}")
    t = time.time()
    g = graphgen.rmat(args.scale, args.edge_factor, seed=args.seed)
    log(f"generated R-MAT scale {args.scale}: n={g.n} nnz={g.nnz} in {time.time() - t:.1f}s")
    t = time.time()
    dg = lvp.Graph.from_csr(g, validate=True)
    log(f"graph resident on the device in {time.time() - t:.1f}s (volume M={dg.volume})")

    if args.copy_probe_mib > 0:
        # a plain streaming kernel of known size under a name no other kernel
        # here has: reads and writes copy_probe_mib MiB
        src = torch.ones(args.copy_probe_mib << 18, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.bitwise_not(src, out=dst)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe_mib} MiB read + {args.copy_probe_mib} MiB written")
        del src, dst

    def profile_marker():
        # with the copy probe on, a 1 KiB launch of the same kernel before
        # and after the instrumented step marks its dispatches in a trace
        if args.copy_probe_mib > 0:
            torch.cuda.synchronize()
            torch.bitwise_not(torch.ones(256, dtype=torch.int32, device="cuda"))
            torch.cuda.synchronize()

    def step(timing, out=None):
        # the job's results: final labels and per-level statistics of Louvain,
        # labels of LPA (the per-level labels stay on the device).  With `out`
        # (two int32 device tensors) both label arrays stay in HBM; without it
        # they are copied to host memory.
        r = lvp.louvain(dg, timing=timing, level_labels=False, out=None if out is None else out[0])
        lp = lvp.lpa(dg, timing=timing, out=None if out is None else out[1])
        return r, lp

    # each timed step leaves its labels in HBM, in buffers of its own
    outs = [(torch.empty(g.n, dtype=torch.int32, device="cuda"), torch.empty(g.n, dtype=torch.int32, device="cuda"))
            for _ in range(max(args.steps, 1))]

    for w in range(args.warmup):
        t = time.time()
        r, lp = step(timing=False, out=outs[0])
        log(f"warmup {w}: {time.time() - t:.2f}s, levels {len(r.accepted)}, Q={r.q:.6f}")

    # timed steps: the production path (captured sweeps, concurrent classes)
    profile_marker()  # before the timed steps (outside the timed region)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = []
    for k in range(args.steps):
        ts = time.perf_counter()
        runs.append(step(timing=False, out=outs[k]))
        log(f"step {k}: {time.perf_counter() - ts:.3f}s")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    profile_marker()  # after the timed steps (outside the timed region)
    # the labels to host memory, after the timed region
    for r, lp in runs:
        r.final_labels = r.final_labels.cpu().numpy()
        lp.labels = lp.labels.cpu().numpy()
    del outs
    for r, lp in runs[1:]:
        assert np.array_equal(r.final_labels, runs[0][0].final_labels) and np.array_equal(lp.labels, runs[0][1].labels)
    golden = golden_check(args, runs[0][0], runs[0][1], g)

    # local-move throughput from the phase events of the timed steps
    lm_edges = lm_ms = lpa_edges = lpa_ms = 0.0
    phases = {"local_move_ms": 0.0, "renumber_ms": 0.0, "aggregate_ms": 0.0, "lpa_ms": 0.0}
    for r, lp in runs:
        for lv in r.levels:
            i = lv.info
            lm_edges += i["nnz"] * i["sweeps"]
            lm_ms += i["sweep_ms"]
            phases["local_move_ms"] += i["sweep_ms"]
            phases["renumber_ms"] += i["renumber_ms"]
            phases["aggregate_ms"] += i["aggregate_ms"]
        lpa_edges += lp.info["nnz"] * lp.info["sweeps"]
        lpa_ms += lp.info["sweep_ms"]
        phases["lpa_ms"] += lp.info["sweep_ms"]
    K = len(runs)
    # per-kernel figures from one instrumented step after the timed region
    # (kernels launched one at a time with HIP events around each)
    kern_ms = np.zeros(lvp.KERNEL_SLOTS)
    kern_launches = np.zeros(lvp.KERNEL_SLOTS, dtype=np.int64)
    kern_bytes = np.zeros(lvp.KERNEL_SLOTS, dtype=np.int64)
    profile_marker()
    ri = lvp.louvain(dg, timing=True, level_labels=False)
    profile_marker()
    lvp.lpa(dg, timing=True)
    profile_marker()
    for lv in ri.levels:
        i = lv.info
        kern_ms += np.array(i["kern_ms"])
        kern_launches += np.array(i["kern_launches"], dtype=np.int64)
        kern_bytes += np.array(i["kern_bytes"], dtype=np.int64)
    assert ri.q_int == runs[0][0].q_int and np.array_equal(ri.final_labels, runs[0][0].final_labels)
    gteps = lm_edges / (lm_ms * 1e-3) / 1e9 if lm_ms > 0 else 0.0
    lpa_gteps = lpa_edges / (lpa_ms * 1e-3) / 1e9 if lpa_ms > 0 else 0.0
    levels, all_frac = level_roofline(runs)
    lpa0 = runs[0][1].info
    lpa_b = (8 * lpa0["nnz"] + 12 * lpa0["n"]) * lpa0["sweeps"]
    lpa_frac = lpa_b / (lpa_ms / K * 1e-3) / (HBM_PEAK_GBS * 1e9) if lpa_ms > 0 else None
    # dominant kernel: the longest-running single move kernel that reads the
    # graph (the hub partition slot reads only the scatter pass's buckets; the
    # commit and cache-refresh slots carry no compulsory bytes)
    dom = int(np.argmax(np.where(kern_bytes > 0, kern_ms, -1.0)))
    avg_launch_ms = kern_ms[dom] / max(1, kern_launches[dom])
    bytes_per_launch = kern_bytes[dom] / max(1, kern_launches[dom])
    achieved = bytes_per_launch / (avg_launch_ms * 1e-3) / 1e9 if avg_launch_ms > 0 else 0.0
    all_bytes = kern_bytes.sum()
    all_gbs = all_bytes / (kern_ms.sum() * 1e-3) / 1e9 if kern_ms.sum() > 0 else 0.0
    r0 = runs[0][0]
    kernels = {lvp.KERNEL_NAMES[s]: {"ms_total": round(float(kern_ms[s]), 4),
                                     "launches": int(kern_launches[s]),
                                     "gbs": round(float(kern_bytes[s] / (kern_ms[s] * 1e-3) / 1e9), 1)}
               for s in range(lvp.KERNEL_SLOTS) if kern_launches[s] > 0}

    # consistency: reported Q equals the modularity of the reported labels
    qi, m, q = lvp.modularity(dg, r0.final_labels)
    assert (qi, m) == (r0.q_int, r0.M), "reported modularity differs from the labels' modularity"

    # the pure-gather ceiling of the move kernels on this graph (stored order):
    # one random 8-byte pair per entry and nothing else
    ceiling = lvp.probe_gather(dg, reps=5)
    gather_ceiling = {"entries_per_s": round(ceiling / 1e9, 3), "unit": "G entries/s",
                      "local_move": round(gteps, 3), "frac": round(gteps * 1e9 / ceiling, 4) if ceiling > 0 else None,
                      "probe": "lv_probe_gather: stream the stored column indices, gather one 8-byte pair each"}
    log(f"gather ceiling: {gather_ceiling}")
    # a STREAM-style copy of the index array with the library's probe kernel:
    # the measured bandwidth beside the 8 TB/s peak
    copy_bps = lvp.probe_copy(dg, reps=5)
    stream_copy = {"gbs": round(copy_bps / 1e9, 1), "frac_of_peak": round(copy_bps / 8.0e12, 4),
                   "dominant_kernel_frac": round(float(achieved) * 1e9 / copy_bps, 4) if copy_bps > 0 else None,
                   "probe": "lv_probe_copy: 16-byte copy of the stored column indices, bytes read + written"}
    log(f"stream copy: {stream_copy}")
    pruned = prune_leg(args, lvp, dg, runs, phases, K, torch) if args.prune_reps > 0 else None
    asynchronous = async_leg(args, lvp, dg, runs, phases, K, torch) if args.async_reps > 0 else None
    edges = None if args.no_edges_leg else edges_leg(args, lvp, graphgen, g, np, torch)

    parity = None
    cpu = None
    if not args.no_cpu_baseline or not args.no_parity:
        import oracle

        adj = oracle.adjacency(g)
        if not args.no_cpu_baseline:
            cpu = cpu_baseline(args, oracle, adj, g, graphgen, np)
        if not args.no_parity:
            # GPU first sweep (one sweep, one level) vs the oracle's first sweep, renumbered
            c1, mv1 = oracle.local_move(adj, oracle.LOUVAIN, max_sweeps=1)
            r1 = lvp.louvain(dg, max_sweeps=1, max_levels=1)
            want_lab, _ = oracle.renumber(c1)
            got_lab = r1.levels[0].labels if r1.levels[0].info["accepted"] else None
            ok = got_lab is not None and np.array_equal(got_lab, want_lab) and r1.levels[0].moves[0] == int(mv1[0])
            parity = {"first_sweep_partition_equal": bool(ok), "first_sweep_moves": int(mv1[0]),
                      "labels_checked": int(g.n),
                      "all_levels_equal_to_golden_digests": None if golden is None else golden["equal"]}
            log(f"parity: {parity}")
            if not ok:
                print("first-sweep partition differs from the oracle", file=sys.stderr, flush=True)
                sys.exit(1)
        del adj

    dg.close()
    gn, gnnz = g.n, g.nnz
    del g
    workloads = None if args.no_workloads else workloads_leg(args, lvp, graphgen, np, torch)
    batch = batch_leg(args, lvp, graphgen, np, torch) if args.batch_graphs > 0 else None
    serving = serving_leg(args, lvp, graphgen, np, torch) if args.serve_jobs > 0 else None

    out = {
        "metric": METRIC,
        "value": round(gteps, 4),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(wall / K * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": f"R-MAT scale {args.scale}, edge factor {args.edge_factor:g} (a=0.57, b=0.19, "
                               "c=0.19), symmetrised, loops/duplicates removed, unit weights; Louvain all levels "
                               "+ LPA max 20 sweeps",
                   "n": gn, "nnz": gnnz, "seed": args.seed},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(lvp.KERNEL_NAMES[dom]) if args.scale == 24 else None,
                     "kernel": lvp.KERNEL_NAMES[dom], "avg_launch_ms": round(float(avg_launch_ms), 4),
                     "bytes_per_launch": int(bytes_per_launch),
                     "bytes_model": "8 per CSR entry + 36 per vertex of the kernel's rows (per launch)",
                     "level0_frac": levels[0]["frac"] if levels else None,
                     "all_levels_frac": round(all_frac, 4) if all_frac is not None else None,
                     "lpa_frac": round(lpa_frac, 4) if lpa_frac is not None else None,
                     "level0_ms_per_sweep": levels[0]["ms_per_sweep"] if levels else None,
                     "sweep_bytes_model": "8E + 36n per sweep (LPA: 8E + 12n)",
                     "levels": levels},
        "gather_ceiling": gather_ceiling, "stream_copy": stream_copy,
        "cpu_baseline": cpu,
        "paper_context": PAPER_CONTEXT,
        "parity": parity,
        "golden": golden,
        "workloads": workloads,
        "louvain": {"levels": len(r0.accepted), "q": r0.q, "q_int": r0.q_int, "M": r0.M,
                    "sweeps_per_level": [lv.info["sweeps"] for lv in r0.levels],
                    "n_per_level": [lv.info["n"] for lv in r0.levels],
                    "move_kernels_all_gbs": round(float(all_gbs), 1)},
        "lpa": {"gteps": round(lpa_gteps, 4), "sweeps": runs[0][1].info["sweeps"], "q": runs[0][1].info["q_end"] / float(dg.volume) ** 2},
        "phase_ms_per_step": {k_: round(v / K, 3) for k_, v in phases.items()},
        "kernels": kernels,
        "pruned": pruned,
        "asynchronous": asynchronous,
        "edges_to_csr": edges,
        "batch": batch,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
