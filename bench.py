#!/usr/bin/env python3
"""Benchmark of the buffer k-d tree exact kNN query on one MI355X.

One step = one complete query call (Algorithm 1 to completion: every
FindLeafBatch, buffer insertion, ProcessAllBuffers leaf scan and the final
conversion) over all m queries of the workload, with the tree built and the
queries resident in HBM before the timed region starts.  Prints one JSON line.

Workloads (seeded synthetic stand-ins for the paper's catalogues, Section 4.1):
  ondevice  n = m = 2^22, d = 10, 16-component Gaussian mixture, k = 10, height 10 (default)
  small     n = 2^15, m = 2^12, d = 10 uniform on [0,1]^10, k = 10, height 6
  streamed  n = 2^28, m = 2^24, same mixture, k = 10, height 14, leaf structure streamed
            through a 2 GB device budget (Section 3.2); also times the same tree resident
  batched   1024 instances, n = 2^U(10,18), m = 2^U(8,16), d in {3,5,10,15}, k in {1,5,10,32},
            4-component mixtures, height floor(log2(n/64)), one persistent graph launch;
            also times the plain per-instance loop on the same GPU
  served    two resident trees (n = 2^27, d = 10, height 14; n = 2^25, d = 15, height 12),
            Poisson requests of m = 2^U(0,16) queries, k in {1,10,32}: saturated throughput
            (closed loop), then p50/p99 latency at 0.5 and 0.8 of it (open loop)
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import datagen  # noqa: E402

T_START = time.perf_counter()


def note(msg):
    """Progress of a long run, on stderr (the JSON line stays alone on stdout)."""
    print(f"bench [{time.perf_counter() - T_START:6.1f} s]: {msg}", file=sys.stderr, flush=True)

# Peaks of one MI355X (vendor figures).
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3  # vendor FP32 vector figure (counts packed dual-rate FP32)
F16_MATRIX_PEAK_TFLOPS = 2500.0  # vendor dense float16 (and bfloat16) matrix-core figure, no sparsity
FP32_NONPACKED_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12  # 256 CU x 64 lanes x FMA x 2.4 GHz = 78.6

WORKLOADS = {
    "ondevice": dict(n=1 << 22, m=1 << 22, d=10, k=10, h=10, kind="mixture", comps=16),
    "small": dict(n=1 << 15, m=1 << 12, d=10, k=10, h=6, kind="uniform", comps=0),
    "streamed": dict(n=1 << 28, m=1 << 24, d=10, k=10, h=14, kind="mixture", comps=16, budget=2_000_000_000),
}


# the dense scan's source, its instantiations, the constants that shape its launches (query tile,
# dense threshold, launch arguments) and the build flags: counters taken before a change to any of
# them no longer describe the launch
KERNEL_FILES = ("paper_1512_02831_amd/csrc/leaf_scan.h", "paper_1512_02831_amd/csrc/scan_inst.h",
                "paper_1512_02831_amd/csrc/internal.h", "paper_1512_02831_amd/compile.py")


def kernel_source_hash():
    """sha256 over the dense scan's source, its instantiation macros and the compile flags."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_FILES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def dense_scan_traffic(summary="profiles/k_leaf_scan_ondevice_n2p22.md"):
    """HBM bytes per dense-scan launch from the committed FETCH_SIZE/WRITE_SIZE summary, or None
    when the kernel's source or build flags have changed since those counters were taken."""
    try:
        text = open(os.path.join(ROOT, summary)).read()
        digest = kernel_source_hash()
    except OSError:
        return None
    fields = dict(line.split(":", 1) for line in text.splitlines()
                  if line.startswith(("traffic_bytes_per_launch:", "source_sha256:")))
    if "source_sha256" not in fields or fields["source_sha256"].split()[0] != digest:
        return None
    return int(fields["traffic_bytes_per_launch"])


def h2d_rate_gbs(torch, nbytes=1 << 30):
    """Pinned host-to-device copy rate of this machine (one 1 GiB copy after a warm-up)."""
    src = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
    dst = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst.copy_(src, non_blocking=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dst.copy_(src, non_blocking=True)
    torch.cuda.synchronize()
    return nbytes / (time.perf_counter() - t0) / 1e9


def timed_steps(bkd, torch, tree, dQ, k, di, dd, stream, steps, warmup):
    for _ in range(warmup):
        bkd.query_async(tree, dQ, k, di, dd, stream=stream)
    torch.cuda.synchronize()
    keys = ("dense_ms", "dense_launches", "dense_pairs", "sparse_ms", "sparse_launches", "sparse_pairs", "pairs",
            "calls", "chunk_copies", "bytes_h2d", "visits", "dense_visits", "alg_bytes", "alg_bytes_dense",
            "find_ms", "group_ms", "copy_ms", "wait_ms")
    acc = {key: 0 for key in keys}
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(steps):
        bkd.query_async(tree, dQ, k, di, dd, stream=stream)
        st = bkd.last_stats(tree)
        for key in acc:
            acc[key] += st[key]
    ev1.record(stream)
    torch.cuda.synchronize()
    return acc, time.perf_counter() - t0, ev0.elapsed_time(ev1)


def make_inputs(w, seed):
    if w["kind"] == "uniform":
        return datagen.small_uniform(seed, w["n"], w["m"], w["d"])
    return datagen.mixture_pq(seed, w["n"], w["m"], w["d"], w["comps"])


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def cpu_baseline(P, Q, k, budget_s, fixed=None, m_total=None):
    """The oracle's float64 k-d tree (leaf size 32), OpenMP over queries on every host core.
    fixed: time exactly the first `fixed` queries; else a sample of about budget_s seconds."""
    import oracle
    threads = oracle.max_threads()
    tree = oracle.KdTree64(P, 32)
    if fixed is not None:
        ns = min(len(Q), fixed)
    else:
        # calibrate on a small sample, then time a bounded sample of about budget_s seconds
        cal = min(len(Q), 2048)
        t0 = time.perf_counter()
        tree.query(Q[:cal], k)
        rate = cal / max(time.perf_counter() - t0, 1e-6)
        ns = int(min(len(Q), max(cal, rate * budget_s)))
    t0 = time.perf_counter()
    tree.query(Q[:ns], k)
    dt = time.perf_counter() - t0
    return {"value": ns / dt, "unit": "queries/s", "cores": threads, "kind": "oracle",
            "sample": f"first {ns} of {m_total or len(Q)} queries against all {len(P)} points; float64 k-d tree, "
                      f"leaf size 32, OpenMP over queries ({threads} threads, {cpu_model()})"}


def run_batched(args, torch, bkd):
    shapes = datagen.batch_shapes(args.seed)
    inst = []
    for i, sh in enumerate(shapes):
        P, Q = datagen.batch_instance(args.seed, i, sh["n"], sh["m"], sh["d"])
        inst.append((P, Q, sh["k"], sh["h"]))
    total_m = sum(len(x[1]) for x in inst)
    stream = torch.cuda.Stream()
    b = bkd.batch_create(inst)
    best, best_ms = bkd.batch_autotune(b)
    for _ in range(args.warmup):
        bkd.batch_run(b, stream=stream)
    torch.cuda.synchronize()
    run_ms = 0.0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        bkd.batch_run(b, stream=stream)
        stream.synchronize()
        st = bkd.batch_stats(b)
        run_ms += st["run_ms"]
        if st["error"]:
            raise RuntimeError(f"batched launch stopped early: {st}")
    wall = time.perf_counter() - t0
    b.free()
    # the plain per-instance loop: one tree and one query call per instance, queries resident
    trees = [bkd.build(P, h, buffer_size=-1, fetch_size=-1) for (P, Q, k, h) in inst]
    dev = [(torch.from_numpy(Q).to("cuda"), torch.empty((len(Q), k), dtype=torch.int64, device="cuda"),
            torch.empty((len(Q), k), dtype=torch.float32, device="cuda")) for (P, Q, k, h) in inst]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for t, (P, Q, k, h), (dq, di, dd) in zip(trees, inst, dev):
        if len(Q):
            bkd.query_async(t, dq, k, di, dd, stream=stream)
    stream.synchronize()
    loop_s = time.perf_counter() - t1
    for t in trees:
        t.free()
    value = total_m * args.steps / wall
    flops = st["flops"]
    achieved = flops / (st["run_ms"] * 1e-3) / 1e12
    return {
        "metric": "kNN queries/s (batched form, 1024 instances)",
        "value": round(value, 1), "unit": "queries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batched: 1024 instances, seed {args.seed}, n=2^U(10,18) m=2^U(8,16) "
                               "d in {3,5,10,15} k in {1,5,10,32}, 4-component mixtures, height floor(log2(n/64)), "
                               "one persistent hipGraph launch per step",
                   "queries": total_m, "points": sum(len(x[0]) for x in inst),
                   "tuning": {"leaves_per_task": best.leaves_per_task, "groups_per_cu": best.groups_per_cu,
                              "solo_max": best.solo_max, "tuned_ms": round(best_ms, 3)},
                   "rounds": st["rounds"], "tasks": st["tasks"], "pairs": st["pairs"],
                   "plain_loop_queries_per_s": round(total_m / loop_s, 1),
                   "speedup_vs_plain_loop": round((total_m / (wall / args.steps)) / (total_m / loop_s), 2)},
        # device code is built without packed FP32, so the vector peak it can reach is the
        # non-packed 78.6 TFLOP/s (the vendor's 157.3 counts dual-rate packed FP32)
        "roofline": {"kernel": "k_batch (persistent)", "bound": "alu", "achieved": round(achieved, 3),
                     "peak": round(FP32_NONPACKED_TFLOPS, 1), "unit": "TFLOP/s",
                     "frac": round(achieved / FP32_NONPACKED_TFLOPS, 4), "traffic": None,
                     "peak_packed_vendor": FP32_VECTOR_PEAK_TFLOPS,
                     "avg_launch_ms": round(run_ms / args.steps, 4), "flops_per_launch": flops},
        **({} if args.no_cpu_baseline else {"cpu_baseline": cpu_baseline_batched(inst, args.cpu_seconds)}),
    }


def cpu_baseline_batched(inst, budget_s):
    """The oracle's float64 k-d tree per instance (build not timed), instances in order until the budget."""
    import oracle
    threads = oracle.max_threads()
    q = 0
    t = 0.0
    used = 0
    for P, Q, k, _ in inst:
        tree = oracle.KdTree64(P, 32)
        t0 = time.perf_counter()
        tree.query(Q, k)
        t += time.perf_counter() - t0
        q += len(Q)
        used += 1
        if t >= budget_s:
            break
    return {"value": q / t, "unit": "queries/s", "cores": threads, "kind": "oracle",
            "sample": f"all queries of the first {used} of {len(inst)} instances; float64 k-d tree per instance, "
                      f"leaf size 32, OpenMP over queries ({threads} threads, {cpu_model()})"}


def run_served(args, torch, bkd, plain_requests=600, cpu_queries=None):

    specs = [dict(n=1 << 27, d=10, h=14), dict(n=1 << 25, d=15, h=12)]
    trees, params, Ps = [], [], []
    for t, sp in enumerate(specs):
        seed = args.seed + 100 * (t + 1)
        pr = datagen.mixture_params(seed, sp["d"], 16)
        P = datagen.mixture(seed, datagen.STREAM_P, sp["n"], sp["d"], 16, pr)
        trees.append(bkd.build(P, sp["h"], buffer_size=-1, fetch_size=-1, flags=bkd.FLAG_DEVICE_BUILD))
        params.append((seed, pr))
        Ps.append(P if cpu_queries else None)
        del P
    note("served: trees built")
    srv = bkd.server_create(slots_per_session=1 << 21, age_max=args.served_age_max, tail_max=args.served_tail_max)
    tids = [bkd.server_add_tree(srv, t) for t in trees]

    def request_queries(trace):
        out = []
        for i, r in enumerate(trace):
            seed, pr = params[r["tree"]]
            g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 7, i])))
            means, stds = pr
            c = g.integers(0, len(means), size=r["m"])
            Q = (means[c] + stds[c] * g.standard_normal((r["m"], specs[r["tree"]]["d"]))).astype(np.float32)
            out.append(Q)
        return out

    def replay(trace, Qs, open_loop):
        hs = [None] * len(trace)
        t0 = time.perf_counter()
        for i, (r, Q) in enumerate(zip(trace, Qs)):
            if open_loop:
                delay = r["t"] - (time.perf_counter() - t0)
                if delay > 0:
                    time.sleep(delay)
            hs[i] = bkd.submit(srv, tids[r["tree"]], Q, r["k"])
        for h in hs:
            bkd.wait(srv, h)
        wall = time.perf_counter() - t0
        lat = np.array([bkd.request_times(srv, h)[2] - bkd.request_times(srv, h)[0] for h in hs])
        for h in hs:
            bkd.release(srv, h)
        return wall, lat

    # warm-up: one request per session (creates the sessions)
    warm = datagen.request_trace(args.seed + 1, 12, 1e9)
    replay(warm, request_queries(warm), False)
    # saturated throughput: every request submitted at once
    closed = datagen.request_trace(args.seed + 2, 600, 1e9)
    Qc = request_queries(closed)
    qc = sum(r["m"] for r in closed)
    s0 = bkd.server_stats(srv)
    wall_c, lat_c = replay(closed, Qc, False)
    x_sat = qc / wall_c
    s1 = bkd.server_stats(srv)
    closed_server = {f: (round(s1[f] - s0[f], 3) if f != "sessions" else s1[f]) for f in s1}
    # the plain per-batch loop: one query call per request, one after another (the first
    # plain_requests requests of the same trace)
    t1 = time.perf_counter()
    npl = min(len(closed), plain_requests)
    for r, Q in zip(closed[:npl], Qc[:npl]):
        bkd.query(trees[r["tree"]], Q, r["k"])
    loop_qps = sum(r["m"] for r in closed[:npl]) / (time.perf_counter() - t1)
    mean_m = (2 ** 16 - 1) / (16 * np.log(2))
    levels = {}
    for frac in (0.5, 0.8):
        note(f"served: open loop at {frac} of the saturated rate")
        rate = frac * x_sat / mean_m
        trace = datagen.request_trace(args.seed + int(frac * 10), args.served_requests, rate)
        Qs = request_queries(trace)
        wall, lat = replay(trace, Qs, True)
        levels[str(frac)] = {"offered_requests_per_s": round(rate, 2),
                             "offered_queries_per_s": round(frac * x_sat, 1),
                             "achieved_queries_per_s": round(sum(r["m"] for r in trace) / wall, 1),
                             "requests": len(trace), "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                             "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3)}
    srv.destroy()
    latency_mode = None
    if args.served_latency_age_max > 0:
        # the same trees and traces with the age hand-over: a query still travelling after
        # that many rounds finishes its traversal alone, which bounds a request's round count
        # (lower latency, lower saturated rate)
        note(f"served: age hand-over after {args.served_latency_age_max} rounds")
        srv = bkd.server_create(slots_per_session=1 << 21, age_max=args.served_latency_age_max,
                                tail_max=args.served_tail_max)
        tids = [bkd.server_add_tree(srv, t) for t in trees]
        replay(warm, request_queries(warm), False)
        wall_l, _ = replay(closed, Qc, False)
        x_sat_l = qc / wall_l
        rate = 0.5 * x_sat_l / mean_m
        trace = datagen.request_trace(args.seed + 5, args.served_requests // 4, rate)
        wall, lat = replay(trace, request_queries(trace), True)
        latency_mode = {"age_max": args.served_latency_age_max, "saturated_queries_per_s": round(x_sat_l, 1),
                        "open_loop_0.5": {"offered_queries_per_s": round(0.5 * x_sat_l, 1),
                                          "achieved_queries_per_s": round(sum(r["m"] for r in trace) / wall, 1),
                                          "requests": len(trace),
                                          "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                                          "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3)}}
        srv.destroy()
    for t in trees:
        t.free()
    cpu = None
    if cpu_queries:
        note("served: CPU oracle baseline")
        cpu = cpu_baseline_served(Ps, closed, Qc, cpu_queries)
    del Ps
    out = {
        "metric": "kNN queries/s (served form) + p50/p99 latency at fixed offered load",
        "value": round(x_sat, 1), "unit": "queries/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": round(wall_c * 1e3, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "served: trees n=2^27 d=10 h=14 and n=2^25 d=15 h=12 (16-component mixtures), "
                               "requests m=floor(2^U(0,16)), k in {1,10,32}, tree uniform; saturated throughput "
                               f"from {len(closed)} requests submitted at once, latency from Poisson arrivals",
                   "age_max": args.served_age_max, "tail_max": args.served_tail_max,
                   "closed_loop_requests": len(closed), "closed_loop_queries": qc,
                   "closed_loop_server": closed_server,
                   "closed_loop_p50_ms": round(float(np.percentile(lat_c, 50)) * 1e3, 3),
                   "closed_loop_p99_ms": round(float(np.percentile(lat_c, 99)) * 1e3, 3),
                   "plain_loop_queries_per_s": round(loop_qps, 1),
                   "plain_loop_requests": npl,
                   "speedup_vs_plain_loop": round(x_sat / loop_qps, 2),
                   "open_loop": levels,
                   "latency_mode": latency_mode},
    }
    if cpu:
        out["cpu_baseline"] = cpu
    return out


def cpu_baseline_served(Ps, trace, Qs, count):
    """The oracle's float64 k-d tree on the served workload: the requests of the closed-loop
    trace in order, each against its own tree with its own k, until `count` queries."""
    import oracle
    threads = oracle.max_threads()
    kd = [oracle.KdTree64(P, 32) for P in Ps]
    q = 0
    used = 0
    t = 0.0
    for r, Q in zip(trace, Qs):
        Q = Q[:count - q]
        t0 = time.perf_counter()
        kd[r["tree"]].query(Q, r["k"])
        t += time.perf_counter() - t0
        q += len(Q)
        used += 1
        if q >= count:
            break
    return {"value": q / t, "unit": "queries/s", "cores": threads, "kind": "oracle",
            "sample": f"the first {q} queries of the closed-loop trace ({used} requests), each against its tree "
                      f"(2^27 points d=10 or 2^25 points d=15) with its k; float64 k-d tree, leaf size 32, "
                      f"OpenMP over queries ({threads} threads, {cpu_model()})"}


def served_summary(args, torch, bkd):
    """The served workload as one object of the default line: saturated queries/s, p50/p99 at
    0.5 and 0.8 of it, the plain per-request loop on the first 100 requests, a 2^16-query
    CPU sample."""
    r = run_served(args, torch, bkd, plain_requests=100, cpu_queries=None if args.no_cpu_baseline else 1 << 16)
    keep = ("metric", "value", "unit", "ms_per_step", "higher_is_better", "dtype", "config", "cpu_baseline")
    return {key: r[key] for key in keep if key in r}


def key_capacity(k):
    """The key-list length the scan kernels are instantiated with for k neighbours."""
    return min(c for c in (1, 2, 4, 5, 8, 10, 16, 32, 64) if c >= k)


def run_outliers(args, torch, bkd):
    """Proximity-based outlier scores of the on-device reference set: every point of the
    n = 2^22 mixture is a query (k + 1 = 11 nearest), scored and ranked by bkd_outlier_scores
    (host arrays in and out, so the host link is inside the timed calls)."""
    w = WORKLOADS["ondevice"]
    n, d, k, h = w["n"], w["d"], w["k"], w["h"]
    P, _ = make_inputs(w, args.seed)
    tree = bkd.build(P, h, buffer_size=-1, fetch_size=-1, flags=bkd.FLAG_TIMING)
    for _ in range(args.warmup):
        bkd.outlier_scores(tree, P, k)
    times, dense_ms, dense_pairs, dense_launches = [], 0.0, 0, 0
    for _ in range(args.steps):
        t0 = time.perf_counter()
        bkd.outlier_scores(tree, P, k)
        times.append(time.perf_counter() - t0)
        st = bkd.last_stats(tree)
        dense_ms += st["dense_ms"]
        dense_pairs += st["dense_pairs"]
        dense_launches += st["dense_launches"]
    tree.free()
    wall = sum(times)
    achieved = 3.0 * d * dense_pairs / max(dense_ms * 1e-3, 1e-12) / 1e12
    out = {
        "metric": "outlier scores/s (all-nearest-neighbours, d=10, k=10)",
        "value": round(n * args.steps / wall, 1), "unit": "points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(wall * 1e3 / args.steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"outliers: the on-device reference set (n={n} d={d}, 16-component Gaussian "
                               f"mixture, seed {args.seed}, height {h}) scored against itself, k={k}, "
                               "host arrays in and out",
                   "n": n, "d": d, "k": k, "height": h},
        "roofline": {"kernel": f"k_leaf_scan<{d},{key_capacity(k + 1)}> (dense leaf scan, {k + 1} nearest)",
                     "bound": "mfma",
                     "achieved": round(achieved, 3), "peak": F16_MATRIX_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / F16_MATRIX_PEAK_TFLOPS, 4), "traffic": None,
                     "avg_launch_ms": round(dense_ms / max(dense_launches, 1), 4),
                     "share_of_step": round(dense_ms * 1e-3 / wall, 4)},
    }
    if not args.no_cpu_baseline:
        cb = cpu_baseline(P, P, k + 1, args.cpu_seconds)
        cb["unit"] = "points/s"
        cb["sample"] += " (the k + 1 nearest of each sampled point; the scoring itself is not timed)"
        out["cpu_baseline"] = cb
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="ondevice", choices=sorted(WORKLOADS) + ["batched", "served", "outliers"])
    ap.add_argument("--served-requests", type=int, default=2000, help="requests per open-loop level")
    ap.add_argument("--served-age-max", type=int, default=0,
                    help="served form: rounds after which a query leaves the rounds for a single walk (0: never)")
    ap.add_argument("--served-latency-age-max", type=int, default=64,
                    help="served form: also measure the age hand-over after this many rounds (0: skip)")
    ap.add_argument("--served-tail-max", type=int, default=0,
                    help="served form: queries in flight at or below which a round hands them to single walks "
                         "(0: the library default)")
    ap.add_argument("--seed", type=int, default=datagen.DEFAULT_SEED)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="CPU baseline sample size in seconds")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain 256 MiB device-to-device copy (counter calibration for profiles)")
    ap.add_argument("--headline-only", action="store_true",
                    help="default workload only: no streamed and served objects in the line")
    ap.add_argument("--streamed-steps", type=int, default=2, help="timed calls of the streamed object (1 warm-up)")
    ap.add_argument("--time-budget", type=float, default=480.0,
                    help="seconds from start within which the streamed and served objects must fit; "
                         "an object that would not fit is reported as skipped")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the query path has no multi-GPU form here "
              "(queries would shard by ranks with no exchange); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1512_02831_amd as bkd

    if args.calibrate_copy:
        src = torch.ones(256 << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload == "batched":
        print(json.dumps(run_batched(args, torch, bkd)), flush=True)
        return
    if args.workload == "served":
        print(json.dumps(run_served(args, torch, bkd, cpu_queries=None if args.no_cpu_baseline else 1 << 16)),
              flush=True)
        return
    if args.workload == "outliers":
        print(json.dumps(run_outliers(args, torch, bkd)), flush=True)
        return
    out = run_plain(args, torch, bkd, args.workload, args.steps, args.warmup)
    if args.workload == "ondevice" and not args.headline_only:
        # the other two configurations of the metric, each in an object of the same line:
        # the bigger-than-budget (streamed) workload and the served form's latency
        deadline = T_START + args.time_budget
        out["streamed"] = section("streamed", deadline, 240, lambda: streamed_summary(args, torch, bkd))
        out["served"] = section("served", deadline, 260, lambda: served_summary(args, torch, bkd))
    print(json.dumps(out), flush=True)


def section(name, deadline, need_s, fn):
    """Run one extra workload of the default line if the time budget allows; a failure of
    it is reported in its object and does not lose the headline."""
    left = deadline - time.perf_counter()
    if left < need_s:
        return {"skipped": f"{left:.0f} s of the bench's time budget left, {name} needs about {need_s} s"}
    print(f"bench: {name} workload ({left:.0f} s of the time budget left)", file=sys.stderr, flush=True)
    try:
        return fn()
    except Exception as e:  # noqa: BLE001 - reported in the line, the headline stays valid
        return {"error": f"{type(e).__name__}: {e}"}


def streamed_summary(args, torch, bkd):
    """The bigger-than-budget workload (n = 2^28, m = 2^24, h = 14, 2 GB leaf budget, 12 chunks)
    as one object: queries/s, its dense scan against the matrix peak, the host link, and the
    streamed/resident ratio, with a 2^16-query CPU sample."""
    r = run_plain(args, torch, bkd, "streamed", args.streamed_steps, 1, cpu_fixed=1 << 16)
    keep = ("metric", "value", "unit", "steps", "warmup", "ms_per_step", "higher_is_better", "dtype", "config",
            "roofline", "cpu_baseline", "stats_per_step")
    return {key: r[key] for key in keep if key in r}


def run_plain(args, torch, bkd, wname, steps, warmup, cpu_fixed=None):
    """One workload of the plain query path: tree built, queries resident in HBM, `steps`
    timed query calls after `warmup` untimed ones."""
    w = WORKLOADS[wname]
    n, m, d, k, h = w["n"], w["m"], w["d"], w["k"], w["h"]
    note(f"{wname}: generating inputs (n={n}, m={m}, d={d})")
    P, Q = make_inputs(w, args.seed)
    note(f"{wname}: building the tree")
    # lock-step rounds: every active query is fetched each iteration (results do not depend on B, M)
    budget = w.get("budget", 0)
    t_build = time.perf_counter()
    # the streamed tree is built on the device (the same canonical tree, a third of the host's time)
    tree = bkd.build(P, h, buffer_size=-1, fetch_size=-1, leaf_budget_bytes=budget,
                     flags=bkd.FLAG_TIMING | (bkd.FLAG_DEVICE_BUILD if budget else 0))
    t_build = time.perf_counter() - t_build
    build = None
    if not budget:
        # the same tree built on the device (both times include the leaf structure's upload)
        t_dev = time.perf_counter()
        dtree = bkd.build(P, h, buffer_size=-1, fetch_size=-1, flags=bkd.FLAG_DEVICE_BUILD)
        t_dev = time.perf_counter() - t_dev
        same = all(np.array_equal(a, b) for a, b in zip(bkd.tree_export(tree), bkd.tree_export(dtree)))
        dtree.free()
        build = {"host_s": round(t_build, 3), "device_s": round(t_dev, 3), "same_tree": same,
                 "what": "bkd_build wall time: canonical tree (host, or device with BKD_FLAG_DEVICE_BUILD) "
                         "plus the leaf structure's upload"}
    dQ = torch.from_numpy(Q).to("cuda")
    di = torch.empty((m, k), dtype=torch.int64, device="cuda")
    dd = torch.empty((m, k), dtype=torch.float32, device="cuda")
    stream = torch.cuda.Stream()
    note(f"{wname}: {warmup} warm-up and {steps} timed query calls")
    acc, wall, gpu_ms = timed_steps(bkd, torch, tree, dQ, k, di, dd, stream, steps, warmup)
    streaming = None
    if budget:
        info = bkd.tree_info(tree)
        tree.free()
        note(f"{wname}: the same tree resident")
        res = bkd.build(P, h, buffer_size=-1, fetch_size=-1, flags=bkd.FLAG_DEVICE_BUILD)
        racc, rwall, _ = timed_steps(bkd, torch, res, dQ, k, di, dd, stream, steps, warmup)
        res.free()
        streaming = {"leaf_budget_bytes": budget, "chunks": info.num_chunks,
                     "chunk_capacity_bytes": info.chunk_capacity_bytes, "leaf_structure_bytes": info.leaf_bytes,
                     "bytes_h2d_per_step": acc["bytes_h2d"] // steps,
                     "structure_copies_per_step": round(acc["bytes_h2d"] / steps / info.leaf_bytes, 3),
                     "chunk_copies_per_step": acc["chunk_copies"] / steps,
                     "h2d_rate_gbs_achieved": round(acc["bytes_h2d"] / wall / 1e9, 2),
                     "h2d_rate_gbs_pinned_copy": round(h2d_rate_gbs(torch), 2),
                     "resident_ms_per_step": round(rwall * 1e3 / steps, 3),
                     "t_streamed_over_t_resident": round(wall / rwall, 4),
                     "schedule": "lock-step rounds, chunk sweep (each resident chunk drained before the next)"}

    end_to_end = None
    if not budget:
        # host queries in, host results out: the blocking bkd_query, host-link transfers included
        # (reported beside the device-resident value, never as it)
        bkd.query(tree, Q, k)
        times = []
        for _ in range(3):
            t0 = time.perf_counter()
            bkd.query(tree, Q, k)
            times.append(time.perf_counter() - t0)
        t_e2e = sorted(times)[1]
        end_to_end = {"queries_per_s": round(m / t_e2e, 1), "ms_per_call": round(t_e2e * 1e3, 3),
                      "what": "bkd_query on host arrays (Q in, idx and dist out), median of 3 calls"}

    ms_per_step = wall * 1e3 / steps
    value = m * steps / wall
    # Dominant kernel: the dense leaf scan.  Algorithmic work per (query, leaf point) pair is
    # the float32 distance, 3d flops (d subtractions and d fused multiply-adds), counted for
    # every pair the kernel covers and set against the dense float16 matrix-core peak, the
    # engine that carries the kernel's contraction.  The kernel itself issues a different
    # amount: its matrix-core filter forms the inner product from d + 2 float16 products
    # padded to steps of sixteen (2 flops each, every pair), reported as mfma_issued_tflops
    # and matrix_core_frac; the exact float32 re-checks of passing pairs are not counted.
    ns = (d + 2 + 15) // 16
    mfma_flops_per_pair = 2 * 16 * ns
    flops = 3.0 * d * acc["dense_pairs"]
    dense_s = acc["dense_ms"] * 1e-3
    achieved = flops / dense_s / 1e12 if dense_s > 0 else 0.0
    issued = mfma_flops_per_pair * acc["dense_pairs"] / dense_s / 1e12 if dense_s > 0 else 0.0
    roofline = {
        "kernel": f"k_leaf_scan<{d},{k}> (dense leaf scan, scaled-float16 MFMA filter, exact float32 re-check)",
        "bound": "mfma",
        "achieved": round(achieved, 3),
        "peak": F16_MATRIX_PEAK_TFLOPS,
        "unit": "TFLOP/s",
        "frac": round(achieved / F16_MATRIX_PEAK_TFLOPS, 4),
        "traffic": dense_scan_traffic() if wname == "ondevice" else None,
        "flops_per_pair": 3 * d,
        "mfma_issued_tflops": round(issued, 3),
        "mfma_flops_per_pair": mfma_flops_per_pair,
        "matrix_core_frac": round(issued / F16_MATRIX_PEAK_TFLOPS, 4),
        "avg_launch_ms": round(acc["dense_ms"] / max(acc["dense_launches"], 1), 4),
        "launches_per_step": acc["dense_launches"] / steps,
        "pairs_per_launch": acc["dense_pairs"] // max(acc["dense_launches"], 1),
        # algorithmic bytes of the dense scan (every buffered leaf once per call, per visit the
        # query, its key list read and written, its buffer entry) and their rate: the HBM side
        "alg_bytes_per_launch": acc["alg_bytes_dense"] // max(acc["dense_launches"], 1),
        "alg_gbs": round(acc["alg_bytes_dense"] / dense_s / 1e9, 1) if dense_s > 0 else 0.0,
        "share_of_step": round(acc["dense_ms"] / max(gpu_ms, 1e-9), 4),
        # the library's sparse timer also covers the tail hand-over launch
        "sparse_and_tail": {"launches_per_step": acc["sparse_launches"] / steps,
                        "avg_launch_ms": round(acc["sparse_ms"] / max(acc["sparse_launches"], 1), 4),
                        "tflops": round(3.0 * d * acc["sparse_pairs"] / max(acc["sparse_ms"] * 1e-3, 1e-12) / 1e12, 3),
                        "share_of_step": round(acc["sparse_ms"] / max(gpu_ms, 1e-9), 4)},
    }
    out = {
        "metric": "kNN queries/s (d=10,k=10)",
        "value": round(value, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{wname}: n={n} m={m} d={d} k={k} height={h} "
                               f"{'16-component Gaussian mixture' if w['kind'] == 'mixture' else 'uniform [0,1]^d'}, "
                               f"seed {args.seed}, lock-step rounds"
                               + (f", leaf structure streamed through a {budget / 1e9:g} GB budget" if budget else ""),
                   "n": n, "m": m, "d": d, "k": k, "height": h, "rounds_per_step": acc["calls"] / steps,
                   "streaming": streaming,
                   "pairs_per_query": acc["pairs"] / (steps * m)},
        "roofline": roofline,
        "end_to_end": end_to_end,
        "build": build,
        "stats_per_step": {key: (round(acc[key] / steps, 3) if key.endswith("_ms") else acc[key] // steps)
                           for key in ("calls", "visits", "pairs", "alg_bytes", "find_ms", "group_ms", "dense_ms",
                                       "sparse_ms", "copy_ms", "wait_ms")},
    }
    if not budget:
        tree.free()
    del dQ, di, dd
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        note(f"{wname}: CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(P, Q, k, args.cpu_seconds, fixed=cpu_fixed)
    return out


if __name__ == "__main__":
    main()
