"""Benchmark: product-graph GTEPS, queries/s and p50/p99 latency of single-source
2-RPQs on one MI355X, batched versus plain.

Default workload (``--workload kg``): the knowledge-graph-shaped graph
(Chung-Lu, 20M vertices, 200M generated edges, power-law exponent 2.1, 1000
labels Zipf(1.2)), one seeded expression (4..12 Glushkov states) and 256
degree-weighted sources. One step = the 256 queries through the stacked path
(rpq_multi_source, one launch); ``value`` is product-graph GTEPS (product edges
out of every reached (state, vertex) pair, summed over the sources, divided by
the step's wall time, graph resident in HBM, results written to a device
buffer). The same 256 queries also run one at a time (plain) and through the
served path, for queries/s and latency beside the batched figure. The
roofline object reports the stacked kernel: algorithmic bytes per launch (the
batched model of rpq.h) over its mean launch duration, timed with HIP events
on the launch stream. A secondary object repeats the plain measurement on the
R-MAT scale-20 workload (100 template queries, one at a time).

Parity: the answers of the timed legs are compared with the oracle's, computed
on the host in a thread pool: a seeded subset of 32 of the 256 batched queries
and all 100 R-MAT queries. The JSON line carries the counts; any mismatch makes
the run exit with status 1 after printing it. cpu_baseline reports the oracle
runs of the batched subset (per-query latency, aggregate rate over the
threads used, host CPU model).

Other workloads: ``rmat`` (the plain path alone), ``grid`` (4096^2 grid, both
expressions, with 1 % shortcuts and without) and ``serve`` (a Poisson stream
of mixed queries on the kg graph, served against plain).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# The stacked pass is the persistent kernel k_stacked<G, QM> plus the phase
# kernels it hands its large push levels to (k_st_expand, k_st_compact,
# k_st_select, launched by the host loop in stacked_host.cpp); its duration
# and traffic are those of all of them together.
STACKED_PASS = "rpq::k_stacked<4, 8> pass (with k_st_expand, k_st_compact, k_st_select)"
KERNEL_SOURCES = {
    "rpq::k_persistent<1>": ("kernels.hip", "device_common.h", "rpq_internal.h"),
    STACKED_PASS: ("stacked.hip", "stacked.h", "stacked_host.cpp", "device_common.h", "rpq_internal.h"),
}
TRAFFIC_FILES = {
    "rpq::k_persistent<1>": "k_persistent_rmat20_traffic.md",
    STACKED_PASS: "k_stacked_kg20M_traffic.md",
}


def source_sha(kernel: str) -> str:
    """SHA-256 (first 16 hex digits) of the sources the kernel is built from."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2412_10287_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def committed_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when the kernel's sources changed since it was measured."""
    import re
    path = os.path.join(ROOT, "profiles", TRAFFIC_FILES.get(kernel, ""))
    try:
        text = open(path).read()
        sha = source_sha(kernel)
    except (OSError, KeyError):
        return None
    m = re.search(r"kernel=(.+?) traffic_bytes_per_launch=(\d+) sources_sha256_16=(\w+)", text)
    if not m or m.group(1) != kernel or m.group(3) != sha:
        return None
    return int(m.group(2))


def log_levels(tag, st, limit=64):
    """Per-level profile of one call on stderr: frontier vertices, new pairs,
    push edges and device microseconds per level."""
    n = len(st.level_us)
    log("%s: %d levels, %.3f ms on the device clock" % (tag, st.levels, st.level_us.sum() / 1e3))
    log("  level  frontier        pairs        edges         us  select_us")
    idx = list(range(n)) if n <= limit else list(range(limit // 2)) + list(range(n - limit // 2, n))
    for i in idx:
        log("  %5d %9d %12d %12d %10.1f %10.1f" % (i, st.level_frontier[i], st.level_counts[i], st.level_edges[i],
                                                  st.level_us[i], st.level_select_us[i]))


def percentile(xs, p):
    return float(np.percentile(np.asarray(xs), p)) if len(xs) else 0.0


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads() -> int:
    """Worker threads for the oracle: the CPUs this process may use, at most
    16 (one GPU's share of the host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


class OracleRuns:
    """Oracle (test infrastructure) answers for a list of (nfa, source)
    queries, computed by a pool of threads (each query one single-threaded
    call of the C oracle, which runs without the interpreter lock). The oracle
    graph is built in a background thread (one core) as soon as the object
    exists, so it overlaps with the GPU legs; the queries start on ``go()``,
    after the timed GPU legs, so that they do not compete with them for the
    host; ``results()`` starts them if needed and waits for everything. Each
    query's host footprint is about 12 |Q| |V| bytes, so the pool admits
    queries by a memory budget."""

    def __init__(self, graph, queries, threads: int, mem_budget: float = 96e9):
        self.queries = queries
        self.threads = threads
        self.mem_budget = mem_budget
        self._og = None
        self._out = [] if not queries else None
        self._err = None
        self.build_s = self.wall_s = 0.0
        self._go = threading.Event()
        self._th = threading.Thread(target=self._run, args=(graph,), daemon=True)
        if queries:
            self._th.start()

    def go(self):
        self._go.set()

    def _run(self, graph):
        try:
            import oracle
            t0 = time.perf_counter()
            self._og = oracle.Graph(graph)
            self.build_s = time.perf_counter() - t0
            log("  oracle: graph built in %.1f s" % self.build_s)
            self._go.wait()
            V = graph.num_vertices
            cond = threading.Condition()
            used = [0.0]

            def one(q):
                nfa, s = q
                need = min(12.0 * nfa.num_states * V, self.mem_budget)
                with cond:
                    cond.wait_for(lambda: used[0] + need <= self.mem_budget)
                    used[0] += need
                try:
                    t = time.perf_counter()
                    r = self._og.ssr(nfa, int(s))
                    dt = time.perf_counter() - t
                    log("  oracle: source %d done in %.2f s" % (int(s), dt))
                    return r.bitmap, int(r.product_edges), int(r.levels), dt
                finally:
                    with cond:
                        used[0] -= need
                        cond.notify_all()

            t0 = time.perf_counter()
            with cf.ThreadPoolExecutor(max_workers=self.threads) as ex:
                self._out = list(ex.map(one, self.queries))
            self.wall_s = time.perf_counter() - t0
        except BaseException as e:  # reported by results()
            self._err = e
        finally:
            if self._og is not None:
                self._og.close()
                self._og = None

    def results(self):
        self._go.set()
        if self.queries:
            self._th.join()
        if self._err is not None:
            raise self._err
        return self._out

    def baseline(self, what: str):
        out = self.results()
        if not out:
            return None
        lat = [o[3] for o in out]
        pe = sum(o[1] for o in out)
        return {"value": round(pe / self.wall_s / 1e9, 6), "unit": "GTEPS", "cores": self.threads,
                "kind": "oracle", "qps": round(len(out) / self.wall_s, 4),
                "latency_ms_p50": round(percentile(lat, 50) * 1e3, 2),
                "latency_ms_p99": round(percentile(lat, 99) * 1e3, 2),
                "cpu_model": cpu_model(),
                "sample": "%d queries (%s), one single-threaded oracle call each, %d threads over the sample; "
                          "%.1f s wall, oracle graph build %.1f s not timed" % (len(out), what, self.threads,
                                                                                self.wall_s, self.build_s)}


def parity_of(got_rows, want_bitmaps):
    bad = [i for i, (a, b) in enumerate(zip(got_rows, want_bitmaps)) if not np.array_equal(a, b)]
    return {"checked": len(want_bitmaps), "mismatches": len(bad), "first_mismatch": bad[0] if bad else None}


# ------------------------------------------------------------------ plain (C2)
def run_plain(args, w, steps, warmup, oracle_threads, with_cpu: bool):
    """The plain path, one query at a time, on workload w (every query's
    answer checked against the oracle). Returns the result dict (with
    parity) and the oracle runs."""
    from paper_2412_10287_amd import rpq
    runs = OracleRuns(w.graph, list(zip(w.nfas, w.sources)), oracle_threads)
    t0 = time.time()
    g = rpq.Graph(w.graph)
    nfas = [rpq.NFA(n) for n in w.nfas]
    log("%s: graph store loaded (%.1fs), %d MB on device" % (w.name, time.time() - t0, g.info("device_bytes") >> 20))
    words = g.words
    out = rpq.DeviceBuffer(8 * len(nfas) * words)
    base_ptr, row_bytes = out.ptr, words * 8
    mode = rpq.HOST_LOOP if args.host_loop else 0
    tuning = None
    if not args.no_tune:
        from paper_2412_10287_amd import autotune
        k = min(16, len(nfas))
        tuning = autotune.tune(g, rpq.TUNE_PLAIN, nfas[:k], [int(s) for s in w.sources[:k]], cache=args.tune_cache)
        log("autotune (plain, %d sample queries): %s" % (k, tuning))
    pe = np.zeros(len(nfas), np.int64)
    ab = np.zeros(len(nfas), np.int64)
    levels = np.zeros(len(nfas), np.int64)
    for i, (nh, s) in enumerate(zip(nfas, w.sources)):
        _, st = g.single_source(nh, int(s), flags=mode | rpq.COUNTERS, out_device_ptr=base_ptr + i * row_bytes)
        pe[i], ab[i], levels[i] = st.product_edges, st.alg_bytes, st.levels
    log("counters: product edges %d, algorithmic bytes %d, levels max %d" % (pe.sum(), ab.sum(), levels.max()))
    for i in (int(np.argmax(pe)), int(np.argsort(pe)[len(pe) // 2])):
        _, st = g.single_source(nfas[i], int(w.sources[i]), flags=mode, level_cap=1 << 14,
                                out_device_ptr=base_ptr + i * row_bytes)
        log_levels("query %d %r" % (i, w.queries[i]), st)

    def step(timing: bool, lat=None, kern=None):
        fl = mode | (rpq.KERNEL_TIMING if timing else 0)
        for i, (nh, s) in enumerate(zip(nfas, w.sources)):
            t = time.perf_counter()
            _, st = g.single_source(nh, int(s), flags=fl, out_device_ptr=base_ptr + i * row_bytes)
            if lat is not None:
                lat.append(time.perf_counter() - t)
            if kern is not None:
                kern.append((st.expand_ms, st.expand_launches))

    for _ in range(warmup):
        step(False)
    rpq.device_synchronize()
    lat, kern = [], []
    t0 = time.perf_counter()
    for k in range(steps):
        step(True, lat, kern)
        log("plain step %d done" % k)
    rpq.device_synchronize()
    dt = time.perf_counter() - t0
    answers = out.to_host().reshape(len(nfas), words)
    kern_ms = np.array([k[0] for k in kern])
    n_launch = int(sum(k[1] for k in kern))
    bytes_total = int(ab.sum()) * steps
    achieved = bytes_total / (kern_ms.sum() * 1e-3) / 1e9 if kern_ms.sum() > 0 else 0.0

    # served path on the same queries: all submitted at once, admitted as
    # slots free up, advanced one level per shared launch
    def served_step(lat=None):
        tickets = [g.submit(nh, int(s)) for nh, s in zip(nfas, w.sources)]
        for i, t in enumerate(tickets):
            _, st = g.poll(t, timeout_us=-1, out_device_ptr=base_ptr + i * row_bytes)
            if lat is not None:
                lat.append(st.latency_ms * 1e-3)
    for _ in range(warmup):
        served_step()
    slat = []
    t0 = time.perf_counter()
    for k in range(steps):
        served_step(slat)
    sdt = time.perf_counter() - t0
    served_answers = out.to_host().reshape(len(nfas), words)
    g.close()
    out.close()
    want = [r[0] for r in runs.results()]
    res = {
        "gteps": round(pe.sum() * steps / dt / 1e9, 4),
        "qps": round(len(nfas) * steps / dt, 2),
        "ms_per_step": round(dt / steps * 1e3, 3),
        "latency_ms_p50": round(percentile(lat, 50) * 1e3, 4),
        "latency_ms_p99": round(percentile(lat, 99) * 1e3, 4),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 5),
                     "traffic": committed_traffic("rpq::k_persistent<1>") if not args.host_loop else None,
                     "kernel": "rpq::k_persistent<1>", "launches": n_launch,
                     "mean_launch_us": round(kern_ms.sum() * 1e3 / max(n_launch, 1), 3),
                     "alg_bytes_per_launch": round(bytes_total / max(n_launch, 1), 1)},
        "served": {"qps": round(len(nfas) * steps / sdt, 2), "gteps": round(pe.sum() * steps / sdt / 1e9, 4),
                   "latency_ms_p50": round(percentile(slat, 50) * 1e3, 4),
                   "latency_ms_p99": round(percentile(slat, 99) * 1e3, 4),
                   "note": "all queries of a step submitted at once; latency = submit to answer"},
        "tuning": tuning,
        "parity": {"plain": parity_of(answers, want), "served": parity_of(served_answers, want)},
        "steps": steps, "warmup": warmup,
    }
    res["served_vs_plain_qps"] = round(res["served"]["qps"] / res["qps"], 3)
    if with_cpu:
        res["cpu_baseline"] = runs.baseline("every query of the step")
    return res


def parity_failed(p) -> bool:
    if isinstance(p, dict) and "mismatches" in p:
        return p["mismatches"] > 0
    if isinstance(p, dict):
        return any(parity_failed(v) for v in p.values())
    return False


def bench_rmat(args):
    from workloads import configs as C
    t0 = time.time()
    w = C.rmat_workload(scale=args.scale)
    log("workload %s: V=%d E=%d queries=%d (%.1fs)" % (w.name, w.graph.num_vertices, w.graph.num_edges,
                                                      len(w.queries), time.time() - t0))
    r = run_plain(args, w, args.steps, args.warmup, host_threads(), not args.no_cpu)
    out = {
        "metric": "product-graph GTEPS (plain one-query-at-a-time path)",
        "value": r["gteps"], "unit": "GTEPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u8", "data": "synthetic",
        "config": {"workload": w.name + " plain, %d queries per step" % len(w.queries), "queries": len(w.queries),
                   "vertices": w.graph.num_vertices, "edges": w.graph.num_edges, "labels": w.graph.num_labels,
                   "levels": "host" if args.host_loop else "persistent"},
    }
    out.update({k: v for k, v in r.items() if k not in ("gteps", "ms_per_step", "steps", "warmup")})
    print(json.dumps(out), flush=True)
    return 1 if parity_failed(out["parity"]) else 0


# ------------------------------------------------------------- batched (C3)
def bench_kg(args):
    from workloads import configs as C
    t0 = time.time()
    n = 20_000_000 if args.scale >= 20 else 1 << args.scale
    w = C.kg_workload(n=n, m=10 * n)
    log("workload %s: V=%d E=%d, %d sources, expression %r (%d states) (%.1fs)" % (
        w.name, w.graph.num_vertices, w.graph.num_edges, len(w.sources), w.queries[0], w.nfas[0].num_states,
        time.time() - t0))
    nfa = w.nfas[0]
    srcs = [int(s) for s in w.sources]
    B = len(srcs)
    # a seeded subset of the batch for the oracle, started now (its graph
    # build overlaps with the GPU legs)
    rs = np.random.default_rng(C.seed(3, 5))
    sample = np.sort(rs.choice(B, size=min(args.parity_sample, B), replace=False))
    runs = OracleRuns(w.graph, [(nfa, srcs[i]) for i in sample], host_threads())

    from paper_2412_10287_amd import rpq
    t0 = time.time()
    g = rpq.Graph(w.graph)
    log("graph store loaded (%.1fs), %d MB on device" % (time.time() - t0, g.info("device_bytes") >> 20))
    edges_distinct = g.info("num_edges")
    nh = rpq.NFA(nfa)
    g.set_option("max_batch", B)
    tuning = None
    if args.stacked_alpha is not None:
        g.set_option("stacked_alpha", args.stacked_alpha)
    elif not args.no_tune:
        from paper_2412_10287_amd import autotune
        tuning = autotune.tune(g, rpq.TUNE_STACKED, [nh], srcs, cache=args.tune_cache)
        log("autotune (stacked, one batch): %s" % tuning)
    words = g.words
    out = rpq.DeviceBuffer(8 * B * words)
    # the batch's algorithmic work (device counters; exact, pinned to the
    # oracle in the tests)
    _, st = g.multi_source(nh, srcs, flags=rpq.COUNTERS, out_device_ptr=out.ptr, level_cap=1 << 14)
    pe_total, alg_bytes, updates, levels = st.product_edges, st.alg_bytes, st.updates, st.levels
    log("batch: product edges %d, algorithmic bytes %d, word updates %d, levels %d" % (
        pe_total, alg_bytes, updates, levels))
    log_levels("stacked", st)
    if args.levels_only:
        return 0

    kern = []

    def stacked_step():
        _, s2 = g.multi_source(nh, srcs, out_device_ptr=out.ptr)
        kern.append(s2.expand_ms)

    for _ in range(args.warmup):
        stacked_step()
    rpq.device_synchronize()
    kern.clear()
    step_s = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        t = time.perf_counter()
        stacked_step()
        step_s.append(time.perf_counter() - t)
        log("stacked step %d done" % k)
    rpq.device_synchronize()
    dt = time.perf_counter() - t0
    stacked_rows = out.to_host().reshape(B, words)
    k_ms = float(np.mean(kern))
    achieved = alg_bytes / (k_ms * 1e-3) / 1e9
    kname = "rpq::k_stacked<%d, %d> pass (with k_st_expand, k_st_compact, k_st_select)" % (
        (B + 63) // 64 if B <= 64 else 1 << ((B + 63) // 64 - 1).bit_length(), 8 if nfa.num_states <= 8 else 32)

    # the same queries one at a time (plain) and through the served path
    cmp_steps = max(1, min(args.steps, args.compare_steps))
    if args.skip_compare:
        g.close()
        out.close()
        want = [r[0] for r in runs.results()]
        res = {"metric": "product-graph GTEPS; queries/s + p50/p99 latency, batched vs plain, 1 GPU",
               "value": round(pe_total * args.steps / dt / 1e9, 3), "unit": "GTEPS", "n_gpus": 1,
               "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 3),
               "note": "stacked leg only (profiling run)", "mean_launch_us": round(k_ms * 1e3, 1),
               "alg_bytes_per_launch": int(alg_bytes),
               "parity": {"stacked": parity_of(stacked_rows[sample], want)}}
        print(json.dumps(res), flush=True)
        return 1 if parity_failed(res["parity"]) else 0
    plain_lat = []

    def plain_step(lat=None):
        for i, s in enumerate(srcs):
            t = time.perf_counter()
            g.single_source(nh, s, out_device_ptr=out.ptr + 8 * i * words)
            if lat is not None:
                lat.append(time.perf_counter() - t)

    plain_step()
    rpq.device_synchronize()
    t0 = time.perf_counter()
    for k in range(cmp_steps):
        plain_step(plain_lat)
        log("plain step %d done" % k)
    rpq.device_synchronize()
    pdt = time.perf_counter() - t0
    plain_rows = out.to_host().reshape(B, words)
    slat = []

    def served_step(lat=None):
        tickets = [g.submit(nh, s) for s in srcs]
        for i, t in enumerate(tickets):
            _, s2 = g.poll(t, timeout_us=-1, out_device_ptr=out.ptr + 8 * i * words)
            if lat is not None:
                lat.append(s2.latency_ms * 1e-3)

    served_step()
    t0 = time.perf_counter()
    for k in range(cmp_steps):
        served_step(slat)
        log("served step %d done" % k)
    sdt = time.perf_counter() - t0
    served_rows = out.to_host().reshape(B, words)
    g.close()
    out.close()

    log("waiting for the oracle (%d queries on %d threads)" % (len(sample), runs.threads))
    want = [r[0] for r in runs.results()]
    parity = {"stacked": parity_of(stacked_rows[sample], want), "plain": parity_of(plain_rows[sample], want),
              "served": parity_of(served_rows[sample], want),
              "plain_equals_stacked_all": bool(np.array_equal(plain_rows, stacked_rows)),
              "served_equals_stacked_all": bool(np.array_equal(served_rows, stacked_rows)),
              "sample": "%d of the %d sources (seeded), bitmaps against the oracle" % (len(sample), B)}
    pe_sample = sum(r[1] for r in runs.results())
    res = {
        "metric": "product-graph GTEPS; queries/s + p50/p99 latency, batched vs plain, 1 GPU",
        "value": round(pe_total * args.steps / dt / 1e9, 3),
        "unit": "GTEPS",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "%s batched: %d sources per launch under one expression" % (w.name, B),
                   "expression": w.queries[0], "states": int(nfa.num_states), "vertices": w.graph.num_vertices,
                   "edges_generated": w.graph.num_edges, "edges_distinct": edges_distinct,
                   "labels": w.graph.num_labels, "levels": int(levels)},
        "qps": round(B * args.steps / dt, 2),
        "latency_ms_p50": round(percentile(step_s, 50) * 1e3, 3),
        "latency_ms_p99": round(percentile(step_s, 99) * 1e3, 3),
        "latency_note": "batched: every query of a launch completes with the launch",
        "plain": {"qps": round(B * cmp_steps / pdt, 2), "gteps": round(pe_total * cmp_steps / pdt / 1e9, 3),
                  "latency_ms_p50": round(percentile(plain_lat, 50) * 1e3, 3),
                  "latency_ms_p99": round(percentile(plain_lat, 99) * 1e3, 3), "steps": cmp_steps},
        "served": {"qps": round(B * cmp_steps / sdt, 2), "gteps": round(pe_total * cmp_steps / sdt / 1e9, 3),
                   "latency_ms_p50": round(percentile(slat, 50) * 1e3, 3),
                   "latency_ms_p99": round(percentile(slat, 99) * 1e3, 3), "steps": cmp_steps,
                   "note": "all queries submitted at once; latency = submit to answer"},
        "batched_vs_plain_qps": round((B * args.steps / dt) / (B * cmp_steps / pdt), 2),
        "tuning": tuning,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": committed_traffic(kname),
                     "kernel": kname, "launches": len(kern), "mean_launch_us": round(k_ms * 1e3, 1),
                     "alg_bytes_per_launch": int(alg_bytes), "product_edges_per_launch": int(pe_total),
                     "word_updates_per_launch": int(updates)},
        "parity": parity,
    }
    if pe_sample:
        res["parity"]["oracle_product_edges_sample"] = int(pe_sample)
    if not args.no_cpu:
        res["cpu_baseline"] = runs.baseline("the parity subset of the batch")
    if not args.no_secondary:
        w2 = C.rmat_workload(scale=20)
        log("secondary: %s plain" % w2.name)
        r2 = run_plain(args, w2, args.steps, args.warmup, host_threads(), False)
        res["rmat_plain"] = {"workload": w2.name + " plain, %d queries per step" % len(w2.queries)}
        res["rmat_plain"].update(r2)
        res["parity"]["rmat"] = r2["parity"]
    print(json.dumps(res), flush=True)
    return 1 if parity_failed(res["parity"]) else 0


# ------------------------------------------------------------------ grid (C5)
def bench_grid(args):
    """Both grid expressions on the 4096^2 grid with 1 % shortcuts and
    without, 64 sources per launch through the stacked path: levels, us per
    level, batch time; plain on a few of the sources for comparison. Parity:
    closed forms for every source on the grid without shortcuts, the oracle on
    a seeded subset with shortcuts."""
    from workloads import configs as C
    from paper_2412_10287_amd import rpq
    side = 4096 if args.scale >= 20 else 1 << (args.scale // 2)
    variants = {}
    parity = {}
    pending = []
    head = None
    for frac in (0.01, 0.0):
        t0 = time.time()
        w = C.grid_workload(side=side, shortcut_frac=frac)
        log("workload %s: V=%d E=%d (%.1fs)" % (w.name, w.graph.num_vertices, w.graph.num_edges, time.time() - t0))
        srcs = [int(s) for s in w.sources]
        B = len(srcs)
        sample = list(range(0, B, max(1, B // args.grid_oracle)))[:args.grid_oracle] if frac > 0 else []
        runs = OracleRuns(w.graph, [(nfa, srcs[i]) for nfa in w.nfas for i in sample], host_threads()) \
            if sample else None
        g = rpq.Graph(w.graph)
        g.set_option("max_batch", B)
        words = g.words
        out = rpq.DeviceBuffer(8 * B * words)
        for qi, (text, nfa) in enumerate(zip(w.queries, w.nfas)):
            nh = rpq.NFA(nfa)
            _, st = g.multi_source(nh, srcs, flags=rpq.COUNTERS, out_device_ptr=out.ptr, level_cap=1 << 14)
            pe, lv = st.product_edges, st.levels
            for _ in range(args.warmup):
                g.multi_source(nh, srcs, out_device_ptr=out.ptr)
            rpq.device_synchronize()
            t0 = time.perf_counter()
            kms = []
            for _ in range(args.steps):
                _, s2 = g.multi_source(nh, srcs, out_device_ptr=out.ptr)
                kms.append(s2.expand_ms)
            rpq.device_synchronize()
            dt = (time.perf_counter() - t0) / args.steps
            rows = out.to_host().reshape(B, words)
            # plain on the first 4 sources (each pays every level alone), and
            # the same queries with levels driven from the host, one launch
            # per phase or as replays of a captured graph of 16 levels
            pt = []
            for s in srcs[:4]:
                t = time.perf_counter()
                g.single_source(nh, s, out_device_ptr=out.ptr)
                pt.append(time.perf_counter() - t)
            modes = {}
            for mname, fl in (("persistent", 0), ("graph_levels", rpq.GRAPH_LEVELS), ("host_loop", rpq.HOST_LOOP)):
                g.single_source(nh, srcs[1], flags=fl, out_device_ptr=out.ptr)  # warm-up (captures the graph)
                t = time.perf_counter()
                _, sm = g.single_source(nh, srcs[1], flags=fl, out_device_ptr=out.ptr)
                dtm = time.perf_counter() - t
                modes[mname] = {"ms": round(dtm * 1e3, 3), "levels": int(sm.levels),
                                "us_per_level": round(dtm * 1e6 / max(sm.levels, 1), 2)}
            key = "%s %s" % ("shortcuts-1%" if frac else "no-shortcuts", text)
            variants[key] = {"levels": int(lv), "batch_ms": round(dt * 1e3, 3),
                             "kernel_ms": round(float(np.mean(kms)), 3),
                             "us_per_level": round(float(np.mean(kms)) * 1e3 / max(lv, 1), 2),
                             "levels_per_s": round(lv / (float(np.mean(kms)) * 1e-3), 1),
                             "qps": round(B / dt, 2), "gteps": round(pe / dt / 1e9, 4),
                             "plain_qps": round(len(pt) / sum(pt), 2), "plain_modes": modes,
                             "alg_bytes_per_launch": int(st.alg_bytes)}
            if frac == 0.0:
                bad = 0
                for i, s in enumerate(srcs):
                    x0, y0 = s % side, s // side
                    if qi == 0:
                        m = np.zeros((side, side), bool)
                        m[y0:, x0:] = True
                    else:
                        m = np.zeros((side, side), bool)
                        if y0 > 0:
                            m[y0 - 1, x0:] = True
                    bits = np.packbits(m.ravel(), bitorder="little")
                    want = np.zeros(words * 8, np.uint8)
                    want[:bits.size] = bits
                    bad += not np.array_equal(rows[i].view(np.uint8), want)
                parity[key] = {"checked": B, "mismatches": int(bad), "against": "closed form"}
            else:
                pending.append((key, qi, rows[sample].copy()))
            if head is None:
                head = (key, variants[key], st, w, B)
            log("%s: %s" % (key, variants[key]))
        g.close()
        out.close()
        for key, qi, got in pending:
            want = [r[0] for r in runs.results()[qi * len(sample):(qi + 1) * len(sample)]]
            parity[key] = dict(parity_of(got, want), against="oracle")
        pending.clear()
    key, v, st, w, B = head
    res = {
        "metric": "product-graph GTEPS; queries/s + p50/p99 latency, batched vs plain, 1 GPU",
        "value": v["gteps"], "unit": "GTEPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": v["batch_ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64", "data": "synthetic",
        "config": {"workload": "grid %dx%d, %d sources per launch: %s" % (side, side, B, key)},
        "variants": variants,
        "parity": parity,
    }
    print(json.dumps(res), flush=True)
    return 1 if parity_failed(parity) else 0


# ----------------------------------------------------------------- serve (C4)
def bench_serve(args):
    """Serving loop on the knowledge graph: a seeded stream of mixed queries
    (template queries and random expressions of 1..31 label occurrences) with
    Poisson arrivals. The served path (rpq_submit / rpq_poll) is driven open
    loop: a submitter thread submits each query at its arrival time and the
    latency of a query is completion minus arrival. The arrival rate is 0.8 of
    the served path's saturated rate (all queries submitted at once). The plain
    path serves the same stream one query at a time in arrival order (a FIFO
    single server), so its latency includes the wait behind earlier queries.
    Parity: a seeded subset of the stream against the oracle."""
    import queue
    from workloads import configs as C
    from workloads import regex as R
    from paper_2412_10287_amd import rpq
    n = 20_000_000 if args.scale >= 20 else 1 << args.scale
    t0 = time.time()
    graph = C.kg_graph(n=n, m=10 * n)
    texts, srcs, _ = C.serve_queries(graph, args.serve_queries, 1.0)
    nfas = [R.compile_regex(q, graph.num_labels) for q in texts]
    states = np.array([a.num_states for a in nfas])
    log("serve workload: V=%d E=%d, %d queries, states %d..%d (mean %.1f) (%.1fs)" % (
        graph.num_vertices, graph.num_edges, len(nfas), states.min(), states.max(), states.mean(), time.time() - t0))
    N = len(nfas)
    rs = np.random.default_rng(C.seed(4, 5))
    sample = np.sort(rs.choice(N, size=min(args.serve_parity, N), replace=False))
    runs = OracleRuns(graph, [(nfas[i], int(srcs[i])) for i in sample], host_threads())
    g = rpq.Graph(graph)
    if args.max_slots:
        g.set_option("max_slots", args.max_slots)
    if args.serve_lanes is not None:
        g.set_option("serve_lanes", args.serve_lanes)
    if args.large_pairs is not None:
        g.set_option("large_query_pairs", args.large_pairs)
    handles = [rpq.NFA(a) for a in nfas]
    words = g.words
    out = rpq.DeviceBuffer(8 * words)
    keep = rpq.DeviceBuffer(8 * max(1, len(sample)) * words)
    slot_of = {int(i): k for k, i in enumerate(sample)}
    pe = np.zeros(N, np.int64)
    for i, (h, s) in enumerate(zip(handles, srcs)):
        _, st = g.single_source(h, int(s), flags=rpq.COUNTERS, out_device_ptr=out.ptr)
        pe[i] = st.product_edges
    log("product edges: total %d, per query median %d max %d" % (pe.sum(), np.median(pe), pe.max()))

    def dst(i):
        k = slot_of.get(i)
        return out.ptr if k is None else keep.ptr + 8 * k * words

    alone = [0]

    def served_saturated():
        t = time.perf_counter()
        tickets = [g.submit(h, int(s)) for h, s in zip(handles, srcs)]
        alone[0] = 0
        for i, tk in enumerate(tickets):
            _, st = g.poll(tk, timeout_us=-1, out_device_ptr=dst(i))
            alone[0] += st.batch == 1
        return N / (time.perf_counter() - t)

    served_saturated()  # warm-up (engine allocation)
    qps_sat = served_saturated()
    sat_rows = keep.to_host().reshape(-1, words)[:len(sample)].copy()
    rate = 0.8 * qps_sat
    arr = np.cumsum(np.random.default_rng(C.seed(4, 4)).exponential(1.0 / rate, size=N))
    log("served saturated %.1f q/s (%d queries through the single-query kernel) -> Poisson arrivals at %.1f q/s"
        % (qps_sat, alone[0], rate))
    tq = queue.Queue()
    start = time.perf_counter() + 0.05

    def submitter():
        for i in range(N):
            d = start + arr[i] - time.perf_counter()
            if d > 0:
                time.sleep(d)
            lag = time.perf_counter() - (start + arr[i])
            tq.put((i, g.submit(handles[i], int(srcs[i])), lag))

    th = threading.Thread(target=submitter)
    th.start()
    lat = np.zeros(N)
    for _ in range(N):
        i, tk, lag = tq.get()
        _, st = g.poll(tk, timeout_us=-1, out_device_ptr=dst(i))
        lat[i] = lag + st.latency_ms * 1e-3
    th.join()
    served_span = max(arr[i] + lat[i] for i in range(N)) - arr[0]
    open_rows = keep.to_host().reshape(-1, words)[:len(sample)].copy()
    log("served open loop done")
    plat = np.zeros(N)
    start = time.perf_counter()
    for i in range(N):
        d = start + arr[i] - time.perf_counter()
        if d > 0:
            time.sleep(d)
        g.single_source(handles[i], int(srcs[i]), out_device_ptr=dst(i))
        plat[i] = time.perf_counter() - start - arr[i]
    plain_span = max(arr[i] + plat[i] for i in range(N)) - arr[0]
    plain_rows = keep.to_host().reshape(-1, words)[:len(sample)].copy()
    t = time.perf_counter()
    for h, s in zip(handles, srcs):
        g.single_source(h, int(s), out_device_ptr=out.ptr)
    plain_sat = N / (time.perf_counter() - t)
    # the same stream through the plain path with the rare-end plan allowed
    # (queries with at most 1024 candidate endpoints run backwards from them)
    g.set_option("rare_end_max", 1024)
    plans = 0
    t = time.perf_counter()
    for i, (h, s) in enumerate(zip(handles, srcs)):
        _, st = g.single_source(h, int(s), out_device_ptr=dst(i))
        plans += st.plan
    rare_sat = N / (time.perf_counter() - t)
    rare_rows = keep.to_host().reshape(-1, words)[:len(sample)].copy()
    g.set_option("rare_end_max", 0)
    slots = g.info("serve_slots")
    lanes = g.info("serve_lanes")
    g.close()
    out.close()
    keep.close()
    want = [r[0] for r in runs.results()]
    parity = {"served_saturated": parity_of(sat_rows, want), "served_open_loop": parity_of(open_rows, want),
              "plain": parity_of(plain_rows, want), "plain_rare_end": parity_of(rare_rows, want),
              "sample": "%d of the %d queries (seeded), bitmaps against the oracle" % (len(sample), N)}
    res = {
        "metric": "queries/s and p50/p99 latency, served path under Poisson arrivals",
        "value": round(N / served_span, 2), "unit": "queries/s",
        "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": round(served_span * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "serve on kg-%d-%d-L1000: %d mixed queries, Poisson arrivals at %.1f q/s"
                   % (graph.num_vertices, graph.num_edges, N, rate),
                   "states_min": int(states.min()), "states_max": int(states.max()), "slots": slots,
                   "lanes": lanes},
        "served": {"qps": round(N / served_span, 2), "gteps": round(pe.sum() / served_span / 1e9, 4),
                   "latency_ms_p50": round(percentile(lat, 50) * 1e3, 3),
                   "latency_ms_p99": round(percentile(lat, 99) * 1e3, 3),
                   "saturated_qps": round(qps_sat, 2), "single_query_kernel": int(alone[0])},
        "plain": {"qps": round(N / plain_span, 2), "gteps": round(pe.sum() / plain_span / 1e9, 4),
                  "latency_ms_p50": round(percentile(plat, 50) * 1e3, 3),
                  "latency_ms_p99": round(percentile(plat, 99) * 1e3, 3),
                  "saturated_qps": round(plain_sat, 2)},
        "plain_rare_end": {"saturated_qps": round(rare_sat, 2), "queries_on_rare_end_plan": int(plans),
                           "note": "plain path with rare_end_max 1024: queries with at most 1024 candidate "
                                   "endpoints run as one reversed stacked traversal from them"},
        "arrival_qps": round(rate, 2),
        "parity": parity,
    }
    if not args.no_cpu:
        res["cpu_baseline"] = runs.baseline("the parity subset of the stream")
    print(json.dumps(res), flush=True)
    return 1 if parity_failed(parity) else 0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="kg", choices=("kg", "rmat", "grid", "serve"))
    ap.add_argument("--scale", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="leave out cpu_baseline (parity still runs)")
    ap.add_argument("--no-secondary", action="store_true", help="kg: leave out the R-MAT plain secondary")
    ap.add_argument("--parity-sample", type=int, default=32, help="kg: batch queries checked against the oracle")
    ap.add_argument("--compare-steps", type=int, default=3, help="kg: steps of the plain and served legs")
    ap.add_argument("--skip-compare", action="store_true", help="kg: stacked leg only (for profiler runs)")
    ap.add_argument("--grid-oracle", type=int, default=8, help="grid: sources checked against the oracle")
    ap.add_argument("--host-loop", action="store_true", help="plain path: drive levels from the host")
    ap.add_argument("--stacked-alpha", type=int, default=None, help="push->pull threshold of the stacked path")
    ap.add_argument("--levels-only", action="store_true", help="kg: per-level profile only")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (library defaults)")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON file for the autotuner's choices (reused when present, e.g. so that "
                         "profiler passes run the settings of an earlier timed run)")
    ap.add_argument("--serve-queries", type=int, default=2000, help="serve: queries in the stream")
    ap.add_argument("--serve-lanes", type=int, default=None, help="serve: single-query executors of the served path")
    ap.add_argument("--large-pairs", type=int, default=None, help="serve: large_query_pairs of the served path")
    ap.add_argument("--serve-parity", type=int, default=128, help="serve: queries checked against the oracle")
    ap.add_argument("--max-slots", type=int, default=0, help="served path: concurrent queries (0 = library default)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run device-to-device copies of MIB MiB (for traffic-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this engine runs on one GPU; --gpus %d is not supported (use --gpus 1)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        from paper_2412_10287_amd import rpq
        n = args.calibrate_copy << 20
        a, b = rpq.DeviceBuffer(n), rpq.DeviceBuffer(n)
        for _ in range(3):
            b.copy_from(a)
        rpq.device_synchronize()
        a.close()
        b.close()
        print(json.dumps({"calibrate_copy_bytes": n, "copies": 3}))
        return 0
    fn = {"kg": bench_kg, "rmat": bench_rmat, "grid": bench_grid, "serve": bench_serve}[args.workload]
    return fn(args)


if __name__ == "__main__":
    sys.exit(main())
