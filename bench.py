"""Benchmark: single-source direction-optimized BFS on one MI355X.

Workload (default): Kronecker graph, scale 30 (2^30 vertices), edgefactor 16,
initiator A/B/C/D = 0.57/0.19/0.19/0.05, seed 2, seeded vertex relabelling,
self-loops and duplicates removed, symmetric CSR (int64 offsets, int32 IDs),
built on the GPU; 16 roots of degree >= 1 drawn with seed 2 + 10^6.

A step is one traversal from each of the 16 roots (init + all levels, the
graph and output buffers already resident).  The metric is traversed
undirected edges per second, harmonic mean over every (root, step) run,
where a run's traversed edges are the undirected edges of the root's
component (half the summed degree of the reached vertices).

Other modes (--mode), each printing one JSON line of its own:
  batch  Kronecker scale 24: 64 roots in one batched pass against the same
         64 roots run one at a time.
  pack   2,000 Kronecker graphs of scales drawn uniformly from 10..18, one
         root each, packed and traversed in one pass, against 2,000 separate
         single-source runs.
  chunglu  Chung-Lu power-law graph standing in for a real-world graph:
         100M core vertices, exponent 2.2, mean degree 20, max 10^6, plus 50
         path tails of 200 vertices (hundreds of levels, several direction
         switches), built on the device; 16 roots, harmonic-mean GTEPS.
  hybrid Kronecker scale 26 split between host and GPU as for a graph
         beyond device memory (Section 3.2): the rows of the highest-degree
         12% of the non-isolated vertices stay in host memory and are
         traversed by host threads, the rest on the device; 16 roots,
         harmonic-mean GTEPS of the whole hybrid run (host work, exchanges
         and the final gather included), with the resident run on the same
         roots as context.
  energy MTEPS/W: the default workload's traversals back to back for a fixed
         window while the GPU's socket power is sampled (Section 4.3's
         energy case, for the GPU alone).
  serve  8 resident Kronecker graphs (scales 18, 20, 22, 24, 24, 25, 26, 26),
         Poisson arrivals of (graph, root) queries at several rates, served
         with continuous batching and, as the baseline, one plain run at a
         time in arrival order; p50/p99 latency and completed queries/s.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GTEPS (harmonic mean over roots) at scale 30; served queries/s + p99 vs plain"
HBM_PEAK_GBS = 8000.0
# the kernel the line's roofline is reported for: the bottom-up level kernel,
# the largest share of a scale-30 traversal's time
DOMINANT = "k_level_bu"
TRAFFIC_KERNELS = ("k_level_bu", "k_level_td", "k_aux", "k_finalize")
DIRECT_CAP = 1 << 16  # a top-down level whose frontier has at most this many edges hands its queue on directly


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def bottom_up_bytes(rec: dict, words_active: int) -> float:
    """Algorithmic bytes of one bottom-up level: visited word read and
    next-frontier word write (16) per active 64-vertex word; one offset (8)
    per scanned vertex; one neighbour ID (4) and one frontier-bit probe (1/8)
    per examined edge up to the first hit; depth and parent (8) per new
    vertex."""
    return 16.0 * words_active + 8.0 * rec["scanned"] + (4.0 + 0.125) * rec["checked"] + 8.0 * rec["found"]


def top_down_bytes(rec: dict) -> float:
    """Algorithmic bytes of one top-down level: queue entry (4) and two
    offsets (16) per frontier vertex; one neighbour ID (4) and one
    visited-bit probe (1/8) per examined edge; per new vertex its two offsets
    (16), depth, parent and queue entry (12) and its visited and frontier bits
    (2/8)."""
    return 20.0 * rec["n_f"] + (4.0 + 0.125) * rec["checked"] + (28.0 + 0.25) * rec["found"]


def to_queue_bytes(log_recs: list, i: int, words_active: int) -> float:
    """Bytes of the frontier conversion before top-down level i (bitmap read,
    the other bitmap cleared: 16 per active word; 4 per queued vertex), which
    runs unless level i-1 was top-down and small enough to hand its queue on
    directly."""
    rec = log_recs[i]
    if rec["dir"] != 0 or i == 0:
        return 0.0
    prev = log_recs[i - 1]
    if prev["dir"] == 0 and prev["m_f"] <= DIRECT_CAP:
        return 0.0
    return 16.0 * words_active + 4.0 * rec["n_f"]


def kernel_source_digest() -> str:
    """Identity of the level kernel's source: measured traffic is only
    reported for the kernel it was measured on.  Comments and blank space
    are left out, so that editing a comment does not void a measurement."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in ("bfs_kernels.hip", "device_common.h", "dobfs_internal.h"):
        with open(os.path.join(ROOT, "paper_1503_04359_amd", "csrc", f), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)  # block comments
        text = re.sub(r"//[^\n]*", " ", text)                # line comments
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def harmonic_mean(xs):
    return len(xs) / sum(1.0 / x for x in xs)


def host_spec() -> dict:
    """CPU model, logical CPUs and memory of the host the baseline ran on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    mem_gib = None
    try:
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal:"):
                    mem_gib = round(int(line.split()[1]) / (1 << 20), 1)
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "cpus_allowed": len(os.sched_getaffinity(0)),
            "mem_gib": mem_gib}


def cpu_baseline(scale: int, seed: int, nroots: int, budget_s: float) -> dict:
    """The oracle (serial queue BFS, one thread pinned to one core) on a
    bounded sample of the workload: a Kronecker graph of the same family
    and seed at a smaller scale (the scale-30 graph needs ~145 GB of host
    memory and minutes per root), built on the device (bit-identical to the
    host builder) and copied to the host; roots drawn as for the GPU run,
    taken in order until `budget_s` seconds of oracle time are spent."""
    import graphgen as gg
    import oracle
    t0 = time.time()
    dg = gg.kronecker_device(scale, seed=seed)
    roots = gg.sample_roots_device(dg, nroots, seed=seed + 1_000_000)
    g = dg.to_host()
    dg.free()
    log(f"[cpu] kronecker scale {scale} built on the device and copied to the host in {time.time() - t0:.1f}s "
        f"(n={g.n}, m={g.m})")
    spec = host_spec()
    allowed = sorted(os.sched_getaffinity(0))
    core = allowed[0]
    os.sched_setaffinity(0, {core})
    teps, used = [], 0.0
    try:
        for r in roots:
            t = time.perf_counter()
            d, _ = oracle.bfs(g.offsets, g.indices, int(r))
            dt = time.perf_counter() - t
            used += dt
            teps.append(oracle.traversed_edges(g.offsets, d) / dt)
            if used >= budget_s:
                break
    finally:
        os.sched_setaffinity(0, set(allowed))
    val = harmonic_mean(teps) / 1e9
    log(f"[cpu] oracle, {len(teps)} roots on core {core} in {used:.1f}s: {val:.4f} GTEPS "
        f"({spec['cpu_model']}, {spec['nproc']} CPUs, {spec['mem_gib']} GiB)")
    return {"value": round(val, 5), "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "sample": f"serial queue BFS, one thread pinned to CPU {core}, over the Kronecker graph of scale {scale} "
                      f"(edgefactor 16, same initiator and seed {seed}; n={g.n}, m={g.m}) standing in for scale 30, "
                      f"whose host copy would need ~145 GB and minutes per root; the first {len(teps)} of "
                      f"{nroots} roots drawn as for the GPU run (until {budget_s:.0f}s of oracle time), "
                      f"harmonic mean; {used:.1f}s of CPU time",
            "scale": scale, "roots": len(teps), "seconds": round(used, 2), "host": spec}


def _timed(stream, fn):
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    out = fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1), out


def bench_batch(args) -> dict:
    """64 roots in one batched pass vs the same roots one at a time."""
    import torch
    import graphgen as gg
    import paper_1503_04359_amd as dobfs
    scale, seed = args.scale if args.scale != 30 else 24, args.seed if args.seed != 2 else 4
    stream = torch.cuda.current_stream()
    t0 = time.time()
    g = gg.kronecker_device(scale, args.edgefactor, seed=seed)
    roots = gg.sample_roots_device(g, 64, seed=seed + 1_000_000)
    reindex = args.reindex == "on"
    dg = dobfs.Graph.from_device_pointers(g.offsets_ptr, g.indices_ptr, g.n, g.m, borrow=not reindex,
                                          reindex=reindex)
    torch.cuda.synchronize()
    log(f"[batch] kronecker scale {scale} resident in {time.time() - t0:.1f}s (n={g.n}, m={g.m})")
    n = g.n
    params = dobfs.make_params(args.policy)
    out = torch.empty((64, n), dtype=torch.int32, device="cuda")
    depth = torch.empty(n, dtype=torch.int32, device="cuda")
    mc = []
    for r in roots:  # traversed edges per root, and warm-up
        _, _, st = dg.run(int(r), depth=depth, want_parent=False, params=params, stats=True, stream=stream)
        mc.append(st.m_c)
    dg.batch(roots, depth=out, params=params, stream=stream)
    torch.cuda.synchronize()
    eager = dobfs.make_params(args.policy, flags=dobfs.RUN_EAGER)
    dg.batch(roots, depth=out, params=eager, stream=stream)
    torch.cuda.synchronize()
    bt, st_, et = [], [], []
    for _ in range(args.steps):
        ms, _ = _timed(stream, lambda: dg.batch(roots, depth=out, params=params, stream=stream))
        bt.append(ms)
        ms, _ = _timed(stream, lambda: dg.batch(roots, depth=out, params=eager, stream=stream))
        et.append(ms)
        ms_seq = 0.0
        for r in roots:
            t, _ = _timed(stream, lambda r=r: dg.run(int(r), depth=depth, want_parent=False, params=params,
                                                         stream=stream))
            ms_seq += t
        st_.append(ms_seq)
    # both forms of the batch must agree with the single runs: `out` holds
    # the kernel-by-kernel batch (the loop's last), then the captured one
    for b in (0, 31, 63):
        dg.run(int(roots[b]), depth=depth, want_parent=False, params=params, stream=stream)
        torch.cuda.synchronize()
        if not torch.equal(depth, out[b]):
            raise RuntimeError(f"batched depths of slot {b} differ from the single-source run")
    dg.batch(roots, depth=out, params=params, stream=stream)
    for b in (0, 31, 63):
        dg.run(int(roots[b]), depth=depth, want_parent=False, params=params, stream=stream)
        torch.cuda.synchronize()
        if not torch.equal(depth, out[b]):
            raise RuntimeError(f"batched depths of slot {b} (captured run) differ from the single-source run")
    batch_ms, seq_ms, eager_ms = min(bt), min(st_), min(et)
    total_mc = float(sum(mc))
    log(f"[batch] 64 roots: batched {batch_ms:.2f} ms as one captured graph ({eager_ms:.2f} ms launched kernel "
        f"by kernel), one at a time {seq_ms:.2f} ms ({seq_ms / batch_ms:.2f}x)")
    dg.free()
    g.free()
    return {"metric": f"batched GTEPS, 64 roots in one pass, kronecker scale {scale}",
            "value": round(total_mc / (batch_ms * 1e-3) / 1e9, 3), "unit": "GTEPS", "n_gpus": 1,
            "steps": args.steps, "warmup": 1, "ms_per_step": round(batch_ms, 3), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
            "config": {"workload": f"kronecker scale {scale} edgefactor {args.edgefactor} seed {seed}, 64 roots "
                                   f"(seed {seed + 1_000_000}), batched vs single-source, degree relabel "
                                   f"{args.reindex}, policy {args.policy}", "n": n, "m": g.m},
            "sequential": {"ms": round(seq_ms, 3), "value": round(total_mc / (seq_ms * 1e-3) / 1e9, 3),
                           "unit": "GTEPS"},
            "eager_batch_ms": round(eager_ms, 3),
            "speedup_vs_sequential": round(seq_ms / batch_ms, 3)}


def bench_pack(args) -> dict:
    """2,000 small graphs in one packed pass vs 2,000 single-source runs."""
    import numpy as np
    import torch
    import graphgen as gg
    import paper_1503_04359_amd as dobfs
    count = args.pack_graphs
    rng = np.random.default_rng(4000)
    scales = rng.integers(10, 19, size=count)
    stream = torch.cuda.current_stream()
    t0 = time.time()
    gs, roots = [], []
    for i in range(count):
        g = gg.kronecker_device(int(scales[i]), args.edgefactor, seed=4000 + i)
        gs.append(g)
        roots.append(int(gg.sample_roots_device(g, 1, seed=4000 + i + 1_000_000)[0]))
    torch.cuda.synchronize()
    n_tot = sum(g.n for g in gs)
    m_tot = sum(g.m for g in gs)
    log(f"[pack] built {count} graphs in {time.time() - t0:.1f}s: {n_tot} vertices, {m_tot} entries")
    reindex = args.reindex == "on"
    t0 = time.time()
    pk = dobfs.Pack.upload(gs, reindex=reindex)
    singles = [dobfs.Graph.from_device_pointers(g.offsets_ptr, g.indices_ptr, g.n, g.m, borrow=True)
               for g in gs]
    torch.cuda.synchronize()
    log(f"[pack] pack and {count} single graphs resident in {time.time() - t0:.1f}s")
    params = dobfs.make_params(args.policy)
    out = torch.empty(pk.n, dtype=torch.int32, device="cuda")
    depth = torch.empty(max(g.n for g in gs), dtype=torch.int32, device="cuda")
    _, _, st = pk.run_pack(roots, depth=out, params=params, stats=True, stream=stream)
    total_mc = float(st.m_c)
    eager = dobfs.make_params(args.policy, flags=dobfs.RUN_EAGER)
    pk.run_pack(roots, depth=out, params=eager, stream=stream)
    pk.run_pack(roots, depth=out, params=params, stream=stream)
    torch.cuda.synchronize()
    pt, stimes, et = [], [], []
    for _ in range(args.steps):
        ms, _ = _timed(stream, lambda: pk.run_pack(roots, depth=out, params=eager, stream=stream))
        et.append(ms)
        ms, _ = _timed(stream, lambda: pk.run_pack(roots, depth=out, params=params, stream=stream))
        pt.append(ms)

        def seq():
            for dg, r in zip(singles, roots):
                dg.run(r, depth=depth, want_parent=False, params=params, stream=stream)
        ms, _ = _timed(stream, seq)
        stimes.append(ms)
    # spot-check the pack against single runs
    for i in (0, count // 2, count - 1):
        singles[i].run(roots[i], depth=depth, want_parent=False, params=params, stream=stream)
        torch.cuda.synchronize()
        lo = int(pk.bases[i])
        if not torch.equal(depth[:gs[i].n], out[lo:lo + gs[i].n]):
            raise RuntimeError(f"packed depths of graph {i} differ from its single-source run")
    pack_ms, seq_ms, eager_ms = min(pt), min(stimes), min(et)
    log(f"[pack] {count} graphs: one pass {pack_ms:.2f} ms as one captured graph ({eager_ms:.2f} ms launched "
        f"kernel by kernel), one at a time {seq_ms:.2f} ms ({seq_ms / pack_ms:.2f}x)")
    for dg in singles:
        dg.free()
    pk.free()
    for g in gs:
        g.free()
    return {"metric": f"packed graphs/s, {count} kronecker graphs of scale 10..18 in one pass",
            "value": round(count / (pack_ms * 1e-3), 1), "unit": "graphs/s", "n_gpus": 1, "steps": args.steps,
            "warmup": 1, "ms_per_step": round(pack_ms, 3), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "int32", "data": "synthetic",
            "config": {"workload": f"{count} kronecker graphs, scales uniform over 10..18 (seed 4000), "
                                   f"edgefactor {args.edgefactor}, graph seeds 4000+i, one root each, degree "
                                   f"relabel {args.reindex}", "n": n_tot, "m": m_tot},
            "gteps": round(total_mc / (pack_ms * 1e-3) / 1e9, 3),
            "sequential": {"ms": round(seq_ms, 3), "value": round(count / (seq_ms * 1e-3), 1),
                           "unit": "graphs/s"},
            "eager_pack_ms": round(eager_ms, 3),
            "speedup_vs_sequential": round(seq_ms / pack_ms, 3)}


def bench_chunglu(args) -> dict:
    """Single-source DOBFS on the Chung-Lu stand-in for a real-world graph."""
    import numpy as np
    import torch
    import graphgen as gg
    import paper_1503_04359_amd as dobfs
    n_core, seed = args.cl_core, 3
    t0 = time.time()
    g = gg.chung_lu_device(n_core, gamma=2.2, avg_deg=20.0, max_deg=1e6, n_tails=50, tail_len=200, seed=seed)
    log(f"[chunglu] built on the device in {time.time() - t0:.1f}s (n={g.n}, m={g.m})")
    roots = gg.sample_roots_device(g, args.roots, seed=seed + 1_000_000)
    reindex = args.reindex == "on"
    t0 = time.time()
    dg = dobfs.Graph.from_device_pointers(g.offsets_ptr, g.indices_ptr, g.n, g.m, borrow=not reindex,
                                          reindex=reindex)
    torch.cuda.synchronize()
    log(f"[chunglu] resident in {time.time() - t0:.1f}s")
    n, m = g.n, g.m
    if reindex:
        g.free()
    stream = torch.cuda.current_stream()
    depth = torch.empty(n, dtype=torch.int32, device="cuda")
    parent = torch.empty(n, dtype=torch.int32, device="cuda")
    params = dobfs.make_params(args.policy)
    for r in roots:  # warm-up
        dg.run(int(r), depth, parent, params=params, stream=stream)
    torch.cuda.synchronize()
    teps, times, lines = [], [], []
    for _ in range(args.steps):
        for r in roots:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            _, _, st = dg.run(int(r), depth, parent, params=params, stats=True, stream=stream)
            e1.record(stream)
            e1.synchronize()
            ms = e0.elapsed_time(e1)
            times.append(ms)
            teps.append(st.m_c / (ms * 1e-3))
            dirs = "".join("TB"[rec["dir"]] for rec in st.log)
            switches = sum(1 for a, b in zip(dirs, dirs[1:]) if a != b)
            lines.append((int(r), st.levels, switches, ms))
    gteps = harmonic_mean(teps) / 1e9
    for r, lv, sw, ms in lines[:len(roots)]:
        log(f"[chunglu] root {r}: {lv} levels, {sw} direction switches, {ms:.2f} ms")
    log(f"[chunglu] {gteps:.1f} GTEPS harmonic mean")
    dg.free()
    if not reindex:
        g.free()
    return {"metric": "GTEPS (harmonic mean over roots), Chung-Lu power-law graph with path tails",
            "value": round(gteps, 3), "unit": "GTEPS", "n_gpus": 1, "steps": args.steps, "warmup": 1,
            "ms_per_step": round(sum(times) / args.steps, 3), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "int32", "data": "synthetic",
            "config": {"workload": f"Chung-Lu {n_core} core vertices, exponent 2.2, mean degree 20, max 1e6, "
                                   f"50 tails x 200 (seed {seed}), {args.roots} roots (seed {seed + 1_000_000}), "
                                   f"policy {args.policy}, degree relabel {args.reindex}", "n": n, "m": m,
                       "levels": [lv for _, lv, _, _ in lines[:len(roots)]],
                       "direction_switches": [sw for _, _, sw, _ in lines[:len(roots)]]}}


def _traversed_edges(dobfs, graphs, queries):
    """Undirected edges each query's traversal covers: one run per graph
    marks the component of its first root; other roots are run alone."""
    import torch
    import numpy as np
    by_graph = {}
    for q in queries:
        by_graph.setdefault(q.gid, set()).add(q.root)
    mc = {}
    for gid, rs in by_graph.items():
        g = graphs[gid]
        rs = sorted(rs)
        d, _, st = g.run(rs[0], want_parent=False, stats=True)
        torch.cuda.synchronize()
        comp = (d >= 0).cpu().numpy()
        for r in rs:
            if comp[r]:
                mc[(gid, r)] = st.m_c
            else:
                _, _, s2 = g.run(r, want_parent=False, stats=True)
                mc[(gid, r)] = s2.m_c
    return mc


def bench_serve(args) -> dict:
    import numpy as np
    import torch
    import graphgen as gg
    import paper_1503_04359_amd as dobfs
    from paper_1503_04359_amd import serve
    scales = [18, 20, 22, 24, 24, 25, 26, 26]
    reindex = args.reindex == "on"
    t0 = time.time()
    graphs, pools, dev = [], [], []
    for j, sc in enumerate(scales):
        g = gg.kronecker_device(sc, args.edgefactor, seed=5000 + j)
        pools.append(gg.sample_roots_device(g, 256, seed=5000 + j + 1_000_000))
        graphs.append(dobfs.Graph.from_device_pointers(g.offsets_ptr, g.indices_ptr, g.n, g.m,
                                                       borrow=not reindex, reindex=reindex))
        if reindex:
            g.free()
        else:
            dev.append(g)
    torch.cuda.synchronize()
    log(f"[serve] {len(graphs)} graphs resident in {time.time() - t0:.1f}s "
        f"({sum(g.n for g in graphs)} vertices)")
    params = dobfs.make_params(args.policy, chunk_levels=args.serve_chunk)
    ex = serve.GpuExecutor(graphs, params=params)
    free, _ = torch.cuda.mem_get_info()
    budget = max(0, free - (16 << 30))
    srv = serve.Server(ex, memory_budget=budget, plain_max=args.serve_plain_max,
                       plain_concurrency=args.serve_plain_concurrency)
    # warm-up: one session and one plain run per graph
    warm = [serve.Query(i, gid, int(pools[gid][0]), 0.0) for i, gid in enumerate(range(len(graphs)))]
    srv.serve(warm, mode="batched", drain_s=30.0)
    srv.serve(warm, mode="plain", drain_s=30.0)
    rates = [float(x) for x in args.serve_rates.split(",")]
    results = []
    all_q = []
    for rate in rates:
        trace = serve.poisson_trace(rate, args.serve_duration, len(graphs), pools, seed=6000 + int(rate))
        row = {"rate": rate, "offered": len(trace)}
        for mode in ("batched", "plain"):
            tr = [serve.Query(q.qid, q.gid, q.root, q.t_arrival) for q in trace]
            torch.cuda.synchronize()
            solo0 = srv.solo_runs
            rep, _ = srv.serve(tr, mode=mode, drain_s=args.serve_drain)
            if mode == "batched":
                row["plain_runs_in_batched"] = srv.solo_runs - solo0
            all_q.extend(q for q in tr if q.t_done is not None)
            row[mode] = rep.as_dict()
            row[mode]["_queries"] = tr
            log(f"[serve] rate {rate:g}/s {mode}: completed {rep.completed}/{rep.offered} "
                f"({rep.unfinished} unfinished), {rep.qps:.0f} q/s, p50 {rep.p50_ms} ms, p99 {rep.p99_ms} ms")
        results.append(row)
    mc = _traversed_edges(dobfs, graphs, all_q)
    for row in results:
        for mode in ("batched", "plain"):
            tr = row[mode].pop("_queries")
            edges = sum(mc[(q.gid, q.root)] for q in tr if q.t_done is not None)
            row[mode]["gteps"] = round(edges / row[mode]["makespan_s"] / 1e9, 3) if row[mode]["makespan_s"] else 0.0
            row[mode].pop("per_graph", None)
            for k in ("p50_ms", "p99_ms", "mean_ms", "qps", "makespan_s"):
                if row[mode][k] is not None:
                    row[mode][k] = round(row[mode][k], 3)
    for g in graphs:
        g.free()
    for g in dev:
        g.free()
    top = results[-1]
    return {"metric": "served queries/s + p99 vs plain (continuous batching)",
            "value": top["batched"]["qps"], "unit": "queries/s", "n_gpus": 1, "steps": len(rates), "warmup": 1,
            "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "int32", "data": "synthetic",
            "config": {"workload": "8 resident kronecker graphs (scales 18,20,22,24,24,25,26,26, edgefactor "
                                   f"{args.edgefactor}, seeds 5000+j), Poisson arrivals (seed 6000+rate) for "
                                   f"{args.serve_duration:g} s per rate, uniform graph choice, roots from 256 per "
                                   f"graph (seed 5000+j+10^6), degree relabel {args.reindex}, chunk "
                                   f"{args.serve_chunk} levels, drain {args.serve_drain:g} s, plain runs while at "
                                   f"most {args.serve_plain_max} queries wait on an idle graph, at most "
                                   f"{args.serve_plain_concurrency} such runs at once",
                       "rates": rates},
            "rates": results}


def power_reader():
    """(read() -> watts, source) for the GPU's socket power: the amdgpu
    hwmon node's instantaneous power1_input (microwatts), else amd-smi."""
    import glob
    for path in sorted(glob.glob("/sys/class/drm/card*/device/hwmon/hwmon*/power1_input")):
        try:
            with open(os.path.join(os.path.dirname(path), "name")) as f:
                if f.read().strip() != "amdgpu":
                    continue
            with open(path) as f:
                int(f.read())
        except (OSError, ValueError):
            continue

        def read(path=path):
            with open(path) as f:
                return int(f.read()) / 1e6
        return read, f"sysfs {path}"
    import shutil
    import subprocess
    if shutil.which("amd-smi"):
        def read_smi():
            out = subprocess.run(["amd-smi", "metric", "-p", "--json"], capture_output=True, text=True, timeout=10)
            return float(json.loads(out.stdout)["gpu_data"][0]["power"]["socket_power"]["value"])
        return read_smi, "amd-smi metric -p (socket_power)"
    return None, None


class PowerSampler:
    """Samples the socket power every `period` seconds in a thread."""

    def __init__(self, read, period: float = 0.01):
        import threading
        self.read, self.period = read, period
        self.samples: list[tuple[float, float]] = []
        self._stop = threading.Event()
        self._th = threading.Thread(target=self._run, daemon=True)

    def _run(self):
        while not self._stop.is_set():
            try:
                self.samples.append((time.perf_counter(), self.read()))
            except Exception:  # noqa: BLE001  (a missed sample is skipped)
                pass
            self._stop.wait(self.period)

    def __enter__(self):
        self._th.start()
        return self

    def __exit__(self, *exc):
        self._stop.set()
        self._th.join()

    def mean(self, t0: float, t1: float):
        xs = [w for t, w in self.samples if t0 <= t <= t1]
        return (sum(xs) / len(xs), len(xs)) if xs else (None, 0)


def bench_energy(args) -> dict:
    """Energy efficiency (Section 4.3's MTEPS/W) of single-source traversals
    on the bench workload: traversals run back to back for a fixed window
    while the GPU's socket power is sampled; idle power is sampled before."""
    import torch
    import graphgen as gg
    import paper_1503_04359_amd as dobfs
    from paper_1503_04359_amd import autotune
    read, source = power_reader()
    if read is None:
        raise RuntimeError("no GPU power reading available (amdgpu hwmon or amd-smi)")
    t0 = time.time()
    g = gg.kronecker_device(args.scale, args.edgefactor, seed=args.seed)
    roots = gg.sample_roots_device(g, args.roots, seed=args.seed + 1_000_000)
    dg = dobfs.Graph.from_device_pointers(g.offsets_ptr, g.indices_ptr, g.n, g.m, borrow=False, reindex=True)
    torch.cuda.synchronize()
    n = g.n
    g.free()
    log(f"[energy] kronecker scale {args.scale} resident in {time.time() - t0:.1f}s; power from {source}")
    tuned = autotune.load_tuned(autotune.tuned_path(args.scale, args.edgefactor))
    params = dobfs.make_params("edge", **(tuned["params"] if tuned else {}))
    stream = torch.cuda.current_stream()
    depth = torch.empty(n, dtype=torch.int32, device="cuda")
    parent = torch.empty(n, dtype=torch.int32, device="cuda")
    mc = {}
    for r in roots:
        _, _, st = dg.run(int(r), depth, parent, params=params, stats=True, stream=stream)
        mc[int(r)] = st.m_c
    torch.cuda.synchronize()
    with PowerSampler(read) as ps:
        time.sleep(0.5)
        i0 = time.perf_counter()
        time.sleep(args.energy_idle)
        i1 = time.perf_counter()
        runs, edges = 0, 0
        a0 = time.perf_counter()
        while time.perf_counter() - a0 < args.energy_seconds:
            for r in roots:
                dg.run(int(r), depth, parent, params=params, stream=stream)
                edges += mc[int(r)]
                runs += 1
            torch.cuda.synchronize()
        a1 = time.perf_counter()
    dg.free()
    idle_w, n_idle = ps.mean(i0, i1)
    busy_w, n_busy = ps.mean(a0, a1)
    secs = a1 - a0
    teps = edges / secs
    log(f"[energy] {runs} traversals in {secs:.1f}s: {teps / 1e9:.1f} GTEPS at {busy_w:.0f} W "
        f"(idle {idle_w:.0f} W; {n_busy} samples): {teps / busy_w / 1e6:.1f} MTEPS/W")
    return {"metric": f"MTEPS/W (GPU socket power), kronecker scale {args.scale}", "value": round(teps / busy_w / 1e6, 2),
            "unit": "MTEPS/W", "n_gpus": 1, "steps": runs, "warmup": 1, "ms_per_step": round(secs * 1e3 / runs, 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
            "config": {"workload": f"kronecker scale {args.scale} edgefactor {args.edgefactor} seed {args.seed}, "
                                   f"{args.roots} roots (seed {args.seed + 1_000_000}) run back to back for "
                                   f"{args.energy_seconds:g} s, degree relabel on, policy edge"
                                   + (" (tuned parameters)" if tuned else ""),
                       "power_source": source},
            "gteps": round(teps / 1e9, 3), "seconds": round(secs, 3), "busy_w": round(busy_w, 1),
            "idle_w": round(idle_w, 1), "energy_j": round(busy_w * secs, 1), "samples": n_busy,
            "dynamic_mteps_per_w": round(teps / max(busy_w - idle_w, 1e-9) / 1e6, 2)}


def hybrid_budget(deg, host_frac: float) -> tuple[int, int]:
    """Device budget that leaves the rows of the first ceil(host_frac * n')
    vertices in the degree-class order (n' = vertices of degree >= 1) to the
    host; returns (budget bytes, host vertices asked for)."""
    import numpy as np
    import paper_1503_04359_amd as dobfs
    deg = np.asarray(deg, dtype=np.int64)
    cls = np.zeros_like(deg)
    nz = deg > 0
    cls[nz] = np.floor(np.log2(deg[nz])).astype(np.int64) + 1
    order = np.lexsort((np.arange(deg.shape[0]), -cls))
    k = int(np.ceil(host_frac * int(nz.sum())))
    host_entries = int(deg[order[:k]].sum())
    return dobfs.hybrid_state_bytes(deg.shape[0]) + 4 * (int(deg.sum()) - host_entries), k


def bench_hybrid(args) -> dict:
    """Hybrid host + GPU traversal of a Kronecker graph with the hubs' rows
    in host memory, against the resident traversal of the same roots."""
    import numpy as np
    import torch
    import graphgen as gg
    import paper_1503_04359_amd as dobfs
    scale = args.hybrid_scale
    t0 = time.time()
    dgen = gg.kronecker_device(scale, args.edgefactor, seed=args.seed)
    roots = gg.sample_roots_device(dgen, args.roots, seed=args.seed + 1_000_000)
    g = dgen.to_host()
    dgen.free()
    log(f"[hybrid] kronecker scale {scale} built (n={g.n}, m={g.m}) in {time.time() - t0:.1f}s")
    deg = g.degrees()
    n_ni = int((deg > 0).sum())
    if args.hybrid_budget_gib > 0:
        budget, k = int(args.hybrid_budget_gib * (1 << 30)), None
        placement = f"a fixed device budget of {args.hybrid_budget_gib:g} GiB"
    else:
        budget, k = hybrid_budget(deg, args.hybrid_host_frac)
        placement = (f"rows of the top {args.hybrid_host_frac:.0%} of non-isolated vertices by degree class on the "
                     "host")
    threads = args.hybrid_threads or min(16, len(os.sched_getaffinity(0)))
    t0 = time.time()
    hg = dobfs.HybridGraph.upload(g.offsets, g.indices, gpu_budget_bytes=budget, threads=threads)
    info = hg.info()
    gpu_share = (n_ni - min(info["split"], n_ni)) / max(n_ni, 1)  # non-isolated vertices form an ID prefix
    log(f"[hybrid] split at {info['split']} ({k} asked), {gpu_share:.1%} of the non-isolated vertices on the device: "
        f"host rows {info['host_entries']} entries, device "
        f"{info['gpu_entries']} entries, {info['gpu_bytes'] / 2**30:.2f} GiB on the device; upload "
        f"{time.time() - t0:.1f}s, {threads} host threads")
    flags = dobfs.RUN_HUB_DECIDES if args.hybrid_hub_decides else 0
    params = dobfs.make_params(args.policy, alpha=args.hybrid_alpha, flags=flags)
    hdepth = torch.empty(g.n, dtype=torch.int32, device="cuda")
    hparent = torch.empty(g.n, dtype=torch.int32, device="cuda")
    for r in roots[:2]:  # warm-up
        hg.run(int(r), hdepth, hparent, params=params)
    teps, times, levels = [], [], []
    for _ in range(args.steps):
        for r in roots:
            t = time.perf_counter()
            _, _, st = hg.run(int(r), hdepth, hparent, params=params, stats=True)
            dt = time.perf_counter() - t
            times.append(dt * 1e3)
            teps.append(st.m_c / dt)
            levels.append(st.levels)
    gteps = harmonic_mean(teps) / 1e9
    log(f"[hybrid] {gteps:.2f} GTEPS harmonic mean, {np.mean(times):.1f} ms per root")
    tp = dobfs.make_params(args.policy, alpha=args.hybrid_alpha, flags=flags | dobfs.RUN_TIME_KERNELS)
    t = time.perf_counter()
    _, _, st = hg.run(int(roots[0]), hdepth, hparent, params=tp, stats=True)
    wall = (time.perf_counter() - t) * 1e3
    prev = 0
    for rec in st.log:
        log(f"[hybrid] root {int(roots[0])} level {rec['level']} {'TB'[rec['dir']]}: n_f {rec['n_f']}, "
            f"checked {rec['checked']}, found {rec['found']}, host {rec['kernel_ms']:.2f} ms, "
            f"level wall {(rec['t_end'] - prev) / 1e6:.2f} ms")
        prev = rec["t_end"]
    log(f"[hybrid] GPU kernels: td {st.td_kernel_ms:.2f} ms, bu {st.bu_kernel_ms:.2f} ms, aux {st.aux_kernel_ms:.2f} ms;"
        f" levels end at {prev / 1e6:.2f} ms of {wall:.2f} ms")
    hg.free()
    del hdepth, hparent
    # the same roots on the resident path (whole graph on the device), with
    # the library's switching constants
    params = dobfs.make_params(args.policy)
    dg = dobfs.Graph.upload(g.offsets, g.indices, reindex=True)
    stream = torch.cuda.current_stream()
    depth = torch.empty(g.n, dtype=torch.int32, device="cuda")
    rt = []
    for r in roots:
        dg.run(int(r), depth, params=params, stream=stream)
    torch.cuda.synchronize()
    for r in roots:
        ms, out = _timed(stream, lambda r=r: dg.run(int(r), depth, params=params, stats=True, stream=stream))
        rt.append(out[2].m_c / (ms * 1e-3))
    dg.free()
    res = harmonic_mean(rt) / 1e9
    log(f"[hybrid] resident run on the same roots: {res:.1f} GTEPS")
    return {"metric": f"GTEPS (harmonic mean over roots), hybrid host + GPU, kronecker scale {scale}",
            "value": round(gteps, 3), "unit": "GTEPS", "n_gpus": 1, "steps": args.steps, "warmup": 1,
            "ms_per_step": round(sum(times) / args.steps, 3), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "int32", "data": "synthetic",
            "config": {"workload": f"kronecker scale {scale} edgefactor {args.edgefactor} seed {args.seed}, "
                                   f"{placement} ({threads} host threads), the rest on the device; "
                                   f"{args.roots} roots (seed {args.seed + 1_000_000}), policy {args.policy} "
                                   + (f"with alpha {args.hybrid_alpha}" if args.policy == "edge" else "")
                                   + (", the host partition deciding the switch" if args.hybrid_hub_decides else ""),
                       "n": g.n, "m": g.m, "split": info["split"], "host_entries": info["host_entries"],
                       "gpu_entries": info["gpu_entries"], "gpu_bytes": info["gpu_bytes"],
                       "device_budget": budget, "gpu_share_nonisolated": round(gpu_share, 4),
                       "levels": levels[:len(roots)]},
            "resident_gteps": round(res, 3), "host": host_spec()}


def traffic_from_counters(fetch_csv: str, write_csv: str, probe_bytes: int, key: str, out_path: str) -> dict:
    """HBM bytes per launch of each traversal kernel from two rocprofv3
    --pmc runs of the same command (FETCH_SIZE, then WRITE_SIZE, KiB per
    dispatch), each scaled by what the counter reads for the copy probe,
    whose kernel reads and writes `probe_bytes` bytes."""
    import csv

    def load(path, counter):
        """Copy-probe reading, then per kernel: summed readings and launches."""
        probe, per = [], {k: [0.0, 0] for k in TRAFFIC_KERNELS}
        with open(path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != counter:
                    continue
                name, val = r["Kernel_Name"], float(r["Counter_Value"]) * 1024.0
                if "CUDAFunctorOnSelf_add" in name:
                    probe.append(val)
                    continue
                for k in TRAFFIC_KERNELS:
                    if f"{k}(" in name:
                        per[k][0] += val
                        per[k][1] += 1
        if not probe or not per[DOMINANT][1]:
            raise ValueError(f"{path}: no copy-probe or {DOMINANT} dispatches for {counter}")
        return probe[0], per

    pf, fetch = load(fetch_csv, "FETCH_SIZE")
    pw, write = load(write_csv, "WRITE_SIZE")
    kf, kw = probe_bytes / pf, probe_bytes / pw
    kernels = {}
    for k in TRAFFIC_KERNELS:
        (fv, fn), (wv, wn) = fetch[k], write[k]
        if not fn or not wn:
            continue
        kernels[k] = {"launches": fn, "fetch_bytes_per_launch": round(fv * kf / fn),
                      "write_bytes_per_launch": round(wv * kw / wn),
                      "bytes_per_launch": round(fv * kf / fn + wv * kw / wn)}
    ent = {"source_sha256": kernel_source_digest(), "fetch_factor": round(kf, 4), "write_factor": round(kw, 4),
           "kernels": kernels}
    data = {}
    if os.path.exists(out_path):
        with open(out_path) as f:
            data = json.load(f)
    data[key] = ent
    with open(out_path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
        f.write("\n")
    return ent


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic.json from two rocprofv3 --pmc counter CSVs of this bench "
                         "(run with --copy-probe) and exit")
    ap.add_argument("--mode", choices=("single", "batch", "pack", "serve", "chunglu", "energy", "hybrid"),
                    default="single")
    ap.add_argument("--hybrid-scale", type=int, default=26, help="hybrid mode: Kronecker scale")
    ap.add_argument("--hybrid-host-frac", type=float, default=0.12,
                    help="hybrid mode: share of the non-isolated vertices (highest degree first) kept on the host")
    ap.add_argument("--hybrid-threads", type=int, default=0, help="hybrid mode: host threads (0: up to 16)")
    ap.add_argument("--hybrid-budget-gib", type=float, default=0.0,
                    help="hybrid mode: a fixed device-memory budget instead of --hybrid-host-frac")
    ap.add_argument("--hybrid-hub-decides", action="store_true",
                    help="hybrid mode: the host partition's own next frontier decides the switch (PAPER policy)")
    ap.add_argument("--hybrid-alpha", type=int, default=56,
                    help="hybrid mode: EDGE policy's alpha (a sweep at scale 26 put the hybrid's best at 56-112; the "
                         "resident path's 14 leaves hub rows to host top-down levels)")
    ap.add_argument("--energy-seconds", type=float, default=20.0, help="energy mode: length of the measured window")
    ap.add_argument("--energy-idle", type=float, default=3.0, help="energy mode: idle power sampled before")
    ap.add_argument("--cl-core", type=int, default=100_000_000, help="chunglu mode: core vertices")
    ap.add_argument("--pack-graphs", type=int, default=2000)
    ap.add_argument("--serve-rates", default="500,2000,8000")
    ap.add_argument("--serve-duration", type=float, default=10.0)
    ap.add_argument("--serve-drain", type=float, default=5.0)
    ap.add_argument("--serve-chunk", type=int, default=4)
    ap.add_argument("--serve-plain-max", type=int, default=8,
                    help="serve mode: waiting queries of an idle graph run plain up to this many")
    ap.add_argument("--serve-plain-concurrency", type=int, default=2,
                    help="serve mode: plain runs of the batched mode that may execute at once")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--param", action="append", default=[], metavar="NAME=VALUE",
                    help="override a dobfs_params field (e.g. alpha=14), repeatable")
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--scale", type=int, default=30)
    ap.add_argument("--edgefactor", type=int, default=16)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--roots", type=int, default=16)
    ap.add_argument("--policy", default="edge")
    ap.add_argument("--reindex", choices=("on", "off"), default="on",
                    help="degree relabelling inside the library (outputs stay in caller labels)")
    ap.add_argument("--cpu-scale", type=int, default=26)
    ap.add_argument("--cpu-roots", type=int, default=16)
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle time for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tuned", action="store_true", help="library defaults instead of the autotuned parameters")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic.json"),
                    help="measured HBM bytes per level-kernel launch (rocprofv3 --pmc), if present")
    ap.add_argument("--copy-probe", type=float, default=0.0,
                    help="first run a plain device copy kernel over this many GiB (counter calibration)")
    args = ap.parse_args()

    if args.traffic_from:
        key = f"kron-s{args.scale}-ef{args.edgefactor}-seed{args.seed}/{args.policy}/reindex-{args.reindex}"
        nbytes = int(args.copy_probe * (1 << 30)) // 4 * 4
        if nbytes <= 0:
            print("--traffic-from needs the --copy-probe size the counters were taken with", file=sys.stderr)
            return 2
        print(json.dumps(traffic_from_counters(args.traffic_from[0], args.traffic_from[1], nbytes, key,
                                               args.traffic)))
        return 0

    if args.gpus != 1:
        print(f"bench.py: runs on one GPU; --gpus {args.gpus} is not supported "
              "(the traversal is not sharded across GPUs; the result is one GPU's throughput).", file=sys.stderr)
        return 2

    import __graft_entry__
    __graft_entry__.ensure_built()
    import torch

    import graphgen as gg
    import paper_1503_04359_amd as dobfs

    torch.cuda.set_device(0)
    if args.mode != "single":
        fn = {"batch": bench_batch, "pack": bench_pack, "serve": bench_serve, "chunglu": bench_chunglu,
              "energy": bench_energy, "hybrid": bench_hybrid}[args.mode]
        print(json.dumps(fn(args)), flush=True)
        return 0
    stream = torch.cuda.current_stream()
    if args.copy_probe > 0:
        # elementwise copy kernel: reads and writes exactly `nbytes` each
        nbytes = int(args.copy_probe * (1 << 30)) // 4 * 4
        a = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        torch.add(a, 0, out=b)
        torch.cuda.synchronize()
        log(f"[gpu] copy probe: {nbytes} bytes read and written by one elementwise kernel")
        del a, b
        torch.cuda.empty_cache()
    t0 = time.time()
    g = gg.kronecker_device(args.scale, args.edgefactor, seed=args.seed)
    torch.cuda.synchronize()
    log(f"[gpu] built kronecker scale {args.scale} on the device in {time.time() - t0:.1f}s "
        f"(n={g.n}, m={g.m})")
    roots = gg.sample_roots_device(g, args.roots, seed=args.seed + 1_000_000)
    reindex = args.reindex == "on"
    t0 = time.time()
    dg = dobfs.Graph.from_device_pointers(g.offsets_ptr, g.indices_ptr, g.n, g.m, borrow=not reindex,
                                          reindex=reindex)
    torch.cuda.synchronize()
    log(f"[gpu] graph resident ({'degree-relabelled copy' if reindex else 'borrowed in place'}) "
        f"in {time.time() - t0:.1f}s")
    n, m = g.n, g.m
    if reindex:
        g.free()  # the library keeps its own relabelled copy
    info = dg.info()
    words_active = ((info["n_nonisolated"] if reindex else info["n"]) + 63) // 64
    depth = torch.empty(n, dtype=torch.int32, device="cuda")
    parent = torch.empty(n, dtype=torch.int32, device="cuda")
    overrides = {k: int(v) for k, v in (kv.split("=", 1) for kv in args.param)}
    # parameters chosen by the autotuner on its own roots (never these), for
    # the configuration it tuned: degree relabel on, the edge-count rule
    from paper_1503_04359_amd import autotune
    tuned = None
    if not args.no_tuned and reindex and args.policy == "edge":
        tuned = autotune.load_tuned(autotune.tuned_path(args.scale, args.edgefactor))
    eff = dict(tuned["params"]) if tuned else {}
    eff.update(overrides)
    params = dobfs.make_params(args.policy, **eff)
    # a separate step, not counted in the metric, brackets every level-kernel
    # launch with events for the per-kernel roofline
    params_prof = dobfs.make_params(args.policy, flags=dobfs.RUN_TIME_KERNELS, **eff)
    if tuned:
        log(f"[gpu] tuned parameters {tuned['params']} ({os.path.relpath(autotune.tuned_path(args.scale, args.edgefactor), ROOT)})")

    def one_step(record, prm):
        for r in roots:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            _, _, st = dg.run(int(r), depth, parent, params=prm, stats=True, stream=stream)
            e1.record(stream)
            record.append((int(r), e0, e1, st))

    for _ in range(args.warmup):
        one_step([], params)
    torch.cuda.synchronize()
    runs: list = []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        one_step(runs, params)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    prof: list = []
    one_step(prof, params_prof)
    torch.cuda.synchronize()

    teps, times, lines = [], [], {}
    for r, e0, e1, st in runs:
        ms = e0.elapsed_time(e1)
        times.append(ms)
        teps.append(st.m_c / (ms * 1e-3))
        lines.setdefault(r, (st.levels, st.m_c, [rec["dir"] for rec in st.log]))
    bu_bytes = td_bytes = 0.0
    bu_ms = td_ms = aux_ms = 0.0
    launches = 0
    for r, _, _, st in prof:
        if st.log_len != st.levels:
            raise RuntimeError(f"root {r}: level log truncated ({st.log_len} of {st.levels})")
        for i, rec in enumerate(st.log):
            if rec["dir"] == 1:
                bu_bytes += bottom_up_bytes(rec, words_active)
            else:
                td_bytes += top_down_bytes(rec) + to_queue_bytes(st.log, i, words_active)
        bu_ms += st.bu_kernel_ms
        td_ms += st.td_kernel_ms
        aux_ms += st.aux_kernel_ms
        launches += st.level_launches
    gteps = harmonic_mean(teps) / 1e9
    ms_per_step = sum(times) / args.steps
    for r, (lv, mc, dirs) in lines.items():
        rt = [t for (rr, _, _, _), t in zip(runs, times) if rr == r]
        log(f"[gpu] root {r}: levels {lv} m_c {mc} dirs {''.join('TB'[d] for d in dirs)} "
            f"best {min(rt):.3f} ms -> {mc / min(rt) / 1e6:.1f} GTEPS")
    # the dominant kernel: k_level_bu is launched once per level slot; a slot
    # whose level is top-down finds it so and returns at once, and those
    # launches count in both the launch count and the summed duration
    bu_avg_ms = bu_ms / max(1, launches)
    bu_per_launch = bu_bytes / max(1, launches)
    achieved = bu_per_launch / (bu_avg_ms * 1e-3) / 1e9 if bu_avg_ms > 0 else 0.0
    td_gbs = td_bytes / ((td_ms + aux_ms) * 1e-3) / 1e9 if td_ms + aux_ms > 0 else 0.0
    traffic = traffic_src = None
    if os.path.exists(args.traffic):
        try:
            with open(args.traffic) as f:
                tr = json.load(f)
            key = f"kron-s{args.scale}-ef{args.edgefactor}-seed{args.seed}/{args.policy}/reindex-{args.reindex}"
            ent = tr.get(key, {})
            if ent.get("source_sha256") == kernel_source_digest():
                traffic = ent["kernels"][DOMINANT]["bytes_per_launch"]
                traffic_src = {k: v["bytes_per_launch"] for k, v in ent["kernels"].items()}
        except (OSError, ValueError, KeyError):
            traffic = traffic_src = None
    roofline = {"bound": "hbm", "kernel": DOMINANT, "source_sha256": kernel_source_digest()[:16],
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "bytes_per_launch": round(bu_per_launch), "avg_launch_ms": round(bu_avg_ms, 5),
                "launches": launches,
                "top_down_path": {"kernels": "k_level_td+k_aux", "bytes": round(td_bytes),
                                  "ms": round(td_ms + aux_ms, 3), "achieved": round(td_gbs, 1),
                                  "frac": round(td_gbs / HBM_PEAK_GBS, 4)},
                "measured_traffic_per_launch": traffic_src}
    log(f"[gpu] {gteps:.1f} GTEPS harmonic mean; wall {wall:.2f}s for {args.steps} steps; "
        f"{DOMINANT} {achieved:.0f} GB/s algorithmic ({bu_ms:.1f} ms over {launches} launches); "
        f"top-down path {td_gbs:.0f} GB/s ({td_ms + aux_ms:.1f} ms)")
    dg.free()
    if not reindex:
        g.free()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.cpu_scale, args.seed, args.cpu_roots, args.cpu_budget)

    out = {"metric": METRIC, "value": round(gteps, 3), "unit": "GTEPS", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
           "config": {"workload": f"kronecker scale {args.scale} edgefactor {args.edgefactor} "
                                  f"A/B/C 0.57/0.19/0.19 seed {args.seed}, {args.roots} roots, "
                                  f"single-source DOBFS, policy {args.policy}, degree relabel {args.reindex}",
                      "scale": args.scale, "edgefactor": args.edgefactor, "n": n, "m": m,
                      "roots": args.roots, "policy": args.policy, "reindex": reindex,
                      "params": {k: getattr(params, k) for k in autotune.SPACE},
                      "tuned_from": (os.path.relpath(autotune.tuned_path(args.scale, args.edgefactor), ROOT)
                                     if tuned else None),
                      "overrides": overrides},
           "roofline": roofline, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
