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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def level_bytes(rec: dict, words_active: int) -> float:
    """Algorithmic bytes of one level of the level kernel.

    top-down: queue entry (4) + two offsets (16) per frontier vertex; one
      neighbour ID (4) and one visited-bit probe (1/8) per examined edge;
      per new vertex its two offsets (16), depth, parent and queue entry (12)
      and its visited and frontier bits (2/8).
    bottom-up: visited word read and next-frontier word write (16) per
      active 64-vertex word; one offset (8) per scanned vertex; one neighbour
      ID (4) and one frontier-bit probe (1/8) per examined edge; depth and
      parent (8) per new vertex.
    """
    if rec["dir"] == 0:
        return (20.0 * rec["n_f"] + (4.0 + 0.125) * rec["checked"] + (28.0 + 0.25) * rec["found"])
    return (16.0 * words_active + 8.0 * rec["scanned"] + (4.0 + 0.125) * rec["checked"] + 8.0 * rec["found"])


def kernel_source_digest() -> str:
    """Identity of the level kernel's source: measured traffic is only
    reported for the kernel it was measured on."""
    import hashlib
    h = hashlib.sha256()
    for f in ("bfs_kernels.hip", "dobfs_internal.h"):
        with open(os.path.join(ROOT, "paper_1503_04359_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def harmonic_mean(xs):
    return len(xs) / sum(1.0 / x for x in xs)


def cpu_baseline(scale: int, seed: int, nroots: int) -> dict:
    """The oracle (serial queue BFS, one thread) on a bounded sample."""
    import graphgen as gg
    import oracle
    t0 = time.time()
    g = gg.kronecker(scale, seed=seed)
    log(f"[cpu] host-built kronecker scale {scale} in {time.time() - t0:.1f}s (n={g.n}, m={g.m})")
    roots = gg.sample_roots(g, nroots, seed=seed + 1_000_000)
    teps = []
    total = 0.0
    for r in roots:
        t = time.perf_counter()
        d, _ = oracle.bfs(g.offsets, g.indices, int(r))
        dt = time.perf_counter() - t
        total += dt
        teps.append(oracle.traversed_edges(g.offsets, d) / dt)
    val = harmonic_mean(teps) / 1e9
    log(f"[cpu] oracle {nroots} roots in {total:.1f}s: {val:.4f} GTEPS")
    return {"value": round(val, 5), "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "sample": f"serial queue BFS (one thread) over a host-built Kronecker graph of scale {scale} "
                      f"(edgefactor 16, same initiator, seed {seed}), {nroots} roots drawn as for the GPU run, "
                      f"harmonic mean; {total:.1f}s of CPU time"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--scale", type=int, default=30)
    ap.add_argument("--edgefactor", type=int, default=16)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--roots", type=int, default=16)
    ap.add_argument("--policy", default="edge")
    ap.add_argument("--reindex", choices=("on", "off"), default="on",
                    help="degree relabelling inside the library (outputs stay in caller labels)")
    ap.add_argument("--cpu-scale", type=int, default=22)
    ap.add_argument("--cpu-roots", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic.json"),
                    help="measured HBM bytes per level-kernel launch (rocprofv3 --pmc), if present")
    ap.add_argument("--copy-probe", type=float, default=0.0,
                    help="first run a plain device copy kernel over this many GiB (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the single-GPU result is the throughput of one GPU).", file=sys.stderr)
        return 2

    import __graft_entry__
    __graft_entry__.ensure_built()
    import torch

    import graphgen as gg
    import paper_1503_04359_amd as dobfs

    torch.cuda.set_device(0)
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
    params = dobfs.make_params(args.policy, flags=dobfs.RUN_TIME_KERNELS)

    def one_step(record):
        for r in roots:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            _, _, st = dg.run(int(r), depth, parent, params=params, stats=True, stream=stream)
            e1.record(stream)
            record.append((int(r), e0, e1, st))

    for _ in range(args.warmup):
        one_step([])
    torch.cuda.synchronize()
    runs: list = []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        one_step(runs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start

    teps, times, lines = [], [], {}
    tot_bytes = tot_kms = 0.0
    tot_launch = 0
    for r, e0, e1, st in runs:
        ms = e0.elapsed_time(e1)
        times.append(ms)
        teps.append(st.m_c / (ms * 1e-3))
        tot_bytes += sum(level_bytes(rec, words_active) for rec in st.log)
        tot_kms += st.level_kernel_ms
        tot_launch += st.level_launches
        lines.setdefault(r, (st.levels, st.m_c, [rec["dir"] for rec in st.log]))
    gteps = harmonic_mean(teps) / 1e9
    ms_per_step = sum(times) / args.steps
    for r, (lv, mc, dirs) in lines.items():
        rt = [t for (rr, _, _, _), t in zip(runs, times) if rr == r]
        log(f"[gpu] root {r}: levels {lv} m_c {mc} dirs {''.join('TB'[d] for d in dirs)} "
            f"best {min(rt):.3f} ms -> {mc / min(rt) / 1e6:.1f} GTEPS")
    avg_ms = tot_kms / max(1, tot_launch)
    per_launch = tot_bytes / max(1, tot_launch)
    achieved = per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    traffic = None
    if os.path.exists(args.traffic):
        try:
            with open(args.traffic) as f:
                tr = json.load(f)
            key = f"kron-s{args.scale}-ef{args.edgefactor}-seed{args.seed}/{args.policy}/reindex-{args.reindex}"
            ent = tr.get(key, {})
            if ent.get("kernel") == "k_level" and ent.get("source_sha256") == kernel_source_digest():
                traffic = ent["bytes_per_launch"]
        except (OSError, ValueError):
            traffic = None
    roofline = {"bound": "hbm", "kernel": "k_level", "source_sha256": kernel_source_digest()[:16], "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "bytes_per_launch": round(per_launch), "avg_launch_ms": round(avg_ms, 5),
                "launches": tot_launch}
    log(f"[gpu] {gteps:.1f} GTEPS harmonic mean; wall {wall:.2f}s for {args.steps} steps; "
        f"level kernel {achieved:.0f} GB/s algorithmic over {tot_launch} launches")

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.cpu_scale, args.seed, args.cpu_roots)

    out = {"metric": METRIC, "value": round(gteps, 3), "unit": "GTEPS", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
           "config": {"workload": f"kronecker scale {args.scale} edgefactor {args.edgefactor} "
                                  f"A/B/C 0.57/0.19/0.19 seed {args.seed}, {args.roots} roots, "
                                  f"single-source DOBFS, policy {args.policy}, degree relabel {args.reindex}",
                      "scale": args.scale, "edgefactor": args.edgefactor, "n": n, "m": m,
                      "roots": args.roots, "policy": args.policy, "reindex": reindex},
           "roofline": roofline, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)
    dg.free()
    g.free()
    return 0


if __name__ == "__main__":
    sys.exit(main())
