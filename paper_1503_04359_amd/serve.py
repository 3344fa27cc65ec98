"""Serving loop for BFS queries (graph id, root) against resident graphs.

Two ways to serve the same open-loop trace of timed arrivals:

* ``batched`` (continuous batching): one worker per graph keeps a session of
  the 64-slot batched traversal running; arrived queries join between level
  chunks as slots and device memory allow, and leave as soon as their own
  traversal ends, so queries that arrive while others run share the device
  with them.  While no session traversal of the graph is in flight and at
  most ``plain_max`` queries wait for it, the oldest runs as a plain
  single-source traversal instead (``solo_plain``): a session level sweeps
  the whole graph, which only pays off when many queries share it (a
  64-root batch costs about as much as 15 plain runs), so a few waiting
  queries finish sooner one after another.  At most ``plain_concurrency``
  such plain runs execute at once over all graphs, started in arrival order
  (the oldest waiting query first, whatever its graph), so that at low load
  the batched mode serves like the plain one.
* ``plain``: one worker serves the queries one at a time in arrival order,
  each a single-source traversal of its own.

Admission is bounded by a device-memory budget: a query holds its output
(4 bytes per vertex of its graph) from admission until its result has been
handed back.  The executor interface keeps the scheduling logic free of the
device, so it can be driven by a CPU stand-in.
"""
from __future__ import annotations

import heapq
import math
import threading
import time
from dataclasses import dataclass, field
from typing import Callable, Optional, Protocol, Sequence

import numpy as np


@dataclass
class Query:
    qid: int
    gid: int
    root: int
    t_arrival: float              # seconds from the start of the trace
    t_done: Optional[float] = None
    error: Optional[str] = None


class SessionLike(Protocol):
    def admit(self, root: int, tag: int): ...
    def step(self) -> list: ...   # [(tag, result)] of the queries that ended
    def close(self) -> None: ...


class Executor(Protocol):
    n_graphs: int

    def output_bytes(self, gid: int) -> int: ...
    def open_session(self, gid: int) -> SessionLike: ...
    def run_plain(self, gid: int, root: int): ...   # blocks until the result is complete
    def release(self, result) -> None: ...


class MemoryBudget:
    """Bytes that admitted queries may hold; take() fails instead of
    waiting."""

    def __init__(self, total: int):
        self.total = int(total)
        self.used = 0
        self.peak = 0
        self._lock = threading.Lock()

    def take(self, nbytes: int) -> bool:
        with self._lock:
            if self.used + nbytes > self.total:
                return False
            self.used += nbytes
            self.peak = max(self.peak, self.used)
            return True

    def give(self, nbytes: int) -> None:
        with self._lock:
            self.used -= nbytes


def poisson_trace(rate: float, duration: float, n_graphs: int, roots: Sequence[Sequence[int]], seed: int,
                  graph_weights: Optional[Sequence[float]] = None) -> list[Query]:
    """Open-loop arrivals: exponential gaps of mean 1/rate over `duration`
    seconds; each query picks a graph (uniformly unless weighted) and one of
    that graph's roots."""
    rng = np.random.default_rng(seed)
    out: list[Query] = []
    t = 0.0
    p = None
    if graph_weights is not None:
        w = np.asarray(graph_weights, dtype=np.float64)
        p = w / w.sum()
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        gid = int(rng.choice(n_graphs, p=p))
        pool = roots[gid]
        out.append(Query(len(out), gid, int(pool[int(rng.integers(len(pool)))]), t))
    return out


@dataclass
class Report:
    mode: str
    offered: int
    completed: int
    failed: int
    unfinished: int
    makespan_s: float
    qps: float
    p50_ms: Optional[float]
    p99_ms: Optional[float]
    mean_ms: Optional[float]
    peak_memory: int
    per_graph: dict = field(default_factory=dict)

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k in self.__dataclass_fields__}


def _percentile_censored(lat: np.ndarray, n_unfinished: int, q: float) -> Optional[float]:
    """Percentile over all offered queries, unfinished ones counting as
    longer than any finished one: None when the percentile falls among
    them."""
    total = lat.size + n_unfinished
    if total == 0:
        return None
    rank = math.ceil(q / 100.0 * total)  # nearest-rank
    if rank > lat.size:
        return None
    return float(np.sort(lat)[max(rank, 1) - 1])


class Server:
    """Serves a trace through an executor; see the module text."""

    def __init__(self, executor: Executor, memory_budget: int, slots: int = 64,
                 clock: Callable[[], float] = time.perf_counter, poll_s: float = 2e-4, solo_plain: bool = True,
                 plain_max: int = 8, plain_concurrency: int = 2):
        if plain_max < 0:
            raise ValueError("plain_max must be >= 0")
        if plain_concurrency < 1:
            raise ValueError("plain_concurrency must be >= 1")
        self.ex = executor
        self.budget = MemoryBudget(memory_budget)
        self.slots = slots
        self.clock = clock
        self.poll_s = poll_s
        self.solo_plain = solo_plain
        self.plain_max = plain_max if solo_plain else 0
        self._plain_cv = threading.Condition()
        self._plain_q: list = []  # (arrival, qid) of the queries waiting to run plain
        self._plain_busy = 0
        self._plain_conc = plain_concurrency
        self.solo_runs = 0
        self._count_lock = threading.Lock()

    # ---- batched -----------------------------------------------------------
    def _plain_acquire(self, key, t0: float, deadline: float) -> bool:
        """Waits until query `key` = (arrival, qid) is the oldest waiting for
        a plain run and a run may start; False if the deadline passes."""
        with self._plain_cv:
            heapq.heappush(self._plain_q, key)
            while not (self._plain_busy < self._plain_conc and self._plain_q[0] == key):
                if self.clock() - t0 > deadline:
                    self._plain_q.remove(key)
                    heapq.heapify(self._plain_q)
                    self._plain_cv.notify_all()
                    return False
                self._plain_cv.wait(timeout=0.01)
            heapq.heappop(self._plain_q)
            self._plain_busy += 1
            self._plain_cv.notify_all()
            return True

    def _plain_release(self) -> None:
        with self._plain_cv:
            self._plain_busy -= 1
            self._plain_cv.notify_all()

    def _graph_worker(self, gid: int, queries: list[Query], t0: float, deadline: float,
                      results: Optional[dict]) -> None:
        ex = self.ex
        need = ex.output_bytes(gid)
        sess = ex.open_session(gid)
        inflight: dict[int, Query] = {}
        nxt = 0
        try:
            while True:
                now = self.clock() - t0
                if now > deadline:
                    break
                waiting = 0
                while (waiting <= self.plain_max and nxt + waiting < len(queries)
                       and queries[nxt + waiting].t_arrival <= now):
                    waiting += 1
                if not inflight and 1 <= waiting <= self.plain_max:
                    q = queries[nxt]
                    if not self._plain_acquire((q.t_arrival, q.qid), t0, deadline):
                        break
                    if not self.budget.take(need):
                        self._plain_release()
                        time.sleep(self.poll_s)
                        continue
                    nxt += 1
                    try:
                        res = ex.run_plain(gid, q.root)
                    except Exception as e:
                        q.error = f"{type(e).__name__}: {e}"
                        self.budget.give(need)
                        continue
                    finally:
                        self._plain_release()
                    q.t_done = self.clock() - t0
                    with self._count_lock:
                        self.solo_runs += 1
                    if results is not None:
                        results[q.qid] = res
                    else:
                        ex.release(res)
                    self.budget.give(need)
                    continue
                while (nxt < len(queries) and queries[nxt].t_arrival <= now and len(inflight) < self.slots
                       and self.budget.take(need)):
                    q = queries[nxt]
                    try:
                        sess.admit(q.root, q.qid)
                    except Exception:
                        self.budget.give(need)
                        raise
                    inflight[q.qid] = q
                    nxt += 1
                if not inflight:
                    if nxt >= len(queries):
                        break
                    wait = queries[nxt].t_arrival - (self.clock() - t0)
                    time.sleep(min(max(wait, 0.0), self.poll_s) if wait > 0 else self.poll_s)
                    continue
                try:
                    ended = sess.step()
                except Exception as e:  # the session is lost: fail its queries, start a new one
                    for q in inflight.values():
                        q.error = f"{type(e).__name__}: {e}"
                        self.budget.give(need)
                    inflight.clear()
                    try:
                        sess.close()
                    except Exception:
                        pass
                    sess = ex.open_session(gid)
                    continue
                t = self.clock() - t0
                for tag, res in ended:
                    q = inflight.pop(int(tag))
                    q.t_done = t
                    if results is not None:
                        results[q.qid] = res
                    else:
                        ex.release(res)
                    self.budget.give(need)
        finally:
            try:
                sess.close()
            except Exception:
                pass

    # ---- plain -------------------------------------------------------------
    def _plain_worker(self, queries: list[Query], t0: float, deadline: float, results: Optional[dict]) -> None:
        ex = self.ex
        for q in queries:
            while True:
                now = self.clock() - t0
                if now >= q.t_arrival or now > deadline:
                    break
                time.sleep(min(q.t_arrival - now, self.poll_s))
            if self.clock() - t0 > deadline:
                return
            need = ex.output_bytes(q.gid)
            if not self.budget.take(need):  # only this worker holds memory, so waiting would never end
                raise RuntimeError("memory budget smaller than one query's output")
            try:
                res = ex.run_plain(q.gid, q.root)
            except Exception as e:
                q.error = f"{type(e).__name__}: {e}"
                self.budget.give(need)
                continue
            q.t_done = self.clock() - t0
            if results is not None:
                results[q.qid] = res
            else:
                ex.release(res)
            self.budget.give(need)

    def serve(self, trace: list[Query], mode: str = "batched", drain_s: float = 10.0,
              keep_results: bool = False):
        """Runs the trace in real time; queries still running `drain_s`
        seconds after the last arrival are left unfinished.  Returns
        (Report, results by qid if keep_results else None)."""
        if mode not in ("batched", "plain"):
            raise ValueError("mode must be 'batched' or 'plain'")
        for q in trace:
            q.t_done, q.error = None, None
        end = max((q.t_arrival for q in trace), default=0.0)
        deadline = end + drain_s
        results: Optional[dict] = {} if keep_results else None
        t0 = self.clock()
        errors: list[BaseException] = []

        def guard(fn, *a):
            try:
                fn(*a)
            except BaseException as e:  # reported after join
                errors.append(e)

        if mode == "plain":
            th = [threading.Thread(target=guard, args=(self._plain_worker, sorted(trace, key=lambda q: q.t_arrival),
                                                        t0, deadline, results))]
        else:
            by_graph: dict[int, list[Query]] = {}
            for q in sorted(trace, key=lambda q: q.t_arrival):
                by_graph.setdefault(q.gid, []).append(q)
            th = [threading.Thread(target=guard, args=(self._graph_worker, gid, qs, t0, deadline, results))
                  for gid, qs in sorted(by_graph.items())]
        for t in th:
            t.start()
        for t in th:
            t.join()
        if errors:
            raise errors[0]
        return self._report(mode, trace), results

    def _report(self, mode: str, trace: list[Query]) -> Report:
        done = [q for q in trace if q.t_done is not None]
        failed = sum(1 for q in trace if q.error is not None)
        unfinished = len(trace) - len(done) - failed
        lat = np.array([(q.t_done - q.t_arrival) * 1e3 for q in done], dtype=np.float64)
        makespan = max([q.t_done for q in done] + [max((q.t_arrival for q in trace), default=0.0)])
        per_graph = {}
        for gid in sorted({q.gid for q in trace}):
            g_done = np.array([(q.t_done - q.t_arrival) * 1e3 for q in done if q.gid == gid])
            g_unf = sum(1 for q in trace if q.gid == gid and q.t_done is None and q.error is None)
            per_graph[gid] = {"completed": int(g_done.size), "unfinished": g_unf,
                              "p50_ms": _percentile_censored(g_done, g_unf, 50),
                              "p99_ms": _percentile_censored(g_done, g_unf, 99)}
        return Report(mode=mode, offered=len(trace), completed=len(done), failed=failed, unfinished=unfinished,
                      makespan_s=makespan, qps=(len(done) / makespan if makespan > 0 else 0.0),
                      p50_ms=_percentile_censored(lat, unfinished, 50),
                      p99_ms=_percentile_censored(lat, unfinished, 99),
                      mean_ms=float(lat.mean()) if lat.size else None, peak_memory=self.budget.peak,
                      per_graph=per_graph)


class GpuExecutor:
    """Executor over graphs resident on the current GPU (the library's
    Graph objects); each graph's session runs on a stream of its own."""

    def __init__(self, graphs: Sequence, params=None):
        import torch
        self.graphs = list(graphs)
        self.n_graphs = len(self.graphs)
        self.params = params
        self.streams = [torch.cuda.Stream() for _ in self.graphs]

    def output_bytes(self, gid: int) -> int:
        return 4 * self.graphs[gid].n

    def open_session(self, gid: int):
        return _GpuSession(self.graphs[gid], self.params, self.streams[gid])

    def run_plain(self, gid: int, root: int):
        """On the graph's own stream: plain runs and the graph's session are
        issued by the same worker, never at once."""
        import torch
        g = self.graphs[gid]
        st = self.streams[gid]
        with torch.cuda.stream(st):
            depth = torch.empty(g.n, dtype=torch.int32, device="cuda")
        g.run(int(root), depth=depth, want_parent=False, params=self.params, stream=st)
        st.synchronize()
        return depth

    def release(self, result) -> None:
        del result


class _GpuSession:
    def __init__(self, graph, params, stream):
        import torch
        self.stream = stream
        self.n = graph.n
        self.s = graph.session(params=params, stream=stream)
        self._torch = torch

    def admit(self, root: int, tag: int):
        with self._torch.cuda.stream(self.stream):
            depth = self._torch.empty(self.n, dtype=self._torch.int32, device="cuda")
        return self.s.admit(int(root), int(tag), depth=depth)

    def step(self) -> list:
        return self.s.step()

    def close(self) -> None:
        self.s.close()
