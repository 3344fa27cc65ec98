"""Serving loop on the CPU stand-in executor: admission by memory budget,
slot refill, failure injection and the same result alone and in the mix."""
from __future__ import annotations

import numpy as np
import pytest

import graphgen as gg
import oracle
from paper_1503_04359_amd import serve
from serve_fakes import CpuExecutor


def _graphs():
    return [gg.kronecker(9, seed=1), gg.disjoint_union(gg.path(60), gg.star(30), gg.from_edges(2, [], [])),
            gg.chung_lu(800, gamma=2.2, avg_deg=5.0, max_deg=100.0, n_tails=1, tail_len=40, seed=3)]


def _roots(gs):
    rng = np.random.default_rng(0)
    return [rng.integers(0, g.n, size=20) for g in gs]


def _expected(gs, trace):
    cache = {}
    for q in trace:
        key = (q.gid, q.root)
        if key not in cache:
            g = gs[q.gid]
            cache[key] = oracle.bfs(g.offsets, g.indices, q.root)[0]
    return cache


def test_poisson_trace_is_seeded_and_has_the_rate():
    a = serve.poisson_trace(2000.0, 2.0, 3, [[1, 2], [3], [4, 5, 6]], seed=6000)
    b = serve.poisson_trace(2000.0, 2.0, 3, [[1, 2], [3], [4, 5, 6]], seed=6000)
    assert [(q.t_arrival, q.gid, q.root) for q in a] == [(q.t_arrival, q.gid, q.root) for q in b]
    assert abs(len(a) - 4000) < 4 * np.sqrt(4000)
    assert all(0 <= q.t_arrival < 2.0 for q in a)
    assert {q.root for q in a if q.gid == 1} == {3}


def test_censored_percentile():
    lat = np.array([1.0, 2.0, 3.0, 4.0])
    assert serve._percentile_censored(lat, 0, 50) == 2.0
    assert serve._percentile_censored(lat, 0, 99) == 4.0
    assert serve._percentile_censored(lat, 1, 50) == 3.0
    assert serve._percentile_censored(lat, 1, 99) is None
    assert serve._percentile_censored(np.array([]), 0, 50) is None


@pytest.mark.parametrize("mode,solo", [("batched", True), ("batched", False), ("plain", True)])
def test_results_equal_single_source(mode, solo):
    gs = _graphs()
    ex = CpuExecutor([(g.offsets, g.indices) for g in gs])
    trace = serve.poisson_trace(400.0, 0.3, len(gs), _roots(gs), seed=1)
    srv = serve.Server(ex, memory_budget=1 << 30, solo_plain=solo)
    rep, res = srv.serve(trace, mode=mode, drain_s=30.0, keep_results=True)
    assert rep.completed == len(trace) and rep.unfinished == 0 and rep.failed == 0
    exp = _expected(gs, trace)
    for q in trace:
        assert np.array_equal(res[q.qid], exp[(q.gid, q.root)]), q
        assert q.t_done >= q.t_arrival
    assert rep.p50_ms is not None and rep.p99_ms >= rep.p50_ms
    if mode == "batched":
        assert (srv.solo_runs > 0) == solo


def test_memory_budget_bounds_inflight_and_slots_refill():
    gs = _graphs()
    ex = CpuExecutor([(g.offsets, g.indices) for g in gs])
    trace = serve.poisson_trace(3000.0, 0.2, len(gs), _roots(gs), seed=2)
    per_query = max(ex.output_bytes(i) for i in range(len(gs)))
    srv = serve.Server(ex, memory_budget=3 * per_query, slots=2)
    rep, res = srv.serve(trace, mode="batched", drain_s=60.0, keep_results=True)
    assert rep.completed == len(trace)
    assert rep.peak_memory <= 3 * per_query
    assert 0 < ex.max_inflight <= 3 * per_query
    exp = _expected(gs, trace)
    for q in trace:
        assert np.array_equal(res[q.qid], exp[(q.gid, q.root)])


def test_failure_injection_fails_only_the_session_queries():
    gs = _graphs()
    ex = CpuExecutor([(g.offsets, g.indices) for g in gs], fail_steps=(5,))
    trace = serve.poisson_trace(500.0, 0.3, len(gs), _roots(gs), seed=3)
    # plain runs only for a lone query, so that sessions carry most queries
    srv = serve.Server(ex, memory_budget=1 << 30, plain_max=1)
    rep, res = srv.serve(trace, mode="batched", drain_s=30.0, keep_results=True)
    assert rep.failed >= 1
    assert rep.completed + rep.failed == len(trace)
    assert srv.budget.used == 0
    exp = _expected(gs, trace)
    for q in trace:
        if q.error is None:
            assert np.array_equal(res[q.qid], exp[(q.gid, q.root)])
        else:
            assert "injected failure" in q.error


def test_alone_equals_in_the_mix():
    gs = _graphs()
    ex = CpuExecutor([(g.offsets, g.indices) for g in gs])
    trace = serve.poisson_trace(2000.0, 0.2, len(gs), _roots(gs), seed=4)
    srv = serve.Server(ex, memory_budget=1 << 30, solo_plain=False)  # every query through a session
    _, mixed = srv.serve(trace, mode="batched", drain_s=30.0, keep_results=True)
    for q in trace[:15]:
        alone_trace = [serve.Query(0, q.gid, q.root, 0.0)]
        _, alone = srv.serve(alone_trace, mode="batched", drain_s=30.0, keep_results=True)
        assert np.array_equal(alone[0], mixed[q.qid])


def test_drain_limit_leaves_queries_unfinished():
    class Slow(CpuExecutor):
        def run_plain(self, gid, root):
            import time
            time.sleep(0.05)
            return super().run_plain(gid, root)

    gs = _graphs()
    ex = Slow([(g.offsets, g.indices) for g in gs])
    trace = serve.poisson_trace(1000.0, 0.1, len(gs), _roots(gs), seed=5)
    srv = serve.Server(ex, memory_budget=1 << 30)
    rep, _ = srv.serve(trace, mode="plain", drain_s=0.2)
    assert rep.unfinished > 0 and rep.completed > 0
    assert rep.p99_ms is None  # the 99th percentile lies among the unfinished


@pytest.mark.parametrize("plain_max,expect_plain", [(1, 0), (3, 3), (8, 3), (0, 0)])
def test_plain_runs_below_the_session_threshold(plain_max, expect_plain):
    """Three queries arrive together on an idle graph: with plain_max >= 3
    they all run plain, one after another; below that they share a session.
    A lone later arrival runs plain whenever plain_max >= 1."""
    gs = _graphs()
    ex = CpuExecutor([(g.offsets, g.indices) for g in gs])
    trace = [serve.Query(0, 0, 3, 0.0), serve.Query(1, 0, 7, 0.0), serve.Query(2, 0, 11, 0.0),
             serve.Query(3, 0, 5, 0.2)]
    srv = serve.Server(ex, memory_budget=1 << 30, plain_max=plain_max)
    rep, res = srv.serve(trace, mode="batched", drain_s=30.0, keep_results=True)
    assert rep.completed == len(trace)
    exp = _expected(gs, trace)
    for q in trace:
        assert np.array_equal(res[q.qid], exp[(q.gid, q.root)])
    assert srv.solo_runs == expect_plain + (1 if plain_max >= 1 else 0)


def test_plain_max_must_not_be_negative():
    with pytest.raises(ValueError):
        serve.Server(CpuExecutor([]), memory_budget=1, plain_max=-1)
    with pytest.raises(ValueError):
        serve.Server(CpuExecutor([]), memory_budget=1, plain_concurrency=0)


def test_plain_runs_never_overlap_across_graphs():
    """With plain_concurrency 1 the graph workers' plain runs execute one
    at a time; results still equal the oracle's."""
    import threading

    class Counting(CpuExecutor):
        def __init__(self, graphs):
            super().__init__(graphs)
            self.lock = threading.Lock()
            self.now = 0
            self.peak = 0

        def run_plain(self, gid, root):
            import time
            with self.lock:
                self.now += 1
                self.peak = max(self.peak, self.now)
            time.sleep(0.002)
            try:
                return super().run_plain(gid, root)
            finally:
                with self.lock:
                    self.now -= 1

    gs = _graphs()
    ex = Counting([(g.offsets, g.indices) for g in gs])
    trace = serve.poisson_trace(300.0, 0.3, len(gs), _roots(gs), seed=7)
    srv = serve.Server(ex, memory_budget=1 << 30, plain_max=8, plain_concurrency=1)
    rep, res = srv.serve(trace, mode="batched", drain_s=30.0, keep_results=True)
    assert rep.completed == len(trace) and srv.solo_runs > 0
    assert ex.peak == 1
    exp = _expected(gs, trace)
    for q in trace:
        assert np.array_equal(res[q.qid], exp[(q.gid, q.root)])
