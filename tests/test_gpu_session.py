"""Continuous batching: queries that join a running 64-slot traversal at
different levels, share it with others and leave when done.  Each result must
equal the oracle's single-source depths from its root, whoever else shared
the session, and equal what the same query gives alone."""
from __future__ import annotations

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dobfs():
    import __graft_entry__
    __graft_entry__.ensure_built()
    import torch
    torch.cuda.set_device(0)
    import paper_1503_04359_amd as lib
    return lib


def _serve(sess, roots, per_step, max_steps=100000):
    """Admit `per_step` queries before each step (as slots allow) until all
    have ended; returns {tag: depth numpy}."""
    import torch
    from paper_1503_04359_amd import EBUSY, DobfsError
    results, nxt, steps = {}, 0, 0
    while len(results) < len(roots):
        admitted = 0
        while nxt < len(roots) and admitted < per_step:
            try:
                sess.admit(int(roots[nxt]), tag=nxt)
            except DobfsError as e:
                assert e.status == EBUSY
                break
            nxt += 1
            admitted += 1
        for tag, d in sess.step():
            torch.cuda.synchronize()
            results[tag] = d.cpu().numpy()
        steps += 1
        assert steps < max_steps
    return results


def _expect(g, roots):
    cache = {}
    for r in set(int(x) for x in roots):
        cache[r] = oracle.bfs(g.offsets, g.indices, r)[0]
    return cache


@pytest.mark.parametrize("reindex", [False, True])
def test_session_staggered_queries_kronecker(dobfs, reindex):
    g = gg.kronecker(13, seed=31)
    roots = gg.sample_roots(g, 150, seed=7)  # more queries than slots: slots are reused
    print(f"[session] kron13 150 queries reindex={reindex}", flush=True)
    exp = _expect(g, roots)
    with dobfs.Graph.upload(g.offsets, g.indices, reindex=reindex) as dg:
        with dg.session(params=dobfs.make_params("edge", chunk_levels=2)) as s:
            res = _serve(s, roots, per_step=5)
    for t, r in enumerate(roots):
        assert np.array_equal(res[t], exp[int(r)]), (t, int(r))


@pytest.mark.parametrize("policy", ["td", "bu", "edge", "random"])
def test_session_long_paths_and_isolated(dobfs, policy):
    """Queries on a graph with long tails, a separate component and isolated
    vertices; some roots isolated.  One level per chunk so queries join at
    many different levels."""
    base = gg.chung_lu(6000, gamma=2.2, avg_deg=6.0, max_deg=600.0, n_tails=3, tail_len=90, seed=4)
    g = gg.disjoint_union(base, gg.path(70), gg.from_edges(3, [], []))
    rng = np.random.default_rng(11)
    roots = rng.integers(0, g.n, size=90)
    roots[::9] = g.n - 1  # an isolated vertex
    roots[1::13] = base.n + 5  # inside the path component
    print(f"[session] chung-lu+path+isolated policy={policy}", flush=True)
    exp = _expect(g, roots)
    for reindex in (False, True):
        with dobfs.Graph.upload(g.offsets, g.indices, reindex=reindex) as dg:
            with dg.session(params=dobfs.make_params(policy, chunk_levels=1)) as s:
                res = _serve(s, roots, per_step=3)
        for t, r in enumerate(roots):
            assert np.array_equal(res[t], exp[int(r)]), (policy, reindex, t, int(r))


def test_session_alone_equals_in_mix(dobfs):
    import torch
    g = gg.kronecker(12, seed=41)
    roots = gg.sample_roots(g, 70, seed=3)
    probe = int(roots[17])
    with dobfs.Graph.upload(g.offsets, g.indices) as dg:
        with dg.session() as s:
            alone = _serve(s, [probe], per_step=1)[0]
        with dg.session(params=dobfs.make_params("edge", chunk_levels=1)) as s:
            mixed = _serve(s, roots, per_step=64)
        d1, _, _ = dg.run(probe)
        torch.cuda.synchronize()
    assert np.array_equal(alone, mixed[17])
    assert np.array_equal(alone, d1.cpu().numpy())
    assert np.array_equal(alone, oracle.bfs(g.offsets, g.indices, probe)[0])


def test_session_limits_and_errors(dobfs):
    from paper_1503_04359_amd import DobfsError
    g = gg.path(50)
    with dobfs.Graph.upload(g.offsets, g.indices) as dg:
        s = dg.session()
        outs = [s.admit(i % 50, tag=i) for i in range(64)]
        with pytest.raises(DobfsError) as ei:
            s.admit(0, tag=99)
        assert ei.value.status == dobfs.EBUSY
        with pytest.raises(DobfsError) as ei:
            s.admit(50, tag=100)
        assert ei.value.status in (dobfs.ERANGE, dobfs.EBUSY)
        with pytest.raises(DobfsError) as ei:
            dg.free()  # a session is open
        assert ei.value.status == dobfs.EBUSY
        done = {}
        while len(done) < 64:
            for t, d in s.step():
                done[t] = d.cpu().numpy()
        for i in range(64):
            assert np.array_equal(done[i], np.abs(np.arange(50) - (i % 50)).astype(np.int32))
        assert s.counts()[:2] == (0, 0)
        assert s.step() == []  # idle
        with pytest.raises(DobfsError) as ei:
            s.admit(-1, tag=1)
        assert ei.value.status == dobfs.ERANGE
        s.close()
        assert len(outs) == 64
