"""Pins of the torch BFS-tree property checker used at full size: it
accepts the oracle's results and rejects planted mistakes."""
from __future__ import annotations

import numpy as np
import pytest

import graphgen as gg
import oracle
from tree_props import bfs_tree_violations


def _t(g, d, p):
    import torch
    return (torch.from_numpy(g.offsets.astype(np.int64)), torch.from_numpy(g.indices.astype(np.int32)),
            torch.from_numpy(d.astype(np.int32)), torch.from_numpy(p.astype(np.int32)))


GRAPHS = [
    gg.kronecker(10, seed=5),
    gg.chung_lu(3000, gamma=2.2, avg_deg=5.0, max_deg=300.0, n_tails=2, tail_len=50, seed=2),
    gg.disjoint_union(gg.cycle(9), gg.star(12), gg.from_edges(3, [], [])),
]


@pytest.mark.parametrize("gi", range(len(GRAPHS)))
@pytest.mark.parametrize("chunk", [7, 1000, 1 << 27])
def test_oracle_results_pass(gi, chunk):
    g = GRAPHS[gi]
    for r in (0, g.n // 2, g.n - 1):
        d, p = oracle.bfs(g.offsets, g.indices, r)
        assert bfs_tree_violations(*_t(g, d, p), r, chunk=chunk) == []


def test_planted_mistakes_are_caught():
    g = GRAPHS[0]
    root = int(gg.sample_roots(g, 1, seed=1)[0])
    d0, p0 = oracle.bfs(g.offsets, g.indices, root)
    deg = g.degrees()
    reached = np.flatnonzero((d0 > 1))
    v = int(reached[0])

    def check(d, p, expect):
        got = bfs_tree_violations(*_t(g, d, p), root, chunk=5000)
        assert expect in got, (expect, got)

    d, p = d0.copy(), p0.copy()
    d[root] = 1
    check(d, p, "root")
    d, p = d0.copy(), p0.copy()
    d[v] += 1  # too deep: some edge spans two levels or the parent is two levels up
    got = bfs_tree_violations(*_t(g, d, p), root, chunk=5000)
    assert "parent-depth" in got or "edge-span" in got
    d, p = d0.copy(), p0.copy()
    p[v] = -1
    check(d, p, "unreached-parent")
    # a parent one level up that is not a neighbour
    d, p = d0.copy(), p0.copy()
    nbrs = set(g.indices[g.offsets[v]:g.offsets[v + 1]].tolist())
    cand = [u for u in np.flatnonzero(d0 == d0[v] - 1) if int(u) not in nbrs]
    p[v] = int(cand[0])
    check(d, p, "parent-edge")
    # an unreached vertex claimed as reached (isolated vertices have degree 0)
    iso = np.flatnonzero(deg == 0)
    if iso.size:
        d, p = d0.copy(), p0.copy()
        d[iso[0]], p[iso[0]] = 1, root
        got = bfs_tree_violations(*_t(g, d, p), root, chunk=5000)
        assert "parent-edge" in got or "parent-depth" in got


def test_depth_first_tree_on_a_cycle_is_rejected():
    g = gg.cycle(10)
    n = g.n
    d = np.arange(n, dtype=np.int32)            # walk one way round
    p = np.concatenate([[0], np.arange(n - 1)]).astype(np.int32)
    got = bfs_tree_violations(*_t(g, d, p), 0)
    assert "edge-span" in got
    d2, p2 = oracle.bfs(g.offsets, g.indices, 0)
    assert bfs_tree_violations(*_t(g, d2, p2), 0) == []


def test_other_component_marked_reached_is_rejected():
    g = gg.disjoint_union(gg.path(5), gg.path(4))
    d, p = oracle.bfs(g.offsets, g.indices, 0)
    d = d.copy()
    p = p.copy()
    d[5:] = [1, 2, 3, 4]
    p[5:] = [0, 5, 6, 7]
    got = bfs_tree_violations(*_t(g, d, p), 0)
    assert "parent-edge" in got


# ---- depth-only checker (batched outputs) -----------------------------------

def _td(g, d):
    import torch
    return (torch.from_numpy(g.offsets.astype(np.int64)), torch.from_numpy(g.indices.astype(np.int32)),
            torch.from_numpy(d.astype(np.int32)))


@pytest.mark.parametrize("gi", range(len(GRAPHS)))
@pytest.mark.parametrize("chunk", [7, 1000, 1 << 27])
def test_depth_checker_accepts_oracle(gi, chunk):
    from tree_props import bfs_depth_violations
    g = GRAPHS[gi]
    for r in (0, g.n // 2, g.n - 1):
        d, _ = oracle.bfs(g.offsets, g.indices, r)
        assert bfs_depth_violations(*_td(g, d), r, chunk=chunk) == []


def test_depth_checker_rejects_planted_mistakes():
    from tree_props import bfs_depth_violations
    g = GRAPHS[0]
    root = int(gg.sample_roots(g, 1, seed=1)[0])
    d0, _ = oracle.bfs(g.offsets, g.indices, root)

    def check(d, expect):
        got = bfs_depth_violations(*_td(g, d), root, chunk=5000)
        assert expect in got, (expect, got)

    d = d0.copy(); d[root] = 1
    check(d, "root")
    far = int(np.flatnonzero(d0 == d0.max())[0])
    d = d0.copy(); d[far] += 1           # one level too deep: an edge spans 2
    check(d, "edge-span")
    d = d0.copy(); d[far] = -1           # a reached vertex left unreached
    check(d, "edge-reach")
    # a second depth-0 vertex and its whole component shifted one level
    # shallower: every edge still spans at most 1, but the fake root has no
    # neighbour of depth -1
    d = d0.copy()
    v = int(np.flatnonzero(d0 == 1)[0])
    d[v] = 0
    check(d, "no-parent")
    # all depths off by the same amount except the root: spans stay <= 1
    d = np.where(d0 > 0, d0 + 1, d0).astype(np.int32)
    check(d, "no-parent")


def test_depth_checker_on_path_fake_root():
    from tree_props import bfs_depth_violations
    g = gg.path(3)
    d = np.array([0, 0, 1], dtype=np.int32)  # vertex 1 claims depth 0 beside the root
    assert "no-parent" in bfs_depth_violations(*_td(g, d), 0)
