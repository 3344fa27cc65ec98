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
