"""Pins of the oracle against facts that do not come from the oracle itself:
closed forms, the hand-worked fixture, boolean reachability powers on tiny
random graphs, scipy's unweighted shortest paths, and planted faults for the
tree checker.  CPU only."""
from __future__ import annotations

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components, shortest_path

import graphgen as gg
import oracle
from golden_io import read_handworked


def _check_ok(g, root, depth, parent):
    code, bad = oracle.check_tree(g.offsets, g.indices, root, depth, parent)
    assert code == 0, (oracle.CHECK_CODES[code], bad)


# --------------------------------------------------------------------------
# Closed forms.

@pytest.mark.parametrize("n", [1, 2, 7, 64, 65])
def test_path(n):
    g = gg.path(n)
    for r in {0, n // 2, n - 1}:
        d, p = oracle.bfs(g.offsets, g.indices, r)
        assert (d == np.abs(np.arange(n) - r)).all()
        _check_ok(g, r, d, p)


@pytest.mark.parametrize("n", [3, 4, 9, 100])
def test_cycle(n):
    g = gg.cycle(n)
    for r in (0, 1, n - 1):
        d, p = oracle.bfs(g.offsets, g.indices, r)
        k = np.abs(np.arange(n) - r)
        assert (d == np.minimum(k, n - k)).all()
        _check_ok(g, r, d, p)


def test_star():
    n = 50
    g = gg.star(n)
    d, p = oracle.bfs(g.offsets, g.indices, 0)
    assert d[0] == 0 and (d[1:] == 1).all() and (p[1:] == 0).all()
    d, p = oracle.bfs(g.offsets, g.indices, 7)
    exp = np.full(n, 2)
    exp[0], exp[7] = 1, 0
    assert (d == exp).all()
    assert p[0] == 7 and (p[np.arange(n) > 0] [np.arange(1, n) != 7] == 0).all()


def test_complete():
    g = gg.complete(33)
    d, p = oracle.bfs(g.offsets, g.indices, 5)
    exp = np.ones(33, dtype=np.int32)
    exp[5] = 0
    assert (d == exp).all()
    assert (p == 5).all()


def test_complete_bipartite():
    a, b = 5, 8
    g = gg.complete_bipartite(a, b)
    for r in (0, a + 2):
        d, p = oracle.bfs(g.offsets, g.indices, r)
        side = np.arange(a + b) >= a
        exp = np.where(side == side[r], 2, 1)
        exp[r] = 0
        assert (d == exp).all()
        _check_ok(g, r, d, p)


def test_grid():
    rows, cols = 9, 13
    g = gg.grid2d(rows, cols)
    r0, c0 = 4, 3
    d, p = oracle.bfs(g.offsets, g.indices, r0 * cols + c0)
    rr, cc = np.divmod(np.arange(rows * cols), cols)
    assert (d == np.abs(rr - r0) + np.abs(cc - c0)).all()
    _check_ok(g, r0 * cols + c0, d, p)


@pytest.mark.parametrize("dim", [1, 4, 7])
def test_hypercube(dim):
    g = gg.hypercube(dim)
    n = 1 << dim
    r = n // 3
    d, p = oracle.bfs(g.offsets, g.indices, r)
    pop = np.array([bin(i ^ r).count("1") for i in range(n)])
    assert (d == pop).all()
    _check_ok(g, r, d, p)


def test_binary_tree():
    n = 200
    g = gg.binary_tree(n)
    d, p = oracle.bfs(g.offsets, g.indices, 0)
    assert (d == np.floor(np.log2(np.arange(n) + 1)).astype(int)).all()
    assert (p[1:] == (np.arange(1, n) - 1) // 2).all()


def test_disjoint_union_and_isolated_root():
    g = gg.disjoint_union(gg.path(5), gg.cycle(6), gg.from_edges(1, [], []))
    d, p = oracle.bfs(g.offsets, g.indices, 2)
    assert list(d[:5]) == [2, 1, 0, 1, 2]
    assert (d[5:] == -1).all() and (p[5:] == -1).all()
    _check_ok(g, 2, d, p)
    iso = g.n - 1
    d, p = oracle.bfs(g.offsets, g.indices, iso)
    assert d[iso] == 0 and p[iso] == iso
    assert (np.delete(d, iso) == -1).all() and (np.delete(p, iso) == -1).all()
    _check_ok(g, iso, d, p)


def test_handworked_fixture():
    n, src, dst, cases = read_handworked("handworked_10.txt")
    g = gg.from_edges(n, src, dst)
    assert len(cases) == 4
    for root, exp in cases:
        d, p = oracle.bfs(g.offsets, g.indices, root)
        assert list(d) == exp, root
        _check_ok(g, root, d, p)
        dp, pp = oracle.bfs_py(g.offsets, g.indices, root)
        assert dp == exp


# --------------------------------------------------------------------------
# Brute force: boolean reachability powers on tiny random graphs, built
# straight from the raw edge list (no CSR involved).

def _reach_depth(n, src, dst, root):
    A = np.zeros((n, n), dtype=bool)
    A[src, dst] = True
    A[dst, src] = True
    np.fill_diagonal(A, False)
    depth = np.full(n, -1)
    R = np.zeros(n, dtype=bool)
    R[root] = True
    depth[root] = 0
    for k in range(1, n):
        R_next = R | (A[:, R].any(axis=1))
        new = R_next & ~R
        depth[new] = k
        if not new.any():
            break
        R = R_next
    return depth


def test_bruteforce_random_tiny_graphs():
    rng = np.random.default_rng(12345)
    for trial in range(400):
        n = int(rng.integers(1, 65))
        k = int(rng.integers(0, 3 * n + 1))
        src = rng.integers(0, n, size=k)
        dst = rng.integers(0, n, size=k)
        if trial % 5 == 0 and k:  # planted self-loops and duplicates
            src[: k // 3] = dst[: k // 3]
            src = np.concatenate([src, src[: k // 2]])
            dst = np.concatenate([dst, dst[: k // 2]])
        g = gg.from_edges(n, src, dst)
        for root in {0, n - 1, int(rng.integers(0, n))}:
            d, p = oracle.bfs(g.offsets, g.indices, root)
            assert (d == _reach_depth(n, src, dst, root)).all(), (trial, root)
            _check_ok(g, root, d, p)


def test_python_twin_matches():
    rng = np.random.default_rng(7)
    for _ in range(50):
        n = int(rng.integers(2, 120))
        k = int(rng.integers(0, 4 * n))
        g = gg.from_edges(n, rng.integers(0, n, k), rng.integers(0, n, k))
        r = int(rng.integers(0, n))
        d, p = oracle.bfs(g.offsets, g.indices, r)
        dp, pp = oracle.bfs_py(g.offsets, g.indices, r)
        assert list(d) == dp and list(p) == pp


# --------------------------------------------------------------------------
# Library routine: scipy's unweighted shortest paths.

def _scipy_depth(g, root):
    A = sp.csr_matrix((np.ones(g.m, dtype=np.int8), g.indices, g.offsets), shape=(g.n, g.n))
    dist = shortest_path(A, directed=False, unweighted=True, indices=root)
    return np.where(np.isinf(dist), -1, dist).astype(np.int64)


@pytest.mark.parametrize("scale", [10, 12, 14])
def test_scipy_kronecker(scale):
    g = gg.kronecker(scale, seed=scale)
    for r in gg.sample_roots(g, 3, seed=99):
        d, p = oracle.bfs(g.offsets, g.indices, int(r))
        assert (d == _scipy_depth(g, int(r))).all()
        _check_ok(g, int(r), d, p)


def test_scipy_chung_lu_with_tails():
    g = gg.chung_lu(20000, gamma=2.2, avg_deg=8.0, max_deg=2000.0, n_tails=4, tail_len=30, seed=5)
    r = int(gg.sample_roots(g, 1, seed=3)[0])
    d, p = oracle.bfs(g.offsets, g.indices, r)
    assert (d == _scipy_depth(g, r)).all()
    _check_ok(g, r, d, p)
    assert d.max() >= 30  # the tails stretch the traversal


# --------------------------------------------------------------------------
# Traversed-edge count: edges inside the root's connected component.

def test_traversed_edges_equals_component_edges():
    g = gg.kronecker(12, seed=4)
    A = sp.csr_matrix((np.ones(g.m), g.indices, g.offsets), shape=(g.n, g.n))
    _, lab = connected_components(A, directed=False)
    for r in gg.sample_roots(g, 4, seed=1):
        d, _ = oracle.bfs(g.offsets, g.indices, int(r))
        comp = lab == lab[int(r)]
        src = np.repeat(np.arange(g.n), g.degrees())
        inside = comp[src] & comp[g.indices]
        assert oracle.traversed_edges(g.offsets, d) == int(inside.sum()) // 2
        assert ((d >= 0) == comp).all()


# --------------------------------------------------------------------------
# The tree checker must reject planted faults.

@pytest.fixture(scope="module")
def kron11():
    g = gg.kronecker(11, seed=8)
    r = int(gg.sample_roots(g, 1, seed=2)[0])
    d, p = oracle.bfs(g.offsets, g.indices, r)
    return g, r, d, p


def _code(g, r, d, p):
    return oracle.check_tree(g.offsets, g.indices, r, d, p)


def test_checker_accepts_other_valid_parents(kron11):
    g, r, d, p = kron11
    p2 = p.copy()
    # any neighbour one level up is a valid parent
    changed = 0
    for v in range(g.n):
        if d[v] > 0:
            nb = g.indices[g.offsets[v]:g.offsets[v + 1]]
            ups = nb[d[nb] == d[v] - 1]
            if len(ups) > 1:
                p2[v] = ups[-1]
                changed += p2[v] != p[v]
    assert changed > 0
    assert _code(g, r, d, p2)[0] == 0


def test_checker_rejects_planted_faults(kron11):
    g, r, d, p = kron11
    reached = np.flatnonzero((d > 1))
    v = int(reached[0])
    # wrong root labels
    p1 = p.copy(); p1[r] = (r + 1) % g.n
    assert _code(g, r, d, p1)[0] == 1
    # depth off by one on one vertex
    d1 = d.copy(); d1[v] += 1
    assert _code(g, r, d1, p)[0] in (5, 6)
    # parent that is not a neighbour (same depth minus one, elsewhere)
    cands = np.flatnonzero(d == d[v] - 1)
    nb = set(g.indices[g.offsets[v]:g.offsets[v + 1]].tolist())
    far = [int(c) for c in cands if int(c) not in nb]
    p2 = p.copy(); p2[v] = far[0]
    assert _code(g, r, d, p2) == (4, v)
    # parent that is a neighbour at the wrong depth
    nbs = g.indices[g.offsets[v]:g.offsets[v + 1]]
    wrong = [int(u) for u in nbs if d[u] != d[v] - 1]
    if wrong:
        p3 = p.copy(); p3[v] = wrong[0]
        assert _code(g, r, d, p3) == (5, v)
    # a reached vertex reported as unreached
    d4, p4 = d.copy(), p.copy(); d4[v] = -1; p4[v] = -1
    assert _code(g, r, d4, p4)[0] in (5, 6)
    # unreached label mismatch
    unreached = np.flatnonzero(d == -1)
    if len(unreached):
        p5 = p.copy(); p5[unreached[0]] = r
        assert _code(g, r, d, p5)[0] == 3
    # out-of-range parent
    p6 = p.copy(); p6[v] = g.n
    assert _code(g, r, d, p6) == (2, v)


def test_checker_rejects_second_depth_zero_vertex():
    # I2 applies to every reached vertex other than the root, depth 0
    # included.  On path(3) from 0, labelling vertex 1 as a second root
    # (depth 0, its own parent) keeps every edge span <= 1.
    g = gg.path(3)
    d = np.array([0, 0, 1], dtype=np.int32)
    p = np.array([0, 1, 1], dtype=np.int32)
    assert oracle.check_tree(g.offsets, g.indices, 0, d, p) == (4, 1)
    # The same vertex given a real neighbour as parent: the parent-depth
    # test must still fail, since no vertex has depth -1 + 1 = 0 but the root.
    p = np.array([0, 0, 1], dtype=np.int32)
    assert oracle.check_tree(g.offsets, g.indices, 0, d, p) == (5, 1)
    # A subtree hung one level too shallow under that vertex: path(4).
    g = gg.path(4)
    d = np.array([0, 0, 1, 2], dtype=np.int32)
    p = np.array([0, 0, 1, 2], dtype=np.int32)
    assert oracle.check_tree(g.offsets, g.indices, 0, d, p) == (5, 1)


def test_checker_rejects_shallow_subtree_kronecker(kron11):
    # Kronecker scale 11: a depth-1 vertex v relabelled as depth 0 and its
    # whole BFS subtree (by the oracle's parents) moved one level up.
    g, r, d, p = kron11
    ones = np.flatnonzero(d == 1)
    children = {}
    for x in range(g.n):
        if d[x] > 0:
            children.setdefault(int(p[x]), []).append(x)
    v = max(ones.tolist(), key=lambda x: len(children.get(int(x), [])))
    d2 = d.copy()
    stack = [int(v)]
    while stack:
        x = stack.pop()
        d2[x] -= 1
        stack.extend(children.get(x, []))
    code, bad = oracle.check_tree(g.offsets, g.indices, r, d2, p)
    assert code != 0
    # and the fake root alone, with the rest of its subtree untouched
    d3 = d.copy(); d3[v] = 0
    code, bad = oracle.check_tree(g.offsets, g.indices, r, d3, p)
    assert code != 0
    if bad == v:
        assert code == 5


def test_checker_rejects_dfs_tree_on_cycle():
    # A depth-first tree satisfies the parent properties but not the edge
    # span: depth i along the cycle from 0.
    n = 12
    g = gg.cycle(n)
    d = np.arange(n, dtype=np.int32)
    p = np.concatenate([[0], np.arange(n - 1)]).astype(np.int32)
    code, bad = oracle.check_tree(g.offsets, g.indices, 0, d, p)
    assert code == 6


# --------------------------------------------------------------------------
# Replay work counts: closed forms and a direct recount.

def test_replay_path_closed_form():
    n = 10
    g = gg.path(n)
    d, _ = oracle.bfs(g.offsets, g.indices, 0)
    levels = n - 1
    out = oracle.replay(g.offsets, g.indices, d, [1] * levels)
    for L in range(levels):
        n_f, m_f, scanned, checked, found, found_deg, unv = out[L]
        assert n_f == 1 and m_f == (1 if L == 0 else 2)
        assert scanned == n - 1 - L
        # vertex L+1 hits its first neighbour L; the others check all of theirs
        exp = 1 + 2 * max(0, n - L - 3) + (1 if L + 2 <= n - 1 else 0)
        assert checked == exp, (L, checked, exp)
        assert found == 1
    out_td = oracle.replay(g.offsets, g.indices, d, [0] * levels)
    assert (out_td[:, 3] == out_td[:, 1]).all() and (out_td[:, 2] == 0).all()


def test_replay_complete_and_star():
    g = gg.complete(20)
    d, _ = oracle.bfs(g.offsets, g.indices, 0)
    out = oracle.replay(g.offsets, g.indices, d, [1])
    assert tuple(out[0, :6]) == (1, 19, 19, 19, 19, 19 * 19)
    g = gg.star(30)
    d, _ = oracle.bfs(g.offsets, g.indices, 3)
    out = oracle.replay(g.offsets, g.indices, d, [1, 1])
    # level 0: all 29 others scanned; the center hits leaf 3 at position 3,
    # leaves check their single edge
    assert tuple(out[0, :5]) == (1, 1, 29, 3 + 28, 1)
    assert tuple(out[1, :5]) == (1, 29, 28, 28, 28)


def test_replay_invariants_kronecker():
    g = gg.kronecker(12, seed=6)
    r = int(gg.sample_roots(g, 1, seed=5)[0])
    d, _ = oracle.bfs(g.offsets, g.indices, r)
    levels = int(d.max()) + 1
    rng = np.random.default_rng(0)
    dirs = rng.integers(0, 2, levels)
    out = oracle.replay(g.offsets, g.indices, d, dirs)
    deg = g.degrees()
    assert out[:, 0].sum() == (d >= 0).sum()
    assert out[:, 1].sum() == deg[d >= 0].sum() == 2 * oracle.traversed_edges(g.offsets, d)
    assert (out[:-1, 4] == out[1:, 0]).all() and out[-1, 4] == 0
    # unvisited degree after level L: total minus everything reached so far
    reached_deg = np.cumsum(out[:, 1]) + out[:, 5]
    assert (out[:, 6] == deg.sum() - reached_deg).all()
    # direct recount of the bottom-up columns
    for L in range(levels):
        if dirs[L] != 1:
            continue
        scanned = checked = 0
        for v in range(g.n):
            if (d[v] == -1 or d[v] > L) and deg[v] > 0:
                scanned += 1
                nb = g.indices[g.offsets[v]:g.offsets[v + 1]]
                hit = np.flatnonzero(d[nb] == L)
                checked += int(hit[0]) + 1 if len(hit) else int(deg[v])
        assert (out[L, 2], out[L, 3]) == (scanned, checked)
