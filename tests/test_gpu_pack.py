"""Packed small graphs and multi-root runs: each graph's slice of one
multi-root traversal is bit-exact to the oracle's run on that graph alone."""
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


def _graphs(seed=0, count=24):
    rng = np.random.default_rng(seed)
    out = [gg.path(30), gg.star(200), gg.from_edges(1, [], []), gg.disjoint_union(gg.cycle(7), gg.path(5))]
    while len(out) < count:
        out.append(gg.kronecker(int(rng.integers(4, 12)), seed=int(rng.integers(1, 10**6))))
    return out


def _check_pack(dobfs, graphs, roots, depth, parent, bases):
    for i, (g, r) in enumerate(zip(graphs, roots)):
        d = depth[bases[i]:bases[i + 1]]
        exp, _ = oracle.bfs(g.offsets, g.indices, int(r))
        assert np.array_equal(d, exp), (i, g.name, int(r))
        if parent is not None:
            p = parent[bases[i]:bases[i + 1]].astype(np.int64)
            p = np.where(p >= 0, p - bases[i], -1).astype(np.int32)
            code, bad = oracle.check_tree(g.offsets, g.indices, int(r), d, p)
            assert code == 0, (i, oracle.CHECK_CODES[code], bad)


@pytest.mark.parametrize("reindex", [False, True])
@pytest.mark.parametrize("policy", ["edge", "td", "bu"])
def test_pack_host_sources(dobfs, reindex, policy):
    import torch
    graphs = _graphs(1)
    roots = [int(gg.sample_roots(g, 1, seed=i)[0]) if g.m else 0 for i, g in enumerate(graphs)]
    print(f"[pack] host count={len(graphs)} reindex={reindex} policy={policy}", flush=True)
    with dobfs.Pack.upload([(g.offsets, g.indices) for g in graphs], reindex=reindex) as pk:
        assert pk.bases[-1] == sum(g.n for g in graphs)
        d, p, st = pk.run_pack(roots, params=dobfs.make_params(policy), want_parent=True, stats=True)
        torch.cuda.synchronize()
        _check_pack(dobfs, graphs, roots, d.cpu().numpy(), p.cpu().numpy(), pk.bases)
        mc = sum(oracle.traversed_edges(g.offsets, oracle.bfs(g.offsets, g.indices, r)[0])
                 for g, r in zip(graphs, roots))
        assert st.m_c == mc


def test_pack_device_sources(dobfs):
    import torch
    devs = [gg.kronecker_device(s, seed=100 + s) for s in (8, 10, 12, 10, 9)]
    hosts = [d.to_host() for d in devs]
    roots = [int(gg.sample_roots(h, 1, seed=3)[0]) for h in hosts]
    print("[pack] device sources", flush=True)
    with dobfs.Pack.upload(devs) as pk:
        d, _, _ = pk.run_pack(roots)
        torch.cuda.synchronize()
        _check_pack(dobfs, hosts, roots, d.cpu().numpy(), None, pk.bases)
    for dv in devs:
        dv.free()


def test_run_multi_nearest_root(dobfs):
    import torch
    g = gg.kronecker(12, seed=31)
    roots = gg.sample_roots(g, 7, seed=2)
    exp = None
    for r in roots:
        d, _ = oracle.bfs(g.offsets, g.indices, int(r))
        d = np.where(d < 0, np.iinfo(np.int32).max, d)
        exp = d if exp is None else np.minimum(exp, d)
    exp = np.where(exp == np.iinfo(np.int32).max, -1, exp)
    for reindex in (False, True):
        print(f"[multi] reindex={reindex}", flush=True)
        with dobfs.Graph.upload(g.offsets, g.indices, reindex=reindex) as dg:
            d, p, _ = dg.run_multi(np.concatenate([roots, roots[:2]]))
            torch.cuda.synchronize()
            d, p = d.cpu().numpy(), p.cpu().numpy()
            assert np.array_equal(d, exp)
            for r in roots:
                assert p[r] == r
            reached = np.flatnonzero(d > 0)
            for v in reached[:2000]:
                nb = g.indices[g.offsets[v]:g.offsets[v + 1]]
                assert p[v] in nb and d[p[v]] == d[v] - 1


def test_pack_errors(dobfs):
    graphs = [gg.path(5), gg.path(3)]
    with dobfs.Pack.upload([(g.offsets, g.indices) for g in graphs]) as pk:
        with pytest.raises(dobfs.DobfsError) as ei:
            pk.run_pack([0, 3])
        assert ei.value.status == dobfs.ERANGE
