"""Traversals run as captured HIP graphs (dobfs_batch_submit and
dobfs_pack_run by default, dobfs_run with DOBFS_RUN_GRAPH) equal the same
traversals launched one kernel at a time: every replay of a cached graph,
with other eager work and synchronisations between replays, after a change
of arguments (a new capture), and when a traversal needs more levels than
the graph holds (ordinary launches continue it)."""
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


def _eager(dobfs, **kw):
    return dobfs.make_params("edge", flags=dobfs.RUN_EAGER, **kw)


@pytest.mark.parametrize("reindex", [True, False])
def test_batch_graph_replays_equal_eager(dobfs, reindex):
    import torch
    g = gg.kronecker(14, seed=61)
    roots_a = [int(r) for r in gg.sample_roots(g, 64, seed=62)]
    roots_b = [int(r) for r in gg.sample_roots(g, 20, seed=63)]
    with dobfs.Graph.upload(g.offsets, g.indices, reindex=reindex) as dg:
        ref_a, _ = dg.batch(roots_a, params=_eager(dobfs))
        ref_b, _ = dg.batch(roots_b, params=_eager(dobfs))
        torch.cuda.synchronize()
        ref_a, ref_b = ref_a.cpu(), ref_b.cpu()
        out = torch.empty((64, g.n), dtype=torch.int32, device="cuda")
        for rep in range(3):
            dg.batch(roots_a, depth=out)  # the same arguments: the cached graph is replayed
            torch.cuda.synchronize()
            assert torch.equal(out.cpu(), ref_a), rep
            d, _, _ = dg.run(roots_b[rep], want_parent=False)  # eager work between replays
            torch.cuda.synchronize()
        got_b, st = dg.batch(roots_b, stats=True)  # new arguments: a new capture
        torch.cuda.synchronize()
        assert torch.equal(got_b.cpu(), ref_b)
        dg.batch(roots_a, depth=out)
        torch.cuda.synchronize()
        assert torch.equal(out.cpu(), ref_a)
    for b in (0, 13, 63):
        exp, _ = oracle.bfs(g.offsets, g.indices, roots_a[b])
        assert np.array_equal(ref_a[b].numpy(), exp)


def test_batch_graph_more_levels_than_captured(dobfs):
    import torch
    # a Kronecker core with a 60-vertex path hung off it: more levels than the
    # 16 slots of the captured run
    core = gg.kronecker(10, seed=64)
    n0 = core.n
    src = np.repeat(np.arange(n0), np.diff(core.offsets))
    dst = core.indices.astype(np.int64)
    anchor = int(gg.sample_roots(core, 1, seed=65)[0])
    tail = np.arange(n0, n0 + 60)
    src = np.concatenate([src, [anchor], tail[:-1]])
    dst = np.concatenate([dst, [tail[0]], tail[1:]])
    g = gg.from_edges(n0 + 60, src, dst)
    roots = [int(r) for r in gg.sample_roots(g, 16, seed=66)] + [n0 + 59]
    with dobfs.Graph.upload(g.offsets, g.indices, reindex=True) as dg:
        ref, _ = dg.batch(roots, params=_eager(dobfs))
        for _ in range(2):
            got, st = dg.batch(roots, stats=True)
            torch.cuda.synchronize()
            assert torch.equal(got.cpu(), ref.cpu())
            assert st.levels > 16
    exp, _ = oracle.bfs(g.offsets, g.indices, roots[-1])
    assert np.array_equal(ref[-1].cpu().numpy(), exp)


def test_pack_graph_replays_equal_eager(dobfs):
    import torch
    gs = [gg.kronecker(s, seed=70 + i) for i, s in enumerate((10, 12, 11, 13, 10))] + [gg.path(40)]
    roots = [int(gg.sample_roots(g, 1, seed=80 + i)[0]) for i, g in enumerate(gs)]
    with dobfs.Pack.upload([(g.offsets, g.indices) for g in gs], reindex=True) as pk:
        ref, _, _ = pk.run_pack(roots, params=_eager(dobfs))
        torch.cuda.synchronize()
        ref = ref.cpu()
        out = torch.empty(pk.n, dtype=torch.int32, device="cuda")
        for rep in range(3):
            pk.run_pack(roots, depth=out)
            torch.cuda.synchronize()
            assert torch.equal(out.cpu(), ref), rep
        for i, g in enumerate(gs):
            exp, _ = oracle.bfs(g.offsets, g.indices, roots[i])
            assert np.array_equal(ref[int(pk.bases[i]):int(pk.bases[i + 1])].numpy(), exp), i


@pytest.mark.parametrize("reindex", [True, False])
def test_single_source_graph_on_request(dobfs, reindex):
    import torch
    g = gg.kronecker(14, seed=90)
    path = gg.path(300)
    prm = dobfs.make_params("edge", flags=dobfs.RUN_GRAPH)
    for graph, roots in ((g, [int(r) for r in gg.sample_roots(g, 3, seed=91)]), (path, [0, 150])):
        with dobfs.Graph.upload(graph.offsets, graph.indices, reindex=reindex) as dg:
            depth = torch.empty(graph.n, dtype=torch.int32, device="cuda")
            parent = torch.empty(graph.n, dtype=torch.int32, device="cuda")
            for r in roots:
                exp, _ = oracle.bfs(graph.offsets, graph.indices, r)
                for _ in range(2):  # capture, then replay
                    _, _, st = dg.run(r, depth, parent, params=prm, stats=True)
                    torch.cuda.synchronize()
                    d, p = depth.cpu().numpy(), parent.cpu().numpy()
                    assert np.array_equal(d, exp), r
                    code, bad = oracle.check_tree(graph.offsets, graph.indices, r, d, p)
                    assert code == 0, (oracle.CHECK_CODES[code], bad)
                    assert st.m_c == oracle.traversed_edges(graph.offsets, exp)


def test_graph_flag_errors(dobfs):
    g = gg.kronecker(8, seed=1)
    with dobfs.Graph.upload(g.offsets, g.indices) as dg:
        for flags in (dobfs.RUN_GRAPH | dobfs.RUN_EAGER, dobfs.RUN_GRAPH | dobfs.RUN_TIME_KERNELS):
            with pytest.raises(dobfs.DobfsError) as ei:
                dg.run(0, params=dobfs.make_params("edge", flags=flags))
            assert ei.value.status == dobfs.EINVAL
        with pytest.raises(dobfs.DobfsError) as ei:
            dg.run_noalloc(0, params=dobfs.make_params("edge", flags=dobfs.RUN_GRAPH))
        assert ei.value.status == dobfs.EINVAL
