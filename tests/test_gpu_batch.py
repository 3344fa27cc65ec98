"""Batched traversal (up to 64 roots in one pass): every slot's depths are
bit-exact to the oracle's single-source run from that root."""
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


def _check(dobfs, g, roots, params=None, reindex=False, label=""):
    import torch
    print(f"[batch] {label or g.name} n={g.n} k={len(roots)} reindex={reindex}", flush=True)
    with dobfs.Graph.upload(g.offsets, g.indices, reindex=reindex) as dg:
        depth, st = dg.batch(roots, params=params, stats=True)
        torch.cuda.synchronize()
        d = depth.cpu().numpy()
    mc = 0
    reached = 0
    for b, r in enumerate(roots):
        exp, _ = oracle.bfs(g.offsets, g.indices, int(r))
        assert np.array_equal(d[b], exp), (label, b, int(r), np.flatnonzero(d[b] != exp)[:8])
        mc += oracle.traversed_edges(g.offsets, exp)
        reached += int((exp >= 0).sum())
    assert st.m_c == mc and st.reached == reached
    return st


def test_batch_64_roots_kronecker(dobfs):
    g = gg.kronecker(14, seed=21)
    roots = gg.sample_roots(g, 64, seed=5)
    for pol in ("edge", "td", "bu"):
        _check(dobfs, g, roots, params=dobfs.make_params(pol), label=f"kron14/{pol}")
    for seed in (1, 2, 3):  # a random direction per slot and level: mixed push/pull levels
        _check(dobfs, g, roots, params=dobfs.make_params("random", seed=seed), label=f"kron14/random{seed}")


def test_batch_relabelled(dobfs):
    g = gg.kronecker(15, seed=22)
    roots = gg.sample_roots(g, 64, seed=6)
    for pol in ("edge", "bu"):
        _check(dobfs, g, roots, params=dobfs.make_params(pol), reindex=True, label=f"kron15/{pol}/reindex")
    _check(dobfs, g, roots, params=dobfs.make_params("random", seed=9), reindex=True, label="kron15/random/reindex")


def test_batch_small_k_duplicates_and_isolated(dobfs):
    g = gg.disjoint_union(gg.kronecker(10, seed=3), gg.path(40), gg.from_edges(2, [], []))
    iso = g.n - 1
    for roots in ([0], [5, 5, 5], [iso, 3, iso - 1, g.n - 10], list(range(17))):
        for reindex in (False, True):
            _check(dobfs, g, roots, reindex=reindex, label=f"union roots={roots[:4]}")


def test_batch_many_levels_and_heavy(dobfs):
    g = gg.chung_lu(20000, gamma=2.2, avg_deg=8.0, max_deg=2000.0, n_tails=4, tail_len=120, seed=9)
    roots = gg.sample_roots(g, 33, seed=2)
    _check(dobfs, g, roots, label="chung-lu+tails")
    _check(dobfs, g, roots, params=dobfs.make_params("random", seed=4), label="chung-lu+tails/random")
    g = gg.star(5000)
    _check(dobfs, g, [0, 1, 4999, 17], params=dobfs.make_params("bu", bu_heavy_cut=64), label="star/bu")
    _check(dobfs, g, [0, 1, 4999, 17], params=dobfs.make_params("td"), label="star/td")
    for seed in range(4):  # the hub is split in push and in pull levels
        _check(dobfs, g, [0, 1, 4999, 17, 2, 3], params=dobfs.make_params("random", seed=seed), label="star/random")


def test_batch_matches_single_runs(dobfs):
    import torch
    g = gg.kronecker(13, seed=8)
    roots = gg.sample_roots(g, 10, seed=1)
    with dobfs.Graph.upload(g.offsets, g.indices) as dg:
        depth, _ = dg.batch(roots)
        for b, r in enumerate(roots):
            d1, _, _ = dg.run(int(r))
            torch.cuda.synchronize()
            assert torch.equal(depth[b], d1)


def test_batch_errors(dobfs):
    g = gg.path(10)
    with dobfs.Graph.upload(g.offsets, g.indices) as dg:
        with pytest.raises(dobfs.DobfsError) as ei:
            dg.batch([0, 10])
        assert ei.value.status == dobfs.ERANGE
        with pytest.raises(dobfs.DobfsError) as ei:
            dg.batch(list(range(10)) * 7)  # 70 roots
        assert ei.value.status == dobfs.EINVAL
