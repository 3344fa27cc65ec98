"""The allocation-free entry point (dobfs_run_noalloc) against dobfs_run:
same depths bit for bit, valid parent trees, the same traversed-edge count,
on two calls in a row with the second on a smaller graph (the fixed scratch
array keeps the first call's contents), relabelled and not, with and without
a parent output; and the size limit is refused with a clear error."""
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


def _pair(dobfs, dg, g, root, want_parent, params=None):
    import torch
    d_ref, p_ref, st_ref = dg.run(root, want_parent=want_parent, stats=True, params=params)
    d_na, p_na, st_na = dg.run_noalloc(root, want_parent=want_parent, stats=True, params=params)
    torch.cuda.synchronize()
    d_ref, d_na = d_ref.cpu().numpy(), d_na.cpu().numpy()
    assert np.array_equal(d_na, d_ref), (root, want_parent)
    exp, _ = oracle.bfs(g.offsets, g.indices, root)
    assert np.array_equal(d_na, exp), root
    assert st_na.m_c == st_ref.m_c == oracle.traversed_edges(g.offsets, exp)
    assert st_na.levels == st_ref.levels and st_na.reached == st_ref.reached
    assert [r["found"] for r in st_na.log] == [r["found"] for r in st_ref.log]
    if want_parent:
        p = p_na.cpu().numpy()
        code, bad = oracle.check_tree(g.offsets, g.indices, root, d_na, p)
        assert code == 0, (oracle.CHECK_CODES[code], bad)
    else:
        assert p_na is None


@pytest.mark.parametrize("reindex", [False, True])
def test_noalloc_matches_run_two_calls_second_smaller(dobfs, reindex):
    big = gg.kronecker(17, seed=51)
    small = gg.kronecker(11, seed=52)
    with dobfs.Graph.upload(big.offsets, big.indices, reindex=reindex) as db, \
         dobfs.Graph.upload(small.offsets, small.indices, reindex=reindex) as ds:
        for want_parent in (True, False):
            rb = int(gg.sample_roots(big, 1, seed=53)[0])
            rs = int(gg.sample_roots(small, 1, seed=54)[0])
            _pair(dobfs, db, big, rb, want_parent)   # first call: the larger graph
            _pair(dobfs, ds, small, rs, want_parent)  # second call: smaller, scratch holds the first's state


def test_noalloc_policies_and_long_paths(dobfs):
    g = gg.kronecker(14, seed=55)
    path = gg.path(3000)
    with dobfs.Graph.upload(g.offsets, g.indices, reindex=True) as dg:
        r = int(gg.sample_roots(g, 1, seed=56)[0])
        for pol in ("edge", "td", "bu", "paper", "random"):
            _pair(dobfs, dg, g, r, True, params=dobfs.make_params(pol, seed=7))
    with dobfs.Graph.upload(path.offsets, path.indices) as dp:
        _pair(dobfs, dp, path, 1500, True, params=dobfs.make_params("edge", chunk_levels=16))


def test_noalloc_refuses_beyond_its_scratch(dobfs):
    g = gg.path(20_000_000)  # its queue alone needs 80 MB, more than the fixed array holds
    with dobfs.Graph.upload(g.offsets, g.indices) as dg:
        with pytest.raises(dobfs.DobfsError) as ei:
            dg.run_noalloc(0)
        assert ei.value.status == dobfs.ENOTSUP
        assert "scratch" in str(ei.value)
