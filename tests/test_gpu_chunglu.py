"""Chung-Lu power-law graph with path tails (the stand-in for a real-world
graph) at reduced size: hundreds of levels and several direction switches;
depths bit-exact to the oracle, parents valid, counters equal to the
oracle's replay."""
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


def test_chunglu_tails_many_levels_and_switches(dobfs):
    import torch
    g = gg.chung_lu(1_000_000, gamma=2.2, avg_deg=20.0, max_deg=1e5, n_tails=50, tail_len=200, seed=3)
    roots = list(gg.sample_roots(g, 3, seed=1_000_003))
    roots.append(g.n - 1)          # end of the last tail
    roots.append(1_000_000 + 100)  # middle of the first tail
    print(f"[chunglu] n={g.n} m={g.m} roots={roots}", flush=True)
    for reindex in (True, False):
        with dobfs.Graph.upload(g.offsets, g.indices, reindex=reindex) as dg:
            for r in roots:
                d, p, st = dg.run(int(r), stats=True)
                torch.cuda.synchronize()
                d, p = d.cpu().numpy(), p.cpu().numpy()
                exp, _ = oracle.bfs(g.offsets, g.indices, int(r))
                assert np.array_equal(d, exp), (reindex, r)
                code, bad = oracle.check_tree(g.offsets, g.indices, int(r), d, p)
                assert code == 0, (oracle.CHECK_CODES[code], bad)
                assert st.levels == int(exp.max()) + 1 >= 200
                dirs = st.dirs()
                assert sum(1 for a, b in zip(dirs, dirs[1:]) if a != b) >= 2, dirs
