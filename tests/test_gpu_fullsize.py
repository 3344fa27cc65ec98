"""Full-size parity in the bench's configuration: Kronecker scale 30
(edgefactor 16, seed 2), roots drawn as the bench draws them, default
parameters and launch configuration.  The oracle cannot traverse 34 billion
entries in a test, so the results are checked by the BFS-tree properties
(tests/tree_props.py), which hold exactly when depths are the hop distances
and parents form a BFS tree; the device counters are checked against the
component's edge count."""
from __future__ import annotations

import sys

import pytest

import graphgen as gg
from tree_props import bfs_tree_violations

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

SCALE, SEED = 30, 2


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dobfs():
    import __graft_entry__
    __graft_entry__.ensure_built()
    import torch
    torch.cuda.set_device(0)
    import paper_1503_04359_amd as lib
    return lib


def _check(off, idx, depth, parent, root, st):
    import torch
    bad = bfs_tree_violations(off, idx, depth, parent, root)
    assert bad == [], (root, bad)
    deg = off[1:] - off[:-1]
    m_c = int(deg[depth >= 0].sum()) // 2
    assert st.m_c == m_c and st.reached == int((depth >= 0).sum())
    torch.cuda.synchronize()


def test_scale30_relabelled_and_borrowed(dobfs):
    import torch
    g = gg.kronecker_device(SCALE, 16, seed=SEED)
    roots = [int(r) for r in gg.sample_roots_device(g, 16, seed=SEED + 1_000_000)]
    _say(f"[fullsize] kronecker {SCALE} built: n={g.n} m={g.m}; roots {roots[:6]}")
    picks = [roots[0], roots[3], roots[5]]
    # relabelled: the library keeps its own copy, so the caller CSR is freed
    dg = dobfs.Graph.from_device_pointers(g.offsets_ptr, g.indices_ptr, g.n, g.m, borrow=False, reindex=True)
    g.free()
    outs = []
    for r in picks:
        d, p, st = dg.run(r, stats=True)
        torch.cuda.synchronize()
        outs.append((r, d, p, st))
        _say(f"[fullsize] relabelled run from {r}: levels {st.levels} reached {st.reached}")
    dg.free()
    g = gg.kronecker_device(SCALE, 16, seed=SEED)
    off, idx = g.offsets_tensor(), g.indices_tensor()
    for r, d, p, st in outs:
        _check(off, idx, d, p, r, st)
        _say(f"[fullsize] relabelled run from {r}: tree properties hold")
    del outs
    # borrowed in place, no relabelling
    dg = dobfs.Graph.from_device_pointers(g.offsets_ptr, g.indices_ptr, g.n, g.m, borrow=True)
    r = roots[1]
    d, p, st = dg.run(r, stats=True)
    torch.cuda.synchronize()
    _check(off, idx, d, p, r, st)
    _say(f"[fullsize] borrowed run from {r}: tree properties hold")
    dg.free()
    g.free()
