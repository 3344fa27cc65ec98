"""Parity of the hybrid host + GPU traversal (specialized partitioning:
hub rows on the host, the rest on the device) with the oracle.  Depths are
compared bit-exact, parents by the BFS-tree properties, and every level's
counters with the oracle's replay of the same direction schedule on the
degree-relabelled graph (both partitions scan rows in internal-ID order,
so the bottom-up first-hit counts are unique).  The split is swept from
"every row on the host" to "every row on the device"."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import graphgen as gg
import oracle
from test_gpu_parity import degree_relabel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dobfs():
    import __graft_entry__
    __graft_entry__.ensure_built()
    import torch
    torch.cuda.set_device(0)
    import paper_1503_04359_amd as lib
    return lib


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _budgets(dobfs, g, fracs=(0.0, 0.3, 0.7, 1.0)):
    """Device budgets that leave the given fraction of the CSR entries'
    bytes on the device, beyond the per-vertex state."""
    base = dobfs.hybrid_state_bytes(g.n)
    return [base + int(f * 4 * g.m) for f in fracs]


def _parity(dobfs, g, roots, budgets, policies=("edge",), label="", threads=8):
    r_off, r_idx, new2old, _ = degree_relabel(g)
    for budget in budgets:
        with dobfs.HybridGraph.upload(g.offsets, g.indices, gpu_budget_bytes=budget, threads=threads) as hg:
            info = hg.info()
            assert info["host_entries"] + info["gpu_entries"] == g.m
            for pol in policies:
                params = dobfs.make_params(pol)
                for r in roots:
                    r = int(r)
                    _say(f"[hybrid] {label or g.name} n={g.n} m={g.m} budget={budget} split={info['split']} "
                         f"policy={pol} root={r}")
                    exp, _ = oracle.bfs(g.offsets, g.indices, r)
                    d, p, st = hg.run(r, params=params, stats=True)
                    d, p = d.cpu().numpy(), p.cpu().numpy()
                    assert np.array_equal(d, exp), (label, budget, pol, r, np.flatnonzero(d != exp)[:10])
                    code, bad = oracle.check_tree(g.offsets, g.indices, r, d, p)
                    assert code == 0, (oracle.CHECK_CODES[code], bad)
                    assert st.reached == int((exp >= 0).sum())
                    assert st.m_c == oracle.traversed_edges(g.offsets, exp)
                    assert st.levels == int(exp.max()) + 1
                    assert len(st.log) == st.levels
                    rep = oracle.replay(r_off, r_idx, exp[new2old], st.dirs())
                    got = np.array([[rec["n_f"], rec["m_f"], rec["scanned"], rec["checked"], rec["found"],
                                     rec["found_deg"]] for rec in st.log])
                    assert np.array_equal(got, rep[:, :6]), (label, budget, pol, r, got, rep[:, :6])


def test_hybrid_split_extremes_and_middle(dobfs):
    g = gg.kronecker(14, seed=21)
    roots = gg.sample_roots(g, 3, seed=5)
    budgets = _budgets(dobfs, g, (0.0, 0.15, 0.5, 0.85, 1.0))
    splits = []
    for b in budgets:
        with dobfs.HybridGraph.upload(g.offsets, g.indices, gpu_budget_bytes=b) as hg:
            splits.append(hg.info()["split"])
    # the host's share shrinks as the budget grows, from every vertex with a
    # row to none
    assert splits == sorted(splits, reverse=True)
    assert splits[0] >= int((g.degrees() > 0).sum()) and splits[-1] == 0
    assert all(s % 64 == 0 or s == g.n for s in splits)
    _parity(dobfs, g, roots, budgets, policies=("edge", "td", "bu", "paper", "cost"), label="kron14")


def test_hybrid_closed_forms(dobfs):
    cases = [gg.path(1), gg.path(2), gg.path(97), gg.cycle(130), gg.star(300), gg.complete(40),
             gg.complete_bipartite(3, 70), gg.grid2d(17, 23), gg.hypercube(9), gg.binary_tree(1000),
             gg.disjoint_union(gg.path(70), gg.cycle(9), gg.from_edges(2, [], []))]
    for g in cases:
        roots = sorted({0, g.n // 2, g.n - 1})
        _parity(dobfs, g, roots, _budgets(dobfs, g, (0.0, 0.5, 1.0)), policies=("edge", "td", "bu"),
                label=g.name)


def test_hybrid_long_device_rows(dobfs):
    """Rows longer than 2,048 entries on the device (the whole budget, or
    half of it) go through the grid-wide top-down expansion: a star whose
    centre has 19,999 neighbours, and Kronecker scale 16 with every row on
    the device."""
    g = gg.star(20000)
    _parity(dobfs, g, [0, 1, 19999], _budgets(dobfs, g, (0.0, 0.5, 1.0)), policies=("td", "edge", "bu"),
            label="star20000")
    g = gg.kronecker(16, seed=13)
    assert int(g.degrees().max()) > 2048
    _parity(dobfs, g, gg.sample_roots(g, 3, seed=2), _budgets(dobfs, g, (1.0,)), policies=("td", "edge"),
            label="kron16/all-device")


def test_hybrid_many_levels_and_tails(dobfs):
    g = gg.chung_lu(30000, gamma=2.2, avg_deg=8.0, max_deg=3000.0, n_tails=5, tail_len=150, seed=3)
    roots = gg.sample_roots(g, 2, seed=4)
    _parity(dobfs, g, roots, _budgets(dobfs, g, (0.2, 0.6)), policies=("edge", "paper"), label="chung-lu+tails")


def test_hybrid_kronecker_s18_threads(dobfs):
    """Scale 18 with the hubs' rows (about half the entries) on the host,
    with one host thread and with sixteen."""
    g = gg.kronecker(18, seed=2)
    roots = gg.sample_roots(g, 3, seed=11)
    _parity(dobfs, g, roots, _budgets(dobfs, g, (0.5,)), label="kron18/t1", threads=1)
    _parity(dobfs, g, roots, _budgets(dobfs, g, (0.5,)), label="kron18/t16", threads=16)


def test_hybrid_direction_schedule_matches_resident(dobfs):
    """Both partitions' counts summed give the resident traversal's
    direction schedule for the same relabelled graph."""
    import torch
    g = gg.kronecker(16, seed=4)
    roots = gg.sample_roots(g, 4, seed=8)
    with dobfs.Graph.upload(g.offsets, g.indices, reindex=True) as dg, \
            dobfs.HybridGraph.upload(g.offsets, g.indices,
                                     gpu_budget_bytes=_budgets(dobfs, g, (0.4,))[0]) as hg:
        for pol in ("edge", "paper", "cost"):
            params = dobfs.make_params(pol)
            for r in roots:
                _, _, st_res = dg.run(int(r), params=params, stats=True)
                torch.cuda.synchronize()
                _, _, st_hyb = hg.run(int(r), params=params, stats=True, want_parent=False)
                assert st_hyb.dirs() == st_res.dirs(), (pol, int(r))
                for a, b in zip(st_hyb.log, st_res.log):
                    for k in ("n_f", "m_f", "m_u", "found", "found_deg"):
                        assert a[k] == b[k], (pol, int(r), a["level"], k)


def test_hybrid_repeat_and_errors(dobfs):
    g = gg.kronecker(12, seed=6)
    r = int(gg.sample_roots(g, 1, seed=2)[0])
    exp, _ = oracle.bfs(g.offsets, g.indices, r)
    with dobfs.HybridGraph.upload(g.offsets, g.indices, gpu_budget_bytes=_budgets(dobfs, g, (0.5,))[0]) as hg:
        for _ in range(3):
            d, p, _ = hg.run(r)
            assert np.array_equal(d.cpu().numpy(), exp)
        d, p, _ = hg.run(r, want_parent=False)
        assert p is None and np.array_equal(d.cpu().numpy(), exp)
        with pytest.raises(dobfs.DobfsError) as ei:
            hg.run(g.n)
        assert ei.value.status == dobfs.ERANGE
        with pytest.raises(dobfs.DobfsError) as ei:
            hg.run(r, params=dobfs.make_params("random"))
        assert ei.value.status == dobfs.ENOTSUP
        with pytest.raises(dobfs.DobfsError) as ei:
            hg.run(r, params=dobfs.make_params("edge", beta=0))
        assert ei.value.status == dobfs.EINVAL
    with pytest.raises(dobfs.DobfsError) as ei:
        dobfs.HybridGraph.upload(g.offsets, g.indices, gpu_budget_bytes=dobfs.hybrid_state_bytes(g.n) - 1)
    assert ei.value.status == dobfs.EINVAL
    bad = g.indices.copy()
    bad[3] = -1
    with pytest.raises(dobfs.DobfsError) as ei:
        dobfs.HybridGraph.upload(g.offsets, bad, gpu_budget_bytes=1 << 30)
    assert ei.value.status == dobfs.EINVAL


def test_hybrid_hub_partition_decides(dobfs):
    """With DOBFS_RUN_HUB_DECIDES the PAPER rule's top-down -> bottom-up test
    sees only the host partition's next frontier; the schedule expected from
    the oracle's depths and the split is recomputed here."""
    g = gg.kronecker(16, seed=9)
    roots = gg.sample_roots(g, 4, seed=3)
    _, _, new2old, old2new = degree_relabel(g)
    deg = g.degrees().astype(np.int64)
    budget = _budgets(dobfs, g, (0.4,))[0]
    with dobfs.HybridGraph.upload(g.offsets, g.indices, gpu_budget_bytes=budget) as hg:
        split = hg.info()["split"]
        assert 0 < split < g.n
        host = old2new < split
        for pct, div, steps in ((10, 64, 3), (1, 16, 2), (50, 256, 5)):
            params = dobfs.make_params("paper", paper_pct=pct, paper_div=div, paper_bu_steps=steps,
                                       flags=dobfs.RUN_HUB_DECIDES)
            for r in roots:
                r = int(r)
                exp, _ = oracle.bfs(g.offsets, g.indices, r)
                d, p, st = hg.run(r, params=params, stats=True)
                d, p = d.cpu().numpy(), p.cpu().numpy()
                assert np.array_equal(d, exp)
                assert oracle.check_tree(g.offsets, g.indices, r, d, p)[0] == 0
                want, cur, phases, run = [], 0, 0, 0
                for L in range(int(exp.max()) + 1):
                    want.append(cur)
                    run = run + 1 if cur == 1 else 0
                    m_host = int(deg[(exp == L + 1) & host].sum())
                    if cur == 0:
                        nxt = 1 if (phases == 0 and m_host * pct > (g.n // div) * 100) else 0
                    else:
                        nxt = 0 if run >= steps else 1
                    if cur == 0 and nxt == 1:
                        phases += 1
                    cur = nxt
                assert st.dirs() == want, (pct, div, steps, r, st.dirs(), want)
    with dobfs.HybridGraph.upload(g.offsets, g.indices, gpu_budget_bytes=budget) as hg:
        with pytest.raises(dobfs.DobfsError) as ei:
            hg.run(int(roots[0]), params=dobfs.make_params("edge", flags=dobfs.RUN_HUB_DECIDES))
        assert ei.value.status == dobfs.EINVAL


def test_hybrid_scale24_bench_shape(dobfs):
    """The hybrid bench's shape at Kronecker scale 24: the rows of the top
    12% of non-isolated vertices on the host, 16 host threads, EDGE with
    alpha 56.  Every one of the bench's 16 roots: depths equal to the
    resident traversal's (itself pinned to the oracle by the parity tests),
    parents a valid BFS tree by the tree properties, m_c equal."""
    import torch
    import bench
    from tree_props import bfs_tree_violations
    dg = gg.kronecker_device(24, 16, seed=2)
    roots = gg.sample_roots_device(dg, 16, seed=1_000_002)
    host = dg.to_host()
    off_t, idx_t = dg.offsets_tensor(), dg.indices_tensor()
    budget, _ = bench.hybrid_budget(host.degrees(), 0.12)
    params = dobfs.make_params("edge", alpha=56)
    with dobfs.HybridGraph.upload(host.offsets, host.indices, gpu_budget_bytes=budget, threads=16) as hg, \
            dobfs.Graph.upload(host.offsets, host.indices, reindex=True) as rg:
        for r in roots:
            r = int(r)
            _say(f"[hybrid] scale 24 bench shape, root {r}")
            d, p, st = hg.run(r, params=params, stats=True)
            rd, _, rst = rg.run(r, stats=True)
            torch.cuda.synchronize()
            assert torch.equal(d, rd), r
            assert st.m_c == rst.m_c and st.reached == rst.reached
            bad = bfs_tree_violations(off_t, idx_t, d, p, r)
            assert bad == [], (r, bad)
    dg.free()
