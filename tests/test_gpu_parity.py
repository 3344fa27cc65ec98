"""Parity of the HIP traversal with the oracle: depths bit-exact, parents
checked by the BFS-tree properties (any valid parent is accepted), work
counters equal to the oracle's replay of the same direction schedule."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import graphgen as gg
import oracle
from golden_io import read_handworked

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


def _run(dobfs, dg, root, **kw):
    import torch
    params = kw.pop("params", None)
    d, p, st = dg.run(root, params=params, stats=True, **kw)
    torch.cuda.synchronize()
    return d.cpu().numpy(), p.cpu().numpy(), st


def degree_class(d):
    """One class per power of two: the bit length of the degree; degree 0
    is class 0."""
    d = np.asarray(d, dtype=np.int64)
    bl = np.zeros_like(d)
    nz = d > 0
    bl[nz] = np.floor(np.log2(d[nz])).astype(np.int64) + 1
    return bl


def degree_relabel(g):
    """The relabelling rule written out: internal ID = rank by degree class,
    highest first, ties by ID; rows sorted by internal ID."""
    deg = g.degrees()
    new2old = np.lexsort((np.arange(g.n), -degree_class(deg)))
    old2new = np.empty_like(new2old)
    old2new[new2old] = np.arange(g.n)
    src = np.repeat(np.arange(g.n), deg)
    key = np.sort(old2new[src].astype(np.int64) * g.n + old2new[g.indices])
    off = np.zeros(g.n + 1, dtype=np.int64)
    off[1:] = np.cumsum(deg[new2old])
    return off, (key % g.n).astype(np.int32), new2old, old2new


def _parity(dobfs, g, roots, params=None, replay=True, label="", reindex=False):
    if reindex:
        r_off, r_idx, new2old, _ = degree_relabel(g)
    with dobfs.Graph.upload(g.offsets, g.indices, reindex=reindex) as dg:
        for r in roots:
            r = int(r)
            _say(f"[parity] {label or g.name} n={g.n} m={g.m} root={r}")
            exp, _ = oracle.bfs(g.offsets, g.indices, r)
            d, p, st = _run(dobfs, dg, r, params=params)
            assert np.array_equal(d, exp), (label, r, np.flatnonzero(d != exp)[:10])
            code, bad = oracle.check_tree(g.offsets, g.indices, r, d, p)
            assert code == 0, (oracle.CHECK_CODES[code], bad)
            assert st.m_c == oracle.traversed_edges(g.offsets, exp)
            assert st.reached == int((exp >= 0).sum())
            assert st.levels == int(exp.max()) + 1
            if replay and len(st.log) == st.levels:
                if reindex:
                    rep = oracle.replay(r_off, r_idx, exp[new2old], st.dirs())
                else:
                    rep = oracle.replay(g.offsets, g.indices, exp, st.dirs())
                got = np.array([[rec["n_f"], rec["m_f"], rec["scanned"], rec["checked"], rec["found"],
                                 rec["found_deg"]] for rec in st.log])
                assert np.array_equal(got, rep[:, :6]), (label, r, got, rep[:, :6])


# ---------------------------------------------------------------------------

def test_closed_form_graphs(dobfs):
    cases = [gg.path(1), gg.path(2), gg.path(97), gg.cycle(130), gg.star(300), gg.complete(40),
             gg.complete_bipartite(3, 70), gg.grid2d(17, 23), gg.hypercube(9), gg.binary_tree(1000),
             gg.disjoint_union(gg.path(70), gg.cycle(9), gg.from_edges(2, [], []))]
    for g in cases:
        roots = sorted({0, g.n // 2, g.n - 1})
        for pol in ("edge", "td", "bu"):
            _parity(dobfs, g, roots, params=dobfs.make_params(pol), label=f"{g.name}/{pol}")


def test_handworked_fixture(dobfs):
    n, src, dst, cases = read_handworked("handworked_10.txt")
    g = gg.from_edges(n, src, dst)
    with dobfs.Graph.upload(g.offsets, g.indices) as dg:
        for root, exp in cases:
            for pol in ("edge", "td", "bu"):
                d, p, _ = _run(dobfs, dg, root, params=dobfs.make_params(pol))
                assert list(d) == exp, (root, pol)
                assert oracle.check_tree(g.offsets, g.indices, root, d, p)[0] == 0


def test_kronecker_s16_sixteen_roots(dobfs):
    """Kronecker scale 16, edgefactor 16, seed 1; 16 roots of degree >= 1."""
    g = gg.kronecker(16, seed=1)
    roots = gg.sample_roots(g, 16, seed=1_000_001)
    _parity(dobfs, g, roots, label="kron16")


def test_kronecker_s22_several_word_groups_per_step(dobfs):
    """Kronecker scale 22 (2.4M non-isolated vertices): more 64-vertex
    words than the bottom-up grid's wavefronts take in one step of four
    words each, so wavefronts hold two word groups per step, with and
    without the degree relabel.  Depths bit-exact, trees valid, and the
    per-level counters equal the oracle's replay."""
    g = gg.kronecker(22, seed=3)
    roots = [int(r) for r in gg.sample_roots(g, 2, seed=5)]
    exp = {r: oracle.bfs(g.offsets, g.indices, r)[0] for r in roots}
    r_off, r_idx, new2old, _ = degree_relabel(g)
    for reindex in (False, True):
        with dobfs.Graph.upload(g.offsets, g.indices, reindex=reindex) as dg:
            for pol in ("edge", "bu"):
                for r in roots:
                    _say(f"[parity] kron22/{pol}/reindex={reindex} root={r}")
                    d, p, st = _run(dobfs, dg, r, params=dobfs.make_params(pol))
                    assert np.array_equal(d, exp[r]), (pol, reindex, r, np.flatnonzero(d != exp[r])[:10])
                    code, bad = oracle.check_tree(g.offsets, g.indices, r, d, p)
                    assert code == 0, (oracle.CHECK_CODES[code], bad)
                    assert len(st.log) == st.levels
                    if reindex:
                        rep = oracle.replay(r_off, r_idx, exp[r][new2old], st.dirs())
                    else:
                        rep = oracle.replay(g.offsets, g.indices, exp[r], st.dirs())
                    got = np.array([[rec["n_f"], rec["m_f"], rec["scanned"], rec["checked"], rec["found"],
                                     rec["found_deg"]] for rec in st.log])
                    assert np.array_equal(got, rep[:, :6]), (pol, reindex, r, got, rep[:, :6])


@pytest.mark.parametrize("policy", ["td", "bu", "paper", "edge"])
def test_policy_invariance_kronecker(dobfs, policy):
    g = gg.kronecker(14, seed=3)
    roots = gg.sample_roots(g, 4, seed=7)
    _parity(dobfs, g, roots, params=dobfs.make_params(policy), label=f"kron14/{policy}")


def test_random_direction_schedules(dobfs):
    g = gg.kronecker(13, seed=5)
    roots = gg.sample_roots(g, 3, seed=9)
    for seed in range(6):
        _parity(dobfs, g, roots, params=dobfs.make_params("random", seed=seed), label=f"kron13/random{seed}")


def test_degree_cutoffs_exercise_every_bin(dobfs):
    """Small cut-offs push vertices through the wave-per-vertex, split and
    cooperative bottom-up paths."""
    g = gg.kronecker(14, seed=11)
    roots = gg.sample_roots(g, 3, seed=2)
    for kw in ({"td_wave_cut": 0, "td_huge_cut": 256, "bu_heavy_cut": 1},
               {"td_wave_cut": 64, "td_huge_cut": 300, "bu_heavy_cut": 8},
               {"td_wave_cut": 4096, "td_huge_cut": 1 << 30, "bu_heavy_cut": 1 << 30}):
        for pol in ("td", "bu", "edge"):
            _parity(dobfs, g, roots, params=dobfs.make_params(pol, **kw), label=f"kron14/{pol}/{kw}")


def test_hub_split_star(dobfs):
    g = gg.star(20000)  # center degree 19999 > every split cut-off
    _parity(dobfs, g, [0, 1, 19999], params=dobfs.make_params("td"), label="star-td")
    _parity(dobfs, g, [0, 1, 19999], params=dobfs.make_params("bu"), label="star-bu")


def test_long_paths_many_levels(dobfs):
    g = gg.chung_lu(30000, gamma=2.2, avg_deg=8.0, max_deg=3000.0, n_tails=5, tail_len=150, seed=3)
    roots = gg.sample_roots(g, 2, seed=4)
    _parity(dobfs, g, roots, label="chung-lu+tails")
    _parity(dobfs, g, roots, params=dobfs.make_params("paper"), label="chung-lu+tails/paper")
    g = gg.path(3000)  # 3000 levels: many host chunks, log cap not reached
    _parity(dobfs, g, [0, 1500], params=dobfs.make_params("edge", chunk_levels=3), label="path3000")


def test_isolated_root_and_tiny(dobfs):
    g = gg.disjoint_union(gg.cycle(5), gg.from_edges(3, [], []))
    _parity(dobfs, g, [6, 7, 0], label="isolated")
    g = gg.from_edges(1, [], [])
    _parity(dobfs, g, [0], label="single vertex")


def test_repeatable_and_parent_optional(dobfs):
    import torch
    g = gg.kronecker(15, seed=2)
    root = int(gg.sample_roots(g, 1, seed=3)[0])
    with dobfs.Graph.upload(g.offsets, g.indices) as dg:
        ref, _, _ = _run(dobfs, dg, root)
        for _ in range(5):
            d, _, _ = _run(dobfs, dg, root)
            assert np.array_equal(d, ref)
        d, p, _ = dg.run(root, want_parent=False)
        torch.cuda.synchronize()
        assert p is None and np.array_equal(d.cpu().numpy(), ref)


def test_device_upload_and_errors(dobfs):
    import torch
    g = gg.kronecker(10, seed=4)
    off = torch.from_numpy(g.offsets).cuda()
    idx = torch.from_numpy(g.indices).cuda()
    with dobfs.Graph.upload(off, idx, check_symmetry=True) as dg:
        r = int(gg.sample_roots(g, 1, seed=1)[0])
        d, _, _ = _run(dobfs, dg, r)
        assert np.array_equal(d, oracle.bfs(g.offsets, g.indices, r)[0])
        with pytest.raises(dobfs.DobfsError) as ei:
            dg.run(g.n)
        assert ei.value.status == dobfs.ERANGE
        with pytest.raises(dobfs.DobfsError) as ei:
            dg.run(0, params=dobfs.make_params("edge", alpha=0))
        assert ei.value.status == dobfs.EINVAL
    bad = g.indices.copy()
    bad[5] = g.n + 3
    with pytest.raises(dobfs.DobfsError) as ei:
        dobfs.Graph.upload(g.offsets, bad)
    assert ei.value.status == dobfs.EINVAL
    asym = gg.from_edges(4, [0, 1], [1, 2])
    idx2 = asym.indices.copy()
    idx2[-1] = 0  # row 2 becomes [0]: edge (2, 0) without (0, 2)
    with pytest.raises(dobfs.DobfsError):
        dobfs.Graph.upload(asym.offsets, idx2, check_symmetry=True)


# ---------------------------------------------------------------------------
# Degree-relabelled graphs: outputs in the caller's labels, work counters
# equal to the replay over the relabelled CSR built by the rule above.

def test_reindex_closed_forms(dobfs):
    cases = [gg.path(50), gg.star(300), gg.complete_bipartite(3, 70), gg.grid2d(9, 11), gg.binary_tree(500),
             gg.disjoint_union(gg.path(70), gg.cycle(9), gg.from_edges(3, [], [])), gg.from_edges(1, [], [])]
    for g in cases:
        roots = sorted({0, g.n // 2, g.n - 1})
        for pol in ("edge", "td", "bu"):
            _parity(dobfs, g, roots, params=dobfs.make_params(pol), label=f"{g.name}/{pol}/reindex", reindex=True)


def test_reindex_kronecker_policies(dobfs):
    g = gg.kronecker(15, seed=6)
    roots = gg.sample_roots(g, 4, seed=8)
    for pol in ("edge", "td", "bu", "paper"):
        _parity(dobfs, g, roots, params=dobfs.make_params(pol), label=f"kron15/{pol}/reindex", reindex=True)
    _parity(dobfs, g, roots[:2], params=dobfs.make_params("random", seed=3), label="kron15/random/reindex",
            reindex=True)


def test_reindex_kronecker_s16_sixteen_roots(dobfs):
    g = gg.kronecker(16, seed=1)
    roots = gg.sample_roots(g, 16, seed=1_000_001)
    _parity(dobfs, g, roots, label="kron16/reindex", reindex=True)


def test_reindex_device_source_and_parent_optional(dobfs):
    import torch
    g = gg.kronecker(12, seed=4)
    off = torch.from_numpy(g.offsets).cuda()
    idx = torch.from_numpy(g.indices).cuda()
    r = int(gg.sample_roots(g, 1, seed=1)[0])
    exp = oracle.bfs(g.offsets, g.indices, r)[0]
    with dobfs.Graph.upload(off, idx, reindex=True) as dg:
        info = dg.info()
        assert info["flags"] & dobfs.REINDEX_DEGREE
        assert info["n_nonisolated"] == int((g.degrees() > 0).sum())
        d, p, _ = dg.run(r, want_parent=False)
        torch.cuda.synchronize()
        assert p is None and np.array_equal(d.cpu().numpy(), exp)
    # the source arrays are left untouched
    assert np.array_equal(off.cpu().numpy(), g.offsets) and np.array_equal(idx.cpu().numpy(), g.indices)


def test_cost_policy(dobfs):
    g = gg.kronecker(14, seed=12)
    roots = gg.sample_roots(g, 3, seed=4)
    for kap in (50, 500, 5000):
        _parity(dobfs, g, roots, params=dobfs.make_params("cost", kappa_x1000=kap), label=f"kron14/cost{kap}")
        _parity(dobfs, g, roots, params=dobfs.make_params("cost", kappa_x1000=kap), label=f"kron14/cost{kap}/reindex",
                reindex=True)

