"""Full-size parity on the other workloads, each at its real size:

* Chung-Lu stand-in for a real-world graph: 100M core vertices, exponent
  2.2, mean degree 20, max 10^6, 50 path tails of 200 (seed 3), built on the
  device; all 16 roots (seed 3 + 10^6) checked by the BFS-tree properties
  and the component edge count, one root against the oracle.
* Batched: Kronecker scale 24 (seed 4), 64 roots (seed 4 + 10^6) in one
  batched pass; every slot checked by the depth properties, three slots
  against the oracle.
* Packed: 2,000 Kronecker graphs of scales drawn uniformly from 10..18
  (seed 4000; graph i seed 4000 + i), one root each, in one packed pass;
  every graph's slice against the oracle.
* Served: the 8 resident Kronecker graphs (scales 18, 20, 22, 24, 24, 25,
  26, 26; seeds 5000 + j) under a Poisson trace, continuous batching and
  plain serving; every completed query's depths equal the reference of its
  (graph, root) bit for bit, where the reference comes from the oracle
  (scales up to 22) or from a plain run whose depths and parents pass the
  BFS-tree properties (larger scales; the properties fix the depths).

The properties (tests/tree_props.py) hold exactly when depths are the hop
distances, so they stand in for the oracle where it would take minutes."""
from __future__ import annotations

import sys
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import graphgen as gg
import oracle
from tree_props import bfs_depth_violations, bfs_tree_violations

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


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


def test_chung_lu_100m_all_roots(dobfs):
    import torch
    g = gg.chung_lu_device(100_000_000, 2.2, 20.0, 1e6, n_tails=50, tail_len=200, seed=3)
    roots = [int(r) for r in gg.sample_roots_device(g, 16, seed=3 + 1_000_000)]
    _say(f"[fullsize] chung-lu built on the device: n={g.n} m={g.m}; roots {roots[:4]}...")
    off, idx = g.offsets_tensor(), g.indices_tensor()
    deg = off[1:] - off[:-1]
    dg = dobfs.Graph.from_device_pointers(g.offsets_ptr, g.indices_ptr, g.n, g.m, borrow=False, reindex=True)
    torch.cuda.synchronize()
    levels = []
    for i, r in enumerate(roots):
        d, p, st = dg.run(r, stats=True)
        torch.cuda.synchronize()
        bad = bfs_tree_violations(off, idx, d, p, r)
        assert bad == [], (r, bad)
        assert st.m_c == int(deg[d >= 0].sum()) // 2 and st.reached == int((d >= 0).sum())
        levels.append(st.levels)
        if i == 0:
            host = g.to_host()
            exp, _ = oracle.bfs(host.offsets, host.indices, r)
            assert np.array_equal(d.cpu().numpy(), exp), r
            del host
            _say(f"[fullsize] chung-lu root {r}: equal to the oracle")
        _say(f"[fullsize] chung-lu root {r}: {st.levels} levels, tree properties hold")
    assert max(levels) >= 200  # the path tails are reached
    dg.free()
    g.free()


def test_batch_scale24_all_slots(dobfs):
    import torch
    g = gg.kronecker_device(24, 16, seed=4)
    roots = [int(r) for r in gg.sample_roots_device(g, 64, seed=4 + 1_000_000)]
    off, idx = g.offsets_tensor(), g.indices_tensor()
    _say(f"[fullsize] kronecker 24 built: n={g.n} m={g.m}")
    dg = dobfs.Graph.from_device_pointers(g.offsets_ptr, g.indices_ptr, g.n, g.m, borrow=False, reindex=True)
    out, _ = dg.batch(roots)
    torch.cuda.synchronize()
    for b, r in enumerate(roots):
        bad = bfs_depth_violations(off, idx, out[b], r)
        assert bad == [], (b, r, bad)
    _say("[fullsize] batch: all 64 slots pass the depth properties")
    host = g.to_host()
    for b in (0, 31, 63):
        exp, _ = oracle.bfs(host.offsets, host.indices, roots[b])
        assert np.array_equal(out[b].cpu().numpy(), exp), b
    _say("[fullsize] batch: slots 0, 31, 63 equal to the oracle")
    dg.free()
    g.free()


def test_pack_2000_graphs_every_graph(dobfs):
    import torch
    count = 2000
    rng = np.random.default_rng(4000)
    scales = rng.integers(10, 19, size=count)
    gs, roots = [], []
    for i in range(count):
        g = gg.kronecker_device(int(scales[i]), 16, seed=4000 + i)
        gs.append(g)
        roots.append(int(gg.sample_roots_device(g, 1, seed=4000 + i + 1_000_000)[0]))
    torch.cuda.synchronize()
    _say(f"[fullsize] pack: {count} graphs built, {sum(g.n for g in gs)} vertices, {sum(g.m for g in gs)} entries")
    pk = dobfs.Pack.upload(gs, reindex=True)
    out, _, _ = pk.run_pack(roots, want_parent=False)
    torch.cuda.synchronize()
    res = out.cpu().numpy()
    bases = pk.bases
    hosts = [g.to_host() for g in gs]
    for g in gs:
        g.free()
    pk.free()

    def one(i):
        exp, _ = oracle.bfs(hosts[i].offsets, hosts[i].indices, roots[i])
        return bool(np.array_equal(res[int(bases[i]):int(bases[i + 1])], exp))

    with ThreadPoolExecutor(max_workers=16) as ex:
        ok = list(ex.map(one, range(count)))
    assert all(ok), [i for i, x in enumerate(ok) if not x][:10]
    _say(f"[fullsize] pack: all {count} graphs equal to the oracle")


class _CheckingExecutor:
    """The serving loop's GPU executor, comparing every result with its
    reference as it is handed back."""

    def __init__(self, inner, refs, qmap):
        self.inner = inner
        self.n_graphs = inner.n_graphs
        self.refs = refs
        self.qmap = qmap
        self.lock = threading.Lock()
        self.checked = 0
        self.wrong: list = []

    def _check(self, gid, root, depth):
        import torch
        ok = torch.equal(depth, self.refs[(gid, root)])
        with self.lock:
            self.checked += 1
            if not ok:
                self.wrong.append((gid, root))

    def output_bytes(self, gid):
        return self.inner.output_bytes(gid)

    def open_session(self, gid):
        inner, outer = self.inner.open_session(gid), self

        class S:
            def admit(self, root, tag):
                return inner.admit(root, tag)

            def step(self):
                ended = inner.step()
                inner.stream.synchronize()
                for tag, d in ended:
                    q_gid, q_root = outer.qmap[int(tag)]
                    outer._check(q_gid, q_root, d)
                return ended

            def close(self):
                inner.close()
        return S()

    def run_plain(self, gid, root):
        d = self.inner.run_plain(gid, root)
        self._check(gid, int(root), d)
        return d

    def release(self, result):
        self.inner.release(result)


def test_served_every_result(dobfs):
    import torch
    from paper_1503_04359_amd import serve
    scales = [18, 20, 22, 24, 24, 25, 26, 26]
    graphs, pools, refs = [], [], {}
    for j, sc in enumerate(scales):
        g = gg.kronecker_device(sc, 16, seed=5000 + j)
        pool = [int(r) for r in gg.sample_roots_device(g, 4, seed=5000 + j + 1_000_000)]
        dg = dobfs.Graph.from_device_pointers(g.offsets_ptr, g.indices_ptr, g.n, g.m, borrow=False, reindex=True)
        if sc <= 22:
            host = g.to_host()
            for r in pool:
                exp, _ = oracle.bfs(host.offsets, host.indices, r)
                refs[(j, r)] = torch.from_numpy(exp).cuda()
        else:
            off, idx = g.offsets_tensor(), g.indices_tensor()
            for r in pool:
                d, p, _ = dg.run(r)
                torch.cuda.synchronize()
                bad = bfs_tree_violations(off, idx, d, p, r)
                assert bad == [], (j, r, bad)
                refs[(j, r)] = d
                del p
        g.free()
        graphs.append(dg)
        pools.append(pool)
        _say(f"[fullsize] served graph {j} (scale {sc}) resident, references fixed")
    params = dobfs.make_params("edge", chunk_levels=4)
    inner = serve.GpuExecutor(graphs, params=params)
    free, _ = torch.cuda.mem_get_info()
    for rate, mode in ((2000.0, "batched"), (2000.0, "plain"), (8000.0, "batched")):
        trace = serve.poisson_trace(rate, 1.0, len(graphs), pools, seed=6000 + int(rate))
        qmap = {q.qid: (q.gid, q.root) for q in trace}
        ex = _CheckingExecutor(inner, refs, qmap)
        srv = serve.Server(ex, memory_budget=max(0, free - (16 << 30)))
        rep, _ = srv.serve(trace, mode=mode, drain_s=30.0)
        assert rep.failed == 0 and rep.unfinished == 0, rep.as_dict()
        assert ex.checked == rep.completed == len(trace)
        assert ex.wrong == [], ex.wrong[:10]
        _say(f"[fullsize] served {mode} at {rate:g}/s: {ex.checked} results, each equal to its reference")
    for dg in graphs:
        dg.free()
