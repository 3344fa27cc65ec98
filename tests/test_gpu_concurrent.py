"""Several traversals at once on one GPU, as the serving loop runs them:
different graphs (and one graph) driven from several host threads, each on
a stream of its own, plain runs and continuous-batching sessions mixed.
Every result must equal the oracle's depths, and parents must pass the tree
checker.

This covers the top-down completion protocol when other streams' kernels
hold the compute units (a workgroup of a top-down launch is then dispatched
late, after others of its launch have finished), and the first run of a
relabelled graph, which builds and publishes the graph's caller-ID column
while other threads start their own runs."""
from __future__ import annotations

import threading

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


def _graphs():
    """Kronecker scales 12 to 18, and a Chung-Lu core with path tails (long
    runs of one-workgroup top-down levels beside other streams' bottom-up
    levels)."""
    gs = [gg.kronecker(s, seed=700 + s) for s in (12, 14, 16, 17, 18)]
    gs.append(gg.chung_lu(200_000, gamma=2.2, avg_deg=20.0, max_deg=2e4, n_tails=20, tail_len=100, seed=77))
    return gs


def _run_threads(work):
    """Runs each callable in its own thread, all released together; re-raises
    the first exception."""
    start = threading.Barrier(len(work))
    errors = []

    def body(fn):
        try:
            start.wait()
            fn()
        except BaseException as e:  # noqa: BLE001  (reported in the main thread)
            errors.append(e)

    threads = [threading.Thread(target=body, args=(fn,)) for fn in work]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=300)
        assert not t.is_alive(), "a traversal thread did not finish"
    if errors:
        raise errors[0]


def _check(g, root, d, p, what):
    exp, _ = oracle.bfs(g.offsets, g.indices, int(root))
    assert np.array_equal(d, exp), what
    if p is not None:
        code, bad = oracle.check_tree(g.offsets, g.indices, int(root), d, p)
        assert code == 0, (what, oracle.CHECK_CODES[code], bad)


def test_concurrent_runs_on_different_graphs(dobfs):
    import torch
    graphs = _graphs()
    roots = [list(gg.sample_roots(g, 4, seed=900 + i)) for i, g in enumerate(graphs)]
    roots[-1].append(graphs[-1].n - 1)  # end of the last tail: a long top-down chain
    dgs = [dobfs.Graph.upload(g.offsets, g.indices, reindex=(i % 2 == 0)) for i, g in enumerate(graphs)]
    streams = [torch.cuda.Stream() for _ in graphs]
    out: dict[tuple[int, int, int], tuple[np.ndarray, np.ndarray]] = {}
    lock = threading.Lock()

    def job(i):
        def fn():
            s = streams[i]
            with torch.cuda.stream(s):
                for rep in range(3):
                    for r in roots[i]:
                        d, p, _ = dgs[i].run(int(r), stream=s)
                        s.synchronize()
                        with lock:
                            out[(i, int(r), rep)] = (d.cpu().numpy(), p.cpu().numpy())
        return fn

    print(f"[concurrent] {len(graphs)} graphs, {sum(map(len, roots))} roots x 3, one thread and stream each",
          flush=True)
    _run_threads([job(i) for i in range(len(graphs))])
    for (i, r, rep), (d, p) in sorted(out.items()):
        _check(graphs[i], r, d, p, (i, r, rep))
    for dg in dgs:
        dg.free()


def test_concurrent_first_runs_of_one_relabelled_graph(dobfs):
    import torch
    g = gg.kronecker(17, seed=712)
    roots = list(gg.sample_roots(g, 6, seed=913))
    dg = dobfs.Graph.upload(g.offsets, g.indices, reindex=True)  # fresh: no caller-ID column yet
    streams = [torch.cuda.Stream() for _ in roots]
    out = {}
    lock = threading.Lock()

    def job(k):
        def fn():
            s = streams[k]
            with torch.cuda.stream(s):
                d, p, _ = dg.run(int(roots[k]), stream=s)
                s.synchronize()
                with lock:
                    out[k] = (d.cpu().numpy(), p.cpu().numpy())
        return fn

    print(f"[concurrent] one relabelled graph, {len(roots)} first runs at once", flush=True)
    _run_threads([job(k) for k in range(len(roots))])
    for k, (d, p) in out.items():
        _check(g, roots[k], d, p, ("first-run", k))
    dg.free()


def test_concurrent_sessions_and_plain_runs(dobfs):
    """The serving loop's mix: a continuous-batching session per graph, each
    in its own thread and stream, and plain runs of the same graphs from
    other threads at the same time."""
    import torch
    from paper_1503_04359_amd import EBUSY, DobfsError
    graphs = [gg.kronecker(s, seed=730 + s) for s in (13, 15, 16, 17)]
    dgs = [dobfs.Graph.upload(g.offsets, g.indices, reindex=(i % 2 == 1)) for i, g in enumerate(graphs)]
    q_roots = [list(gg.sample_roots(g, 70, seed=940 + i)) for i, g in enumerate(graphs)]
    p_roots = [list(gg.sample_roots(g, 3, seed=960 + i)) for i, g in enumerate(graphs)]
    results: dict[tuple[str, int, int], np.ndarray] = {}
    lock = threading.Lock()

    def session_job(i):
        def fn():
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                sess = dgs[i].session(params=dobfs.make_params(chunk_levels=2), stream=s)
                nxt, done = 0, 0
                while done < len(q_roots[i]):
                    for _ in range(5):
                        if nxt >= len(q_roots[i]):
                            break
                        try:
                            sess.admit(int(q_roots[i][nxt]), tag=nxt)
                        except DobfsError as e:
                            assert e.status == EBUSY
                            break
                        nxt += 1
                    for tag, d in sess.step():
                        s.synchronize()
                        with lock:
                            results[("session", i, tag)] = d.cpu().numpy()
                        done += 1
                sess.close()
        return fn

    def plain_job(i):
        def fn():
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                for k, r in enumerate(p_roots[i]):
                    d, _, _ = dgs[i].run(int(r), stream=s, want_parent=False)
                    s.synchronize()
                    with lock:
                        results[("plain", i, k)] = d.cpu().numpy()
        return fn

    print(f"[concurrent] {len(graphs)} sessions x 70 queries + plain runs, 8 threads", flush=True)
    _run_threads([session_job(i) for i in range(len(graphs))] + [plain_job(i) for i in range(len(graphs))])
    for (kind, i, k), d in sorted(results.items()):
        r = q_roots[i][k] if kind == "session" else p_roots[i][k]
        _check(graphs[i], r, d, None, (kind, i, k))
    assert len(results) == sum(len(x) for x in q_roots) + sum(len(x) for x in p_roots)
    for dg in dgs:
        dg.free()
