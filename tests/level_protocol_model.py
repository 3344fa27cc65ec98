"""Host model of the single-source level loop's completion protocol (test
infrastructure, CPU only).

The device kernels (``bfs_kernels.hip``: ``level_body``, ``top_down``,
``decide``, ``k_aux``; ``device_common.h``: ``finish_block_all``) advance a
traversal through one shared control block: every workgroup reads the
level's state on entry, does its share, reports to a completion count, and
the last one to report closes the level (``decide``).  This module replays
that protocol step by step, with each workgroup a Python generator that
yields at every access to shared state, under a scheduler that chooses the
interleaving and the order in which workgroups are dispatched.  A workgroup
can be held back until the rest of its launch has finished, which is what
happens on the GPU when other streams' kernels occupy the compute units.

Two protocols are modelled:

* ``"fixed"``: the kernels as they are: every workgroup of a top-down
  launch reports (those without queue entries with empty counters), the
  one that closes a level runs the following one-workgroup levels alone,
  and the traversal's init clears the completion groups.
* ``"unchecked"``: the earlier form, in which only the ceil(n_f/kBlock)
  workgroups a top-down level needs reported, the others left at once, and
  workgroup 0 ran the one-workgroup chain.

The traversal is forced top-down (the direction rule plays no part in the
protocol), on an undirected graph given as adjacency lists.  Violations
recorded:

* ``stale-entry``: a queue position read for level L that was not written
  for level L (on the device: an uninitialised or stale vertex ID, used as
  an index);
* ``closed-while-running``: a level closed while a workgroup was still
  working on it;
* ``late-level``: a workgroup of a launch working on a level that was
  opened by another workgroup of the same launch;
* ``stale-ticket``: a completion count left non-zero when a launch ends;
* ``depth``: final depths differ from a plain BFS.
"""
from __future__ import annotations

import random
from collections import deque
from dataclasses import dataclass, field

AUX_NONE, AUX_TO_QUEUE = 0, 2


@dataclass
class Group:
    found: int = 0
    deg: int = 0
    ticket: int = 0


@dataclass
class Ctl:
    level: int = 0
    done: int = 0
    aux: int = AUX_NONE
    n_f: int = 0
    m_f: int = 0
    q_direct: int = 0
    q_append: int = 0
    qd_fill: int = 0
    q_fill: int = 0
    nf_next: int = 0
    mf_next: int = 0
    ticket: int = 0
    levels: int = 0
    groups: list = field(default_factory=list)


class Model:
    def __init__(self, adj, protocol: str, grid: int = 4, block: int = 2, ngroups: int = 2, direct_cap: int = 6):
        assert protocol in ("fixed", "unchecked")
        self.adj = adj
        self.n = len(adj)
        self.protocol = protocol
        self.G, self.B, self.KG, self.CAP = grid, block, ngroups, direct_cap
        self.ctl = Ctl(groups=[Group() for _ in range(ngroups)])
        self.violations: list[str] = []
        self.launch_id = 0

    # -- traversal state -----------------------------------------------------
    def init(self, root: int) -> None:
        c = self.ctl
        self.visited = {root}
        self.depth = [-1] * self.n
        self.depth[root] = 0
        self.fr = [{root}, set()]
        self.q0 = {0: (0, root)}
        self.qd = [{}, {}]
        c.level, c.done, c.aux = 0, 0, AUX_NONE
        c.n_f, c.m_f = 1, len(self.adj[root])
        c.q_direct, c.q_append = 0, int(len(self.adj[root]) <= self.CAP)
        c.qd_fill = c.q_fill = c.nf_next = c.mf_next = 0
        if self.protocol == "fixed":  # k_init_roots: reset_groups
            c.ticket = 0
            for g in c.groups:
                g.found = g.deg = g.ticket = 0
        self.working: dict[int, int] = {}  # level -> workgroups working on it
        self.opened_in: dict[int, int] = {0: -1}  # level -> launch that opened it

    # -- finish_block_all ----------------------------------------------------
    def finish(self, b, found, deg, count):
        c = self.ctl
        if count == 1:
            c.nf_next += found
            c.mf_next += deg
            return True
        ng = min(count, self.KG)
        gs = c.groups[b % ng]
        gsize = (count - b % ng + ng - 1) // ng
        yield
        gs.found += found
        gs.deg += deg
        yield
        t = gs.ticket
        gs.ticket += 1
        if t != gsize - 1:
            return False
        yield
        c.nf_next += gs.found
        c.mf_next += gs.deg
        gs.found = gs.deg = 0
        gs.ticket = 0
        yield
        t2 = c.ticket
        c.ticket += 1
        if t2 != ng - 1:
            return False
        c.ticket = 0
        return True

    # -- decide (forced top-down) ----------------------------------------------
    def decide(self):
        c = self.ctl
        L = c.level
        if self.working.get(L, 0) > 0:
            self.violations.append("closed-while-running")
        nfn, mfn = c.nf_next, c.mf_next
        if nfn == 0:
            c.done = 1
            c.levels = L + 1
        appended = c.q_append
        next_td = not c.done
        c.aux = AUX_TO_QUEUE if (next_td and not appended) else AUX_NONE
        c.q_direct = int(next_td and bool(appended))
        c.q_append = int(next_td and mfn <= self.CAP)
        c.qd_fill = 0
        c.q_fill = 0
        c.n_f, c.m_f = nfn, mfn
        c.level = L + 1
        c.nf_next = c.mf_next = 0
        self.opened_in[L + 1] = self.launch_id

    # -- top_down ------------------------------------------------------------
    def top_down(self, L, vb, nb, acc):
        c = self.ctl
        if self.opened_in.get(L, -1) == self.launch_id and not acc.get("alone"):
            self.violations.append("late-level")
        self.working[L] = self.working.get(L, 0) + 1
        q_cur = self.qd[L & 1] if c.q_direct else self.q0
        append = c.q_append
        q_app = self.qd[1 - (L & 1)] if append else None
        f_cur, f_nxt = self.fr[L & 1], self.fr[1 - (L & 1)]
        nf = c.n_f
        for i in range(vb * self.B, nf, nb * self.B):
            for j in range(i, min(i + self.B, nf)):
                yield
                ent = q_cur.get(j)
                if ent is None or ent[0] != L:
                    self.violations.append("stale-entry")
                    continue
                u = ent[1]
                if append:
                    f_cur.discard(u)
                for v in self.adj[u]:
                    yield
                    if v in self.visited:
                        continue
                    self.visited.add(v)
                    self.depth[v] = L + 1
                    f_nxt.add(v)
                    if append:
                        pos = c.qd_fill
                        c.qd_fill += 1
                        yield
                        q_app[pos] = (L + 1, v)
                    acc["found"] += 1
                    acc["deg"] += len(self.adj[v])
        self.working[L] -= 1

    # -- k_level_td ----------------------------------------------------------
    def wg_level_td(self, b):
        c = self.ctl
        yield
        if c.done or c.aux != AUX_NONE:
            return
        if self.protocol == "unchecked":
            chained = False
            while True:
                yield
                if c.done or c.aux != AUX_NONE:
                    return
                L = c.level
                nb = min(self.G, max(1, -(-c.n_f // self.B)))
                if b >= nb:
                    return
                acc = {"found": 0, "deg": 0, "alone": chained}
                chained = True
                yield from self.top_down(L, b, nb, acc)
                last = yield from self.finish(b, acc["found"], acc["deg"], nb)
                if last:
                    self.decide()
                if nb != 1:
                    return
                yield
                if not c.q_direct or c.n_f > self.B:
                    return
        alone = False
        while True:
            yield
            L = c.level
            vb = 0 if alone else b
            nb = min(1 if alone else self.G, max(1, -(-c.n_f // self.B)))
            acc = {"found": 0, "deg": 0, "alone": alone}
            if vb < nb:
                yield from self.top_down(L, vb, nb, acc)
            last = yield from self.finish(b, acc["found"], acc["deg"], 1 if alone else self.G)
            if not last:
                return
            self.decide()
            yield
            if c.done or c.aux != AUX_NONE or not c.q_direct or c.n_f > self.B:
                return
            alone = True

    # -- k_aux, bitmap to queue ------------------------------------------------
    def wg_aux(self, b):
        c = self.ctl
        yield
        if c.done or c.aux != AUX_TO_QUEUE:
            return
        L = c.level
        f_cur, f_old = self.fr[L & 1], self.fr[1 - (L & 1)]
        per = -(-self.n // self.G)
        lo, hi = b * per, min(self.n, (b + 1) * per)
        mine = sorted(v for v in f_cur if lo <= v < hi)
        f_old.difference_update(range(lo, hi))
        yield
        base = c.q_fill
        c.q_fill += len(mine)
        yield
        for k, v in enumerate(mine):
            self.q0[base + k] = (L, v)
        last = yield from self.finish(b, 0, 0, self.G)
        if last:
            c.aux = AUX_NONE

    # -- scheduling ----------------------------------------------------------
    def run_launch(self, kernel, rng: random.Random, late: frozenset, resident: int, late_prob: float = 0.0):
        self.launch_id += 1
        late = late | {b for b in range(self.G) if rng.random() < late_prob}
        pending = [b for b in range(self.G) if b not in late]
        held = [b for b in range(self.G) if b in late]
        running: dict[int, object] = {}
        while pending or held or running:
            can_dispatch = bool(pending) and len(running) < resident
            if not pending and not running:
                pending, held = held, []  # late workgroups come after the rest has finished
                continue
            if can_dispatch and (not running or rng.random() < 0.5):
                b = pending.pop(0)
                running[b] = kernel(b)
                continue
            b = rng.choice(list(running))
            try:
                next(running[b])
            except StopIteration:
                del running[b]
        c = self.ctl
        if c.ticket or any(g.ticket for g in c.groups):
            self.violations.append("stale-ticket")

    def traverse(self, root: int, rng: random.Random, late=frozenset(), resident: int | None = None,
                 late_prob: float = 0.0, max_slots: int = 400) -> list[int]:
        """One traversal from root.  Workgroups in `late`, and each other one
        with probability `late_prob` per launch, are dispatched only after
        the rest of their launch has finished; at most `resident` run at
        once."""
        self.init(root)
        res = resident or self.G
        for _ in range(max_slots):
            if self.ctl.done:
                break
            self.run_launch(self.wg_level_td, rng, late, res, late_prob)
            self.run_launch(self.wg_aux, rng, late, res, late_prob)
        exp = bfs_depths(self.adj, root)
        if self.depth != exp:
            self.violations.append("depth")
        return self.depth


def bfs_depths(adj, root):
    d = [-1] * len(adj)
    d[root] = 0
    q = deque([root])
    while q:
        u = q.popleft()
        for v in adj[u]:
            if d[v] < 0:
                d[v] = d[u] + 1
                q.append(v)
    return d


def broom(handle: int, bristles: int, tail: int):
    """Root 0, a path of `handle` vertices, then `bristles` leaves off its end,
    each continued by a path of `tail` vertices: level sizes 1, 1, ..., then
    `bristles` for `tail`+1 levels.  Undirected adjacency lists."""
    adj: list[list[int]] = [[]]

    def add(u):
        adj.append([])
        v = len(adj) - 1
        adj[u].append(v)
        adj[v].append(u)
        return v

    u = 0
    for _ in range(handle):
        u = add(u)
    for _ in range(bristles):
        x = add(u)
        for _ in range(tail):
            x = add(x)
    return adj


def random_graph(n: int, p: float, rng: random.Random):
    adj = [[] for _ in range(n)]
    for u in range(n):
        for v in range(u + 1, n):
            if rng.random() < p:
                adj[u].append(v)
                adj[v].append(u)
    return adj
