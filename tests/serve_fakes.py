"""CPU stand-in for the serving executor: a numpy bit-parallel multi-source
BFS session with the same admit/step contract as the device session (one
level per step), for testing the scheduler without a GPU."""
from __future__ import annotations

import threading

import numpy as np


class CpuSession:
    def __init__(self, offsets, indices, owner):
        self.off = np.asarray(offsets, dtype=np.int64)
        self.idx = np.asarray(indices, dtype=np.int64)
        self.n = self.off.size - 1
        self.deg = np.diff(self.off)
        self.visit = np.zeros(self.n, dtype=np.uint64)
        self.cur = np.zeros(self.n, dtype=np.uint64)
        self.slots: dict[int, tuple[int, int, np.ndarray]] = {}  # bit -> (tag, start level, depths)
        self.pending: list[tuple[int, int]] = []
        self.level = 0
        self.owner = owner

    def admit(self, root: int, tag: int):
        if not 0 <= root < self.n:
            raise ValueError("root out of range")
        if len(self.slots) + len(self.pending) >= 64:
            raise RuntimeError("busy")
        self.pending.append((int(root), int(tag)))

    def _one_level(self) -> np.ndarray:
        acc = np.zeros(self.n, dtype=np.uint64)
        if self.idx.size:
            nz = self.deg > 0
            acc[nz] = np.bitwise_or.reduceat(self.cur[self.idx], self.off[:-1][nz])
        return acc & ~self.visit

    def step(self) -> list:
        self.owner.on_step()
        for root, tag in self.pending:
            b = next(i for i in range(64) if i not in self.slots)
            bit = np.uint64(1 << b)
            self.visit &= ~bit
            self.cur &= ~bit
            self.visit[root] |= bit
            self.cur[root] |= bit
            d = np.full(self.n, -1, dtype=np.int32)
            d[root] = 0
            self.slots[b] = (tag, self.level, d)
        self.pending.clear()
        self.owner.note_inflight(4 * self.n * len(self.slots))
        new = self._one_level()
        self.visit |= new
        ended = []
        for b, (tag, start, d) in list(self.slots.items()):
            hit = (new >> np.uint64(b)) & np.uint64(1)
            vs = np.flatnonzero(hit)
            d[vs] = self.level + 1 - start
            if vs.size == 0:
                ended.append((tag, d))
                del self.slots[b]
        self.cur = new
        self.level += 1
        self.owner.note_inflight(4 * self.n * len(self.slots))
        return ended

    def close(self) -> None:
        pass


class CpuExecutor:
    """graphs: list of (offsets, indices); fail_steps: global step numbers at
    which a session step raises (failure injection)."""

    def __init__(self, graphs, fail_steps=()):
        self.graphs = list(graphs)
        self.n_graphs = len(self.graphs)
        self.fail_steps = set(fail_steps)
        self.steps = 0
        self.max_inflight = 0
        self.total_inflight_now = {}
        self._lock = threading.Lock()

    def on_step(self):
        with self._lock:
            self.steps += 1
            if self.steps in self.fail_steps:
                raise RuntimeError(f"injected failure at step {self.steps}")

    def note_inflight(self, nbytes):
        """Output bytes held by the calling thread's session."""
        with self._lock:
            tid = threading.get_ident()
            self.total_inflight_now[tid] = nbytes
            self.max_inflight = max(self.max_inflight, sum(self.total_inflight_now.values()))

    def output_bytes(self, gid):
        return 4 * (len(self.graphs[gid][0]) - 1)

    def open_session(self, gid):
        off, idx = self.graphs[gid]
        return CpuSession(off, idx, self)

    def run_plain(self, gid, root):
        off, idx = self.graphs[gid]
        s = CpuSession(off, idx, _NoOwner())
        s.admit(root, 0)
        while True:
            out = s.step()
            if out:
                return out[0][1]

    def release(self, result):
        pass


class _NoOwner:
    def on_step(self):
        pass

    def note_inflight(self, k):
        pass
