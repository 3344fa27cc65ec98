"""Oracle for breadth-first search over a symmetric CSR graph.

TEST INFRASTRUCTURE ONLY: the plain, slow, obviously correct statement of
what the traversal computes.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may use it; the device library never does, and
this package never imports the library.

* :func:`bfs` -- serial FIFO-queue BFS in C (``bfs_oracle.c``): hop distance
  from the root (-1 if unreachable) and the first-discoverer parent
  (definition of level-synchronous BFS, Section 2.2; top-down branch of
  Algorithm 1).
* :func:`check_tree` -- the BFS-tree properties that fix every depth and
  accept any valid parent (the Graph500 methodology asks for parents,
  Section 4).
* :func:`traversed_edges` -- undirected edges of the root's component, the
  TEPS numerator (Section 4, "Methodology").
* :func:`replay` -- exact per-level work of a direction schedule (Algorithm 1,
  both branches; bottom-up stops at the first frontier neighbour).
* :func:`bfs_py` -- a pure-Python twin of :func:`bfs` for tiny graphs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from collections import deque

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

CHECK_CODES = {
    0: "ok",
    1: "root labels",
    2: "value out of range",
    3: "reached/unreached labels disagree",
    4: "parent is not a neighbour",
    5: "parent depth is not depth-1",
    6: "edge spans more than one level or leaves the component",
}

REPLAY_FIELDS = ("n_f", "m_f", "scanned", "checked", "found", "found_deg", "unvisited_deg")


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        subprocess.run(["make", "-s", "-C", _HERE], check=True)
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    lib.oracle_bfs.restype = ctypes.c_int
    lib.oracle_bfs.argtypes = [i64, vp, vp, i64, vp, vp, vp]
    lib.oracle_check_tree.restype = ctypes.c_int
    lib.oracle_check_tree.argtypes = [i64, vp, vp, i64, vp, vp, ctypes.POINTER(i64)]
    lib.oracle_traversed_edges.restype = i64
    lib.oracle_traversed_edges.argtypes = [i64, vp, vp]
    lib.oracle_replay.restype = ctypes.c_int
    lib.oracle_replay.argtypes = [i64, vp, vp, vp, ctypes.c_int32, vp, vp]
    _lib = lib
    return lib


def _csr(offsets, indices):
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    idx = np.ascontiguousarray(indices, dtype=np.int32)
    if idx.shape[0] == 0:
        idx = np.zeros(1, dtype=np.int32)
    return off, idx


def bfs(offsets, indices, root: int) -> tuple[np.ndarray, np.ndarray]:
    """(depth int32[n], parent int32[n]) of a serial queue BFS from root."""
    off, idx = _csr(offsets, indices)
    n = off.shape[0] - 1
    depth = np.empty(n, dtype=np.int32)
    parent = np.empty(n, dtype=np.int32)
    rc = _load().oracle_bfs(n, off.ctypes.data, idx.ctypes.data, int(root), depth.ctypes.data,
                            parent.ctypes.data, None)
    if rc:
        raise ValueError(f"oracle_bfs: invalid arguments (status {rc})")
    return depth, parent


def check_tree(offsets, indices, root: int, depth, parent) -> tuple[int, int]:
    """(code, vertex): code 0 when every BFS-tree property holds, else the
    failure code (see CHECK_CODES) and the smallest offending vertex."""
    off, idx = _csr(offsets, indices)
    n = off.shape[0] - 1
    d = np.ascontiguousarray(depth, dtype=np.int32)
    p = np.ascontiguousarray(parent, dtype=np.int32)
    if d.shape[0] != n or p.shape[0] != n:
        raise ValueError("depth/parent length differs from n")
    bad = ctypes.c_int64(-1)
    rc = _load().oracle_check_tree(n, off.ctypes.data, idx.ctypes.data, int(root), d.ctypes.data,
                                   p.ctypes.data, ctypes.byref(bad))
    if rc < 0:
        raise ValueError(f"oracle_check_tree: invalid arguments (status {rc})")
    return int(rc), int(bad.value)


def traversed_edges(offsets, depth) -> int:
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    d = np.ascontiguousarray(depth, dtype=np.int32)
    return int(_load().oracle_traversed_edges(off.shape[0] - 1, off.ctypes.data, d.ctypes.data))


def replay(offsets, indices, depth, dirs) -> np.ndarray:
    """int64[len(dirs), 7] of per-level work counts (columns REPLAY_FIELDS)
    for direction schedule ``dirs`` (0 = top-down, 1 = bottom-up)."""
    off, idx = _csr(offsets, indices)
    d = np.ascontiguousarray(depth, dtype=np.int32)
    dr = np.ascontiguousarray(dirs, dtype=np.int8)
    out = np.zeros((max(1, dr.shape[0]), 8), dtype=np.int64)
    rc = _load().oracle_replay(off.shape[0] - 1, off.ctypes.data, idx.ctypes.data, d.ctypes.data,
                               int(dr.shape[0]), dr.ctypes.data, out.ctypes.data)
    if rc:
        raise ValueError(f"oracle_replay: invalid arguments (status {rc})")
    return out[: dr.shape[0], :7]


def bfs_py(offsets, indices, root: int) -> tuple[list[int], list[int]]:
    """Pure-Python serial queue BFS (same definition as :func:`bfs`)."""
    n = len(offsets) - 1
    depth = [-1] * n
    parent = [-1] * n
    depth[root] = 0
    parent[root] = root
    q = deque([root])
    while q:
        u = q.popleft()
        for e in range(int(offsets[u]), int(offsets[u + 1])):
            v = int(indices[e])
            if depth[v] < 0:
                depth[v] = depth[u] + 1
                parent[v] = u
                q.append(v)
    return depth, parent
