"""Seeded synthetic graph inputs shared by the traversal library's tests and
benchmarks and by the oracle's tests.

This module only says which graph is traversed and from which roots; it holds
none of the traversal's arithmetic.  Every graph is a symmetric CSR (each
undirected edge stored as two directed entries, self-loops and duplicates
removed, rows sorted by ascending neighbour ID) with ``int64`` offsets and
``int32`` neighbour IDs, built by the native host builder in
``csrc/gg_cpu.cpp`` (OpenMP; deterministic whatever the thread count).

Families:
  * :func:`kronecker` -- R-MAT / Kronecker graphs (quadrant probabilities
    A, B, C, D = 1-A-B-C, ``edgefactor * 2**scale`` generated edges, seeded
    vertex relabelling), the synthetic workload of the paper's experiments
    (Section 4, "Workloads").
  * :func:`chung_lu` -- power-law expected-degree graphs with long path
    tails, the stand-in for the paper's real-world social graphs.
  * small closed-form families (path, cycle, star, ...) for tests.
"""
from __future__ import annotations

import ctypes
import hashlib
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None

# Parameters of the synthetic workloads (A/B/C quadrant probabilities of the
# Graph500-style Kronecker generator, edge factor 16).
KRON_A, KRON_B, KRON_C = 0.57, 0.19, 0.19
KRON_EDGEFACTOR = 16


class _GgCsr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64),
                ("offsets", ctypes.POINTER(ctypes.c_int64)),
                ("indices", ctypes.POINTER(ctypes.c_int32))]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from graphgen import _build
        _build.build_host()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.POINTER
    lib.gg_kronecker.restype = P(_GgCsr)
    lib.gg_kronecker.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_int, P(ctypes.c_int)]
    lib.gg_chung_lu.restype = P(_GgCsr)
    lib.gg_chung_lu.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, P(ctypes.c_int)]
    lib.gg_from_edges.restype = P(_GgCsr)
    lib.gg_from_edges.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                  P(ctypes.c_int)]
    lib.gg_csr_free.restype = None
    lib.gg_csr_free.argtypes = [P(_GgCsr)]
    lib.gg_sample_roots.restype = ctypes.c_int64
    lib.gg_sample_roots.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int64,
                                    ctypes.c_void_p]
    lib.gg_kronecker_edges.restype = None
    lib.gg_kronecker_edges.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_int, ctypes.c_int64, ctypes.c_int64,
                                       ctypes.c_void_p, ctypes.c_void_p]
    lib.gg_permute_value.restype = ctypes.c_uint32
    lib.gg_permute_value.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32]
    lib.gg_rmat_thresholds.restype = None
    lib.gg_rmat_thresholds.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_void_p]
    lib.gg_set_threads.restype = None
    lib.gg_set_threads.argtypes = [ctypes.c_int]
    lib.gg_chung_lu_weights.restype = ctypes.c_int
    lib.gg_chung_lu_weights.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                        P(ctypes.c_double), P(ctypes.c_double)]
    _lib = lib
    return lib


@dataclass
class CSR:
    """Symmetric CSR: ``offsets`` int64[n+1], ``indices`` int32[m]."""
    offsets: np.ndarray
    indices: np.ndarray
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def m(self) -> int:
        return int(self.indices.shape[0])

    def degrees(self) -> np.ndarray:
        return np.diff(self.offsets)

    def digest(self) -> str:
        """SHA-256 over (n, m, offsets, indices): the identity of a graph."""
        h = hashlib.sha256()
        h.update(np.array([self.n, self.m], dtype=np.int64).tobytes())
        h.update(np.ascontiguousarray(self.offsets, dtype=np.int64).tobytes())
        h.update(np.ascontiguousarray(self.indices, dtype=np.int32).tobytes())
        return h.hexdigest()


def _take(ptr, status, what: str, name: str) -> CSR:
    if not ptr:
        raise RuntimeError(f"graphgen: {what} failed (status {status.value})")
    g = ptr.contents
    n, m = int(g.n), int(g.m)
    offsets = np.ctypeslib.as_array(g.offsets, shape=(n + 1,)).copy()
    indices = (np.ctypeslib.as_array(g.indices, shape=(m,)).copy() if m > 0
               else np.zeros(0, dtype=np.int32))
    _load().gg_csr_free(ptr)
    return CSR(offsets, indices, name)


def set_threads(n: int) -> None:
    _load().gg_set_threads(int(n))


def rmat_thresholds(a=KRON_A, b=KRON_B, c=KRON_C) -> tuple[int, int, int]:
    out = (ctypes.c_uint32 * 3)()
    _load().gg_rmat_thresholds(a, b, c, ctypes.addressof(out))
    return int(out[0]), int(out[1]), int(out[2])


def kronecker(scale: int, edgefactor: int = KRON_EDGEFACTOR, seed: int = 1,
              a: float = KRON_A, b: float = KRON_B, c: float = KRON_C,
              permute: bool = True) -> CSR:
    """Kronecker (R-MAT) graph with ``2**scale`` vertices and
    ``edgefactor * 2**scale`` generated undirected edges, cleaned and
    symmetrised."""
    st = ctypes.c_int(0)
    ptr = _load().gg_kronecker(int(scale), int(edgefactor), int(seed) & (2**64 - 1), a, b, c,
                               1 if permute else 0, ctypes.byref(st))
    return _take(ptr, st, "kronecker", f"kron-s{scale}-ef{edgefactor}-seed{seed}")


def kronecker_edges(scale: int, first: int, count: int, seed: int = 1, a=KRON_A, b=KRON_B, c=KRON_C,
                    permute: bool = True) -> tuple[np.ndarray, np.ndarray]:
    """Raw generated edges ``first .. first+count-1`` (before cleanup)."""
    u = np.empty(count, dtype=np.uint32)
    v = np.empty(count, dtype=np.uint32)
    _load().gg_kronecker_edges(int(scale), int(seed), a, b, c, 1 if permute else 0, int(first), int(count),
                               u.ctypes.data, v.ctypes.data)
    return u, v


def permute_value(seed: int, scale: int, x: int) -> int:
    return int(_load().gg_permute_value(int(seed), int(scale), int(x)))


def chung_lu(n_core: int, gamma: float = 2.2, avg_deg: float = 20.0, max_deg: float = 1e6,
             n_tails: int = 50, tail_len: int = 200, seed: int = 3) -> CSR:
    """Chung-Lu power-law graph plus ``n_tails`` path tails of ``tail_len``
    new vertices (IDs ``n_core + t*tail_len + j``)."""
    st = ctypes.c_int(0)
    ptr = _load().gg_chung_lu(int(n_core), float(gamma), float(avg_deg), float(max_deg), int(n_tails),
                              int(tail_len), int(seed), ctypes.byref(st))
    return _take(ptr, st, "chung_lu", f"cl-n{n_core}-g{gamma}-d{avg_deg}-t{n_tails}x{tail_len}-seed{seed}")


def chung_lu_weights(n_core: int, gamma: float, avg_deg: float, max_deg: float) -> tuple[float, float]:
    i0, c = ctypes.c_double(0), ctypes.c_double(0)
    rc = _load().gg_chung_lu_weights(int(n_core), gamma, avg_deg, max_deg, ctypes.byref(i0), ctypes.byref(c))
    if rc:
        raise ValueError(f"no Chung-Lu weights for these parameters (status {rc})")
    return i0.value, c.value


def from_edges(n: int, src, dst, name: str = "") -> CSR:
    """Cleaned symmetric CSR from an explicit edge list."""
    src = np.ascontiguousarray(src, dtype=np.int64)
    dst = np.ascontiguousarray(dst, dtype=np.int64)
    if src.shape != dst.shape:
        raise ValueError("src and dst differ in length")
    st = ctypes.c_int(0)
    ptr = _load().gg_from_edges(int(n), int(src.shape[0]), src.ctypes.data, dst.ctypes.data, ctypes.byref(st))
    return _take(ptr, st, "from_edges", name)


def sample_roots(g: CSR, count: int, seed: int) -> np.ndarray:
    """``count`` distinct roots of degree >= 1, uniform, drawn by seed."""
    off = np.ascontiguousarray(g.offsets, dtype=np.int64)
    out = np.empty(count, dtype=np.int64)
    k = _load().gg_sample_roots(off.ctypes.data, g.n, int(seed), int(count), out.ctypes.data)
    if k < count:
        raise ValueError(f"only {k} roots of degree >= 1 available, {count} requested")
    return out


# ---------------------------------------------------------------------------
# Small closed-form families (inputs only; expected distances live in tests).

def path(n: int) -> CSR:
    i = np.arange(n - 1)
    return from_edges(n, i, i + 1, f"path{n}")


def cycle(n: int) -> CSR:
    i = np.arange(n)
    return from_edges(n, i, (i + 1) % n, f"cycle{n}")


def star(n: int) -> CSR:
    """Center 0, leaves 1..n-1."""
    i = np.arange(1, n)
    return from_edges(n, np.zeros_like(i), i, f"star{n}")


def complete(n: int) -> CSR:
    u, v = np.triu_indices(n, 1)
    return from_edges(n, u, v, f"K{n}")


def complete_bipartite(a: int, b: int) -> CSR:
    """Sides [0, a) and [a, a+b)."""
    u, v = np.meshgrid(np.arange(a), np.arange(a, a + b), indexing="ij")
    return from_edges(a + b, u.ravel(), v.ravel(), f"K{a},{b}")


def grid2d(rows: int, cols: int) -> CSR:
    """Vertex r*cols + c; 4-neighbour grid."""
    r, c = np.meshgrid(np.arange(rows), np.arange(cols), indexing="ij")
    vid = r * cols + c
    src = np.concatenate([vid[:, :-1].ravel(), vid[:-1, :].ravel()])
    dst = np.concatenate([vid[:, 1:].ravel(), vid[1:, :].ravel()])
    return from_edges(rows * cols, src, dst, f"grid{rows}x{cols}")


def hypercube(d: int) -> CSR:
    n = 1 << d
    v = np.arange(n)
    src = np.concatenate([v for _ in range(d)])
    dst = np.concatenate([v ^ (1 << b) for b in range(d)])
    return from_edges(n, src, dst, f"Q{d}")


def binary_tree(n: int) -> CSR:
    """Heap-ordered complete binary tree: parent of i is (i-1)//2."""
    i = np.arange(1, n)
    return from_edges(n, (i - 1) // 2, i, f"bintree{n}")


def disjoint_union(*gs: CSR) -> CSR:
    srcs, dsts, base = [], [], 0
    for g in gs:
        deg = g.degrees()
        srcs.append(np.repeat(np.arange(g.n), deg) + base)
        dsts.append(g.indices.astype(np.int64) + base)
        base += g.n
    return from_edges(base, np.concatenate(srcs), np.concatenate(dsts), "union")
