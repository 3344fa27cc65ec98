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
    lib.gg_root_candidates.restype = None
    lib.gg_root_candidates.argtypes = [ctypes.c_int64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64,
                                       ctypes.c_void_p]
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


# ---------------------------------------------------------------------------
# Device builder (graphs too large for the host builder).

_dlib = None
_DLIB_PATH = os.path.join(_HERE, "libgraphgen_gpu.so")


def _load_device():
    global _dlib
    if _dlib is not None:
        return _dlib
    if not os.path.exists(_DLIB_PATH):
        raise ImportError(f"{_DLIB_PATH} is missing: build it first (python graphgen/_build.py)")
    import torch  # noqa: F401  (the HIP runtime the device builder shares; see the binding)
    lib = ctypes.CDLL(_DLIB_PATH)
    P = ctypes.POINTER
    lib.ggd_kronecker.restype = ctypes.c_int
    lib.ggd_kronecker.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int,
                                  P(ctypes.c_void_p), P(ctypes.c_void_p), P(ctypes.c_int64), P(ctypes.c_int64),
                                  ctypes.c_void_p]
    lib.ggd_chung_lu.restype = ctypes.c_int
    lib.ggd_chung_lu.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                 ctypes.c_int32, ctypes.c_uint64, P(ctypes.c_void_p), P(ctypes.c_void_p),
                                 P(ctypes.c_int64), P(ctypes.c_int64), ctypes.c_void_p]
    lib.ggd_free.restype = None
    lib.ggd_free.argtypes = [ctypes.c_void_p]
    lib.ggd_last_error.restype = ctypes.c_char_p
    lib.ggd_last_error.argtypes = []
    _dlib = lib
    return lib


class _CudaArray:
    """Exposes a raw device allocation to torch through the CUDA array
    interface (no copy)."""

    def __init__(self, ptr: int, n: int, typestr: str):
        self.__cuda_array_interface__ = {"shape": (n,), "typestr": typestr, "data": (ptr, False),
                                         "version": 2, "strides": None}


class DeviceCSR:
    """Symmetric CSR resident on the current GPU, owned by this object
    (released by :meth:`free`).  ``offsets_ptr``/``indices_ptr`` are raw
    device addresses of int64[n+1] / int32[m]."""

    def __init__(self, off_ptr: int, idx_ptr: int, n: int, m: int, name: str):
        self.offsets_ptr = off_ptr
        self.indices_ptr = idx_ptr
        self.n = n
        self.m = m
        self.name = name

    def offsets_tensor(self):
        import torch
        return torch.as_tensor(_CudaArray(self.offsets_ptr, self.n + 1, "<i8"), device="cuda")

    def indices_tensor(self):
        import torch
        return torch.as_tensor(_CudaArray(self.indices_ptr, max(self.m, 1), "<i4"), device="cuda")[: self.m]

    def to_host(self) -> CSR:
        return CSR(self.offsets_tensor().cpu().numpy(), self.indices_tensor().cpu().numpy(), self.name)

    def degree_of(self, vertices: np.ndarray) -> np.ndarray:
        import torch
        off = self.offsets_tensor()
        v = torch.as_tensor(np.asarray(vertices, dtype=np.int64), device="cuda")
        return (off[v + 1] - off[v]).cpu().numpy()

    def free(self) -> None:
        if self.offsets_ptr:
            _load_device().ggd_free(ctypes.c_void_p(self.offsets_ptr))
            _load_device().ggd_free(ctypes.c_void_p(self.indices_ptr))
            self.offsets_ptr = self.indices_ptr = 0

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def kronecker_device(scale: int, edgefactor: int = KRON_EDGEFACTOR, seed: int = 1, a: float = KRON_A,
                     b: float = KRON_B, c: float = KRON_C, permute: bool = True, stream=None) -> DeviceCSR:
    """Same graph as :func:`kronecker`, built on the current GPU."""
    import torch
    lib = _load_device()
    thr = (ctypes.c_uint32 * 3)(*rmat_thresholds(a, b, c))
    off, idx = ctypes.c_void_p(), ctypes.c_void_p()
    n, m = ctypes.c_int64(0), ctypes.c_int64(0)
    s = stream if stream is not None else torch.cuda.current_stream()
    rc = lib.ggd_kronecker(int(scale), int(edgefactor), int(seed), ctypes.addressof(thr), 1 if permute else 0,
                           ctypes.byref(off), ctypes.byref(idx), ctypes.byref(n), ctypes.byref(m),
                           ctypes.c_void_p(int(s.cuda_stream)))
    if rc:
        raise RuntimeError(f"graphgen device builder failed ({rc}): {lib.ggd_last_error().decode()}")
    return DeviceCSR(off.value, idx.value, n.value, m.value, f"kron-s{scale}-ef{edgefactor}-seed{seed}")


def chung_lu_device(n_core: int, gamma: float = 2.2, avg_deg: float = 20.0, max_deg: float = 1e6,
                    n_tails: int = 50, tail_len: int = 200, seed: int = 3, stream=None) -> DeviceCSR:
    """Same graph as :func:`chung_lu`, built on the current GPU (the alias
    table and the tail anchors on the host, every edge on the device)."""
    import torch
    lib = _load_device()
    off, idx = ctypes.c_void_p(), ctypes.c_void_p()
    n, m = ctypes.c_int64(0), ctypes.c_int64(0)
    s = stream if stream is not None else torch.cuda.current_stream()
    rc = lib.ggd_chung_lu(int(n_core), float(gamma), float(avg_deg), float(max_deg), int(n_tails), int(tail_len),
                          int(seed), ctypes.byref(off), ctypes.byref(idx), ctypes.byref(n), ctypes.byref(m),
                          ctypes.c_void_p(int(s.cuda_stream)))
    if rc:
        raise RuntimeError(f"device Chung-Lu builder failed ({rc}): {lib.ggd_last_error().decode()}")
    return DeviceCSR(off.value, idx.value, n.value, m.value,
                     f"cl-n{n_core}-g{gamma}-d{avg_deg}-t{n_tails}x{tail_len}-seed{seed}")


def sample_roots_device(g: DeviceCSR, count: int, seed: int) -> np.ndarray:
    """Same roots as :func:`sample_roots` would draw for this graph."""
    lib = _load()
    out: list[int] = []
    first, batch = 0, max(64, 4 * count)
    while len(out) < count:
        if first > 64 * g.n + 4096:
            raise ValueError("not enough roots of degree >= 1")
        cand = np.empty(batch, dtype=np.int64)
        lib.gg_root_candidates(g.n, int(seed), first, batch, cand.ctypes.data)
        deg = g.degree_of(cand)
        for c_, d_ in zip(cand.tolist(), deg.tolist()):
            if d_ >= 1 and c_ not in out:
                out.append(c_)
                if len(out) == count:
                    break
        first += batch
    return np.array(out, dtype=np.int64)
