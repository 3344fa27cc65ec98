"""Direction-optimized breadth-first search on one MI355X (gfx950).

Thin Python binding over the C ABI declared in ``include/dobfs.h`` and built
into ``libdobfs.so``: argument marshalling only.  Every step of a traversal
runs in the library's HIP kernels; PyTorch supplies device memory and
streams.  There is no fallback: importing this package fails when the HIP
library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdobfs.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it first (python __graft_entry__.py build, "
        "or python paper_1503_04359_amd/_build.py)")


def _check_stamp() -> None:
    """Refuses a library built from sources other than the ones in the tree
    (its stamp holds their digest; see _build.py)."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("_dobfs_build", os.path.join(_HERE, "_build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    if not mod.is_current():
        raise ImportError(f"{LIB_PATH} is older than its sources: rebuild it (python __graft_entry__.py build)")


_check_stamp()

# torch first: it brings the process's HIP runtime, which the library then
# shares; loading the library first would start a second runtime that sees
# no device once torch's is up.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

# ---- status codes and flags (include/dobfs.h) ------------------------------
OK, EINVAL, ERANGE, ENOMEM, EDEVICE, EBUSY, ENOTSUP = 0, -1, -2, -3, -4, -5, -6
SRC_DEVICE, VALIDATE, VALIDATE_SYMMETRY, REINDEX_DEGREE, BORROW = 0x1, 0x2, 0x4, 0x8, 0x10
RUN_TIME_KERNELS, RUN_GRAPH, RUN_EAGER, RUN_HUB_DECIDES = 0x1, 0x2, 0x4, 0x8
POLICY_EDGE, POLICY_PAPER, POLICY_FORCED_TD, POLICY_FORCED_BU, POLICY_RANDOM, POLICY_COST = 0, 1, 2, 3, 4, 5
POLICIES = {"edge": POLICY_EDGE, "paper": POLICY_PAPER, "td": POLICY_FORCED_TD,
            "bu": POLICY_FORCED_BU, "random": POLICY_RANDOM, "cost": POLICY_COST}

EXPORTED = ("dobfs_default_params", "dobfs_graph_upload", "dobfs_graph_free", "dobfs_graph_info",
            "dobfs_run", "dobfs_run_noalloc", "dobfs_run_multi", "dobfs_batch_submit", "dobfs_pack_upload", "dobfs_pack_bases",
            "dobfs_pack_run", "dobfs_session_open", "dobfs_session_admit", "dobfs_session_step",
            "dobfs_session_counts", "dobfs_session_levels", "dobfs_session_close", "dobfs_hybrid_upload",
            "dobfs_hybrid_info", "dobfs_hybrid_run", "dobfs_hybrid_free", "dobfs_strerror", "dobfs_last_error")


class DobfsError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = _lib.dobfs_strerror(status).decode()
        detail = _lib.dobfs_last_error().decode()
        super().__init__(f"{where}: {msg}" + (f" ({detail})" if detail else ""))


class CParams(ctypes.Structure):
    _fields_ = [("policy", ctypes.c_int32), ("alpha", ctypes.c_int32), ("beta", ctypes.c_int32),
                ("paper_pct", ctypes.c_int32), ("paper_div", ctypes.c_int32),
                ("paper_bu_steps", ctypes.c_int32), ("td_wave_cut", ctypes.c_int32),
                ("td_huge_cut", ctypes.c_int32), ("bu_heavy_cut", ctypes.c_int32),
                ("chunk_levels", ctypes.c_int32), ("flags", ctypes.c_uint32), ("kappa_x1000", ctypes.c_int32),
                ("seed", ctypes.c_uint64)]


class LevelRec(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("dir", ctypes.c_int32), ("n_f", ctypes.c_int64),
                ("m_f", ctypes.c_int64), ("m_u", ctypes.c_int64), ("scanned", ctypes.c_int64),
                ("checked", ctypes.c_int64), ("found", ctypes.c_int64), ("found_deg", ctypes.c_int64),
                ("t_end", ctypes.c_uint64), ("kernel_ms", ctypes.c_float), ("reserved", ctypes.c_int32)]


class CStats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("log_len", ctypes.c_int32), ("reached", ctypes.c_int64),
                ("m_c", ctypes.c_int64), ("checked", ctypes.c_int64), ("t_begin", ctypes.c_uint64),
                ("log", ctypes.POINTER(LevelRec)), ("log_cap", ctypes.c_int32),
                ("level_launches", ctypes.c_int32), ("level_kernel_ms", ctypes.c_double),
                ("td_kernel_ms", ctypes.c_double), ("bu_kernel_ms", ctypes.c_double),
                ("aux_kernel_ms", ctypes.c_double)]


class CGraphInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("n_nonisolated", ctypes.c_int64),
                ("max_degree", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("flags", ctypes.c_uint32), ("reserved", ctypes.c_int32)]


_vp, _i64 = ctypes.c_void_p, ctypes.c_int64
_lib.dobfs_default_params.restype = None
_lib.dobfs_default_params.argtypes = [ctypes.POINTER(CParams)]
_lib.dobfs_graph_upload.restype = ctypes.c_int
_lib.dobfs_graph_upload.argtypes = [_vp, _vp, _i64, _i64, ctypes.c_uint32, _vp, ctypes.POINTER(_vp)]
_lib.dobfs_graph_free.restype = ctypes.c_int
_lib.dobfs_graph_free.argtypes = [_vp]
_lib.dobfs_graph_info.restype = ctypes.c_int
_lib.dobfs_graph_info.argtypes = [_vp, ctypes.POINTER(CGraphInfo)]
_lib.dobfs_run.restype = ctypes.c_int
_lib.dobfs_run.argtypes = [_vp, _i64, _vp, _vp, ctypes.POINTER(CParams), ctypes.POINTER(CStats), _vp]
_lib.dobfs_batch_submit.restype = ctypes.c_int
_lib.dobfs_batch_submit.argtypes = [_vp, _vp, ctypes.c_int32, _vp, ctypes.POINTER(CParams), ctypes.POINTER(CStats),
                                    _vp]
_lib.dobfs_run_multi.restype = ctypes.c_int
_lib.dobfs_run_multi.argtypes = [_vp, _vp, ctypes.c_int32, _vp, _vp, ctypes.POINTER(CParams), ctypes.POINTER(CStats),
                                 _vp]
_lib.dobfs_pack_upload.restype = ctypes.c_int
_lib.dobfs_pack_upload.argtypes = [ctypes.c_int32, _vp, _vp, _vp, _vp, ctypes.c_uint32, _vp, ctypes.POINTER(_vp)]
_lib.dobfs_pack_bases.restype = ctypes.c_int
_lib.dobfs_pack_bases.argtypes = [_vp, _vp]
_lib.dobfs_pack_run.restype = ctypes.c_int
_lib.dobfs_pack_run.argtypes = [_vp, _vp, _vp, _vp, ctypes.POINTER(CParams), ctypes.POINTER(CStats), _vp]
_lib.dobfs_session_open.restype = ctypes.c_int
_lib.dobfs_session_open.argtypes = [_vp, ctypes.POINTER(CParams), _vp, ctypes.POINTER(_vp)]
_lib.dobfs_session_admit.restype = ctypes.c_int
_lib.dobfs_session_admit.argtypes = [_vp, _i64, _vp, _i64]
_lib.dobfs_session_step.restype = ctypes.c_int
_lib.dobfs_session_step.argtypes = [_vp, _vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
_lib.dobfs_session_counts.restype = ctypes.c_int
_lib.dobfs_session_counts.argtypes = [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(_i64)]
_lib.dobfs_session_levels.restype = ctypes.c_int
_lib.dobfs_session_levels.argtypes = [_vp, ctypes.POINTER(LevelRec), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
_lib.dobfs_session_close.restype = ctypes.c_int
_lib.dobfs_session_close.argtypes = [_vp]
_lib.dobfs_strerror.restype = ctypes.c_char_p
_lib.dobfs_hybrid_upload.restype = ctypes.c_int
_lib.dobfs_hybrid_upload.argtypes = [_vp, _vp, _i64, _i64, _i64, ctypes.c_int32, _vp, ctypes.POINTER(_vp)]
_lib.dobfs_hybrid_info.restype = ctypes.c_int
_lib.dobfs_hybrid_info.argtypes = [_vp, _vp, _vp, _vp, _vp]
_lib.dobfs_hybrid_run.restype = ctypes.c_int
_lib.dobfs_hybrid_run.argtypes = [_vp, _i64, _vp, _vp, ctypes.POINTER(CParams), ctypes.POINTER(CStats), _vp]
_lib.dobfs_hybrid_free.restype = ctypes.c_int
_lib.dobfs_hybrid_free.argtypes = [_vp]
_lib.dobfs_strerror.argtypes = [ctypes.c_int]
_lib.dobfs_last_error.restype = ctypes.c_char_p
_lib.dobfs_last_error.argtypes = []


def _check(status: int, where: str) -> None:
    if status != OK:
        raise DobfsError(status, where)


def default_params() -> CParams:
    p = CParams()
    _lib.dobfs_default_params(ctypes.byref(p))
    return p


def make_params(policy: str | int = "edge", **kw) -> CParams:
    p = default_params()
    p.policy = POLICIES[policy] if isinstance(policy, str) else int(policy)
    for k, v in kw.items():
        if not hasattr(p, k):
            raise TypeError(f"unknown parameter {k}")
        setattr(p, k, int(v))
    return p


@dataclass
class Stats:
    levels: int
    reached: int
    m_c: int
    checked: int
    log: list = field(default_factory=list)
    level_launches: int = 0
    level_kernel_ms: float = 0.0
    td_kernel_ms: float = 0.0
    bu_kernel_ms: float = 0.0
    aux_kernel_ms: float = 0.0
    log_len: int = 0

    def dirs(self) -> list[int]:
        return [r["dir"] for r in self.log]


def _make_stats(stats: bool, log_cap: int = 4096):
    if not stats:
        return None, None
    log = (LevelRec * log_cap)()
    cs = CStats()
    cs.log = ctypes.cast(log, ctypes.POINTER(LevelRec))
    cs.log_cap = log_cap
    return cs, log


def _read_stats(cs, log):
    if cs is None:
        return None
    recs = [{f: getattr(log[i], f) for f, _ in LevelRec._fields_} for i in range(cs.log_len)]
    return Stats(cs.levels, cs.reached, cs.m_c, cs.checked, recs, cs.level_launches, cs.level_kernel_ms,
                 cs.td_kernel_ms, cs.bu_kernel_ms, cs.aux_kernel_ms, cs.log_len)


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(int(t.data_ptr()))


class Graph:
    """A graph resident on the current device."""

    def __init__(self, handle: ctypes.c_void_p, n: int, m: int):
        self._h = handle
        self.n = n
        self.m = m

    @classmethod
    def from_device_pointers(cls, offsets_ptr: int, indices_ptr: int, n: int, m: int, *, borrow: bool = True,
                             reindex: bool = False, check_symmetry: bool = False, stream=None) -> "Graph":
        """CSR already on the device as raw pointers (int64[n+1], int32[m]).
        With ``borrow`` the arrays are used in place and must outlive the
        graph."""
        flags = SRC_DEVICE | VALIDATE | (BORROW if borrow else 0)
        flags |= (VALIDATE_SYMMETRY if check_symmetry else 0) | (REINDEX_DEGREE if reindex else 0)
        h = ctypes.c_void_p()
        _check(_lib.dobfs_graph_upload(ctypes.c_void_p(offsets_ptr), ctypes.c_void_p(indices_ptr), int(n), int(m),
                                       flags, _stream_ptr(stream), ctypes.byref(h)), "dobfs_graph_upload")
        return cls(h, int(n), int(m))

    @classmethod
    def upload(cls, offsets, indices, *, reindex: bool = False, check_symmetry: bool = False,
               stream=None) -> "Graph":
        """offsets int64[n+1], indices int32[m]: numpy arrays (host) or torch
        tensors on the GPU (copied on the device)."""
        import torch
        flags = VALIDATE | (VALIDATE_SYMMETRY if check_symmetry else 0) | (REINDEX_DEGREE if reindex else 0)
        if isinstance(offsets, torch.Tensor):
            if offsets.dtype != torch.int64 or indices.dtype != torch.int32:
                raise TypeError("offsets must be int64 and indices int32")
            if not (offsets.is_cuda and indices.is_cuda):
                offsets, indices = offsets.numpy(), indices.numpy()
            else:
                offsets, indices = offsets.contiguous(), indices.contiguous()
                flags |= SRC_DEVICE
                n, m = offsets.shape[0] - 1, indices.shape[0]
                h = ctypes.c_void_p()
                _check(_lib.dobfs_graph_upload(_ptr(offsets), _ptr(indices), n, m, flags, _stream_ptr(stream),
                                               ctypes.byref(h)), "dobfs_graph_upload")
                return cls(h, n, m)
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        idx = np.ascontiguousarray(indices, dtype=np.int32)
        n, m = off.shape[0] - 1, idx.shape[0]
        h = ctypes.c_void_p()
        _check(_lib.dobfs_graph_upload(off.ctypes.data, idx.ctypes.data if m else None, n, m, flags,
                                       _stream_ptr(stream), ctypes.byref(h)), "dobfs_graph_upload")
        return cls(h, n, m)

    def info(self) -> dict:
        i = CGraphInfo()
        _check(_lib.dobfs_graph_info(self._h, ctypes.byref(i)), "dobfs_graph_info")
        return {k: getattr(i, k) for k, _ in CGraphInfo._fields_ if k != "reserved"}

    def run(self, root: int, depth=None, parent=None, params: CParams | None = None, stats: bool = False,
            stream=None, want_parent: bool = True, log_cap: int = 4096):
        """Single-source traversal.  Returns (depth, parent, Stats|None);
        depth/parent are int32 CUDA tensors valid after the stream syncs."""
        import torch
        if depth is None:
            depth = torch.empty(self.n, dtype=torch.int32, device="cuda")
        if parent is None and want_parent:
            parent = torch.empty(self.n, dtype=torch.int32, device="cuda")
        for t in (depth, parent):
            if t is not None and (t.dtype != torch.int32 or t.numel() < self.n or not t.is_cuda
                                  or not t.is_contiguous()):
                raise ValueError("depth/parent must be contiguous int32 CUDA tensors of length n")
        cs, log = _make_stats(stats, log_cap)
        st = _lib.dobfs_run(self._h, int(root), _ptr(depth), _ptr(parent) if parent is not None else None,
                            ctypes.byref(params) if params is not None else None,
                            ctypes.byref(cs) if cs is not None else None, _stream_ptr(stream))
        _check(st, "dobfs_run")
        out_stats = _read_stats(cs, log)
        return depth, parent, out_stats

    def run_noalloc(self, root: int, depth=None, parent=None, params: CParams | None = None, stats: bool = False,
                    stream=None, want_parent: bool = True, log_cap: int = 4096):
        """dobfs_run_noalloc: the traversal of run() with the library's fixed
        scratch array as workspace (the library allocates nothing).  The
        output tensors are allocated here unless given.  Returns as run()."""
        import torch
        if depth is None:
            depth = torch.empty(self.n, dtype=torch.int32, device="cuda")
        if parent is None and want_parent:
            parent = torch.empty(self.n, dtype=torch.int32, device="cuda")
        for t in (depth, parent):
            if t is not None and (t.dtype != torch.int32 or t.numel() < self.n or not t.is_cuda
                                  or not t.is_contiguous()):
                raise ValueError("depth/parent must be contiguous int32 CUDA tensors of length n")
        cs, log = _make_stats(stats, log_cap)
        _check(_lib.dobfs_run_noalloc(self._h, int(root), _ptr(depth), _ptr(parent) if parent is not None else None,
                                      ctypes.byref(params) if params is not None else None,
                                      ctypes.byref(cs) if cs is not None else None, _stream_ptr(stream)),
               "dobfs_run_noalloc")
        return depth, parent, _read_stats(cs, log)

    def run_multi(self, roots, depth=None, parent=None, params: CParams | None = None, stats: bool = False,
                  stream=None, want_parent: bool = True):
        """One traversal from several roots: depth = distance to the nearest
        root.  Returns (depth, parent, Stats|None)."""
        import torch
        r = np.ascontiguousarray(np.asarray(roots, dtype=np.int64).ravel())
        if depth is None:
            depth = torch.empty(self.n, dtype=torch.int32, device="cuda")
        if parent is None and want_parent:
            parent = torch.empty(self.n, dtype=torch.int32, device="cuda")
        cs, log = _make_stats(stats)
        _check(_lib.dobfs_run_multi(self._h, r.ctypes.data, int(r.shape[0]), _ptr(depth),
                                    _ptr(parent) if parent is not None else None,
                                    ctypes.byref(params) if params is not None else None,
                                    ctypes.byref(cs) if cs is not None else None, _stream_ptr(stream)),
               "dobfs_run_multi")
        return depth, parent, _read_stats(cs, log)

    def batch(self, roots, depth=None, params: CParams | None = None, stats: bool = False, stream=None,
              log_cap: int = 4096):
        """Up to 64 traversals in one pass.  Returns (depth int32[k, n]
        CUDA tensor, root-major; Stats|None with totals over the slots)."""
        import torch
        r = np.ascontiguousarray(np.asarray(roots, dtype=np.int64).ravel())
        k = int(r.shape[0])
        if depth is None:
            depth = torch.empty((k, self.n), dtype=torch.int32, device="cuda")
        if depth.dtype != torch.int32 or depth.numel() < k * self.n or not depth.is_cuda or not depth.is_contiguous():
            raise ValueError("depth must be a contiguous int32 CUDA tensor of k*n elements")
        cs, log = _make_stats(stats, log_cap)
        _check(_lib.dobfs_batch_submit(self._h, r.ctypes.data, k, _ptr(depth),
                                       ctypes.byref(params) if params is not None else None,
                                       ctypes.byref(cs) if cs is not None else None, _stream_ptr(stream)),
               "dobfs_batch_submit")
        out = _read_stats(cs, log)
        return depth, out

    def session(self, params: CParams | None = None, stream=None) -> "Session":
        """A continuous-batching session over this graph."""
        return Session(self, params, stream)

    def free(self) -> None:
        if self._h:
            _check(_lib.dobfs_graph_free(self._h), "dobfs_graph_free")
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.free()


class Session:
    """Continuous batching over one graph: queries join the running 64-slot
    traversal between level chunks and leave when their frontier empties."""

    SLOTS = 64

    def __init__(self, graph: Graph, params: CParams | None = None, stream=None):
        self.graph = graph
        self._h = ctypes.c_void_p()
        self._done = np.zeros(self.SLOTS, dtype=np.int64)
        self._nd = ctypes.c_int32()
        self._outs: dict[int, object] = {}
        _check(_lib.dobfs_session_open(graph._h, ctypes.byref(params) if params is not None else None,
                                       _stream_ptr(stream), ctypes.byref(self._h)), "dobfs_session_open")

    def admit(self, root: int, tag: int, depth=None):
        """Queue a query; returns its depth tensor (complete once `tag` is
        reported by step()).  Raises DobfsError(EBUSY) when 64 are in flight."""
        import torch
        if depth is None:
            depth = torch.empty(self.graph.n, dtype=torch.int32, device="cuda")
        if depth.dtype != torch.int32 or depth.numel() < self.graph.n or not depth.is_cuda:
            raise ValueError("depth must be an int32 CUDA tensor of n elements")
        _check(_lib.dobfs_session_admit(self._h, int(root), _ptr(depth), int(tag)), "dobfs_session_admit")
        self._outs[int(tag)] = depth
        return depth

    def step(self) -> list[tuple[int, object]]:
        """One level chunk; returns [(tag, depth tensor)] of the queries that
        ended."""
        _check(_lib.dobfs_session_step(self._h, self._done.ctypes.data, self.SLOTS, ctypes.byref(self._nd)),
               "dobfs_session_step")
        return [(int(t), self._outs.pop(int(t))) for t in self._done[:self._nd.value]]

    def counts(self) -> tuple[int, int, int]:
        a, p, lv = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        _check(_lib.dobfs_session_counts(self._h, ctypes.byref(a), ctypes.byref(p), ctypes.byref(lv)),
               "dobfs_session_counts")
        return a.value, p.value, lv.value

    def levels(self) -> list[dict]:
        """Per-level records of the last step's chunk."""
        recs = (LevelRec * 1024)()
        k = ctypes.c_int32()
        _check(_lib.dobfs_session_levels(self._h, recs, 1024, ctypes.byref(k)), "dobfs_session_levels")
        return [{f: getattr(recs[i], f) for f, _ in LevelRec._fields_} for i in range(k.value)]

    def close(self) -> None:
        if self._h:
            _check(_lib.dobfs_session_close(self._h), "dobfs_session_close")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Pack(Graph):
    """Many small graphs resident as one pack, traversed in one pass with
    one root per graph."""

    def __init__(self, handle, n: int, m: int, bases: np.ndarray):
        super().__init__(handle, n, m)
        self.bases = bases

    @classmethod
    def upload(cls, graphs, *, reindex: bool = False, check_symmetry: bool = False, stream=None) -> "Pack":
        """graphs: sequence of (offsets, indices) as host numpy arrays, or of
        objects with offsets_ptr/indices_ptr/n/m (device CSRs)."""
        count = len(graphs)
        offp = (ctypes.c_void_p * count)()
        idxp = (ctypes.c_void_p * count)()
        ns = np.zeros(count, dtype=np.int64)
        ms = np.zeros(count, dtype=np.int64)
        keep = []
        device = hasattr(graphs[0], "offsets_ptr")
        for i, gr in enumerate(graphs):
            if device:
                offp[i], idxp[i], ns[i], ms[i] = gr.offsets_ptr, gr.indices_ptr, gr.n, gr.m
            else:
                off = np.ascontiguousarray(gr[0], dtype=np.int64)
                idx = np.ascontiguousarray(gr[1], dtype=np.int32)
                keep.append((off, idx))
                offp[i], idxp[i] = off.ctypes.data, (idx.ctypes.data if idx.shape[0] else None)
                ns[i], ms[i] = off.shape[0] - 1, idx.shape[0]
        flags = VALIDATE | (SRC_DEVICE if device else 0) | (VALIDATE_SYMMETRY if check_symmetry else 0)
        flags |= REINDEX_DEGREE if reindex else 0
        h = ctypes.c_void_p()
        _check(_lib.dobfs_pack_upload(count, offp, idxp, ns.ctypes.data, ms.ctypes.data, flags, _stream_ptr(stream),
                                      ctypes.byref(h)), "dobfs_pack_upload")
        bases = np.zeros(count + 1, dtype=np.int64)
        _check(_lib.dobfs_pack_bases(h, bases.ctypes.data), "dobfs_pack_bases")
        return cls(h, int(bases[-1]), int(ms.sum()), bases)

    def run_pack(self, roots, depth=None, parent=None, params: CParams | None = None, stats: bool = False,
                 stream=None, want_parent: bool = False):
        """roots: one graph-local root per graph.  Returns (depth, parent,
        Stats|None) over the pack's IDs; parents are pack IDs."""
        import torch
        r = np.ascontiguousarray(np.asarray(roots, dtype=np.int64).ravel())
        if depth is None:
            depth = torch.empty(self.n, dtype=torch.int32, device="cuda")
        if parent is None and want_parent:
            parent = torch.empty(self.n, dtype=torch.int32, device="cuda")
        cs, log = _make_stats(stats)
        _check(_lib.dobfs_pack_run(self._h, r.ctypes.data, _ptr(depth), _ptr(parent) if parent is not None else None,
                                   ctypes.byref(params) if params is not None else None,
                                   ctypes.byref(cs) if cs is not None else None, _stream_ptr(stream)),
               "dobfs_pack_run")
        return depth, parent, _read_stats(cs, log)


def hybrid_state_bytes(n: int) -> int:
    """Device bytes a hybrid graph of n vertices needs before any row: the
    smallest budget dobfs_hybrid_upload takes."""
    w = (n + 63) // 64
    return 8 * (n + 1) + 16 * n + 40 * w + 64


class HybridGraph:
    """A graph split between host memory (the hub rows, traversed by host
    threads) and the current device (every other row and all per-vertex
    state), for graphs whose rows do not fit the device budget."""

    def __init__(self, handle: ctypes.c_void_p, n: int, m: int):
        self._h = handle
        self.n = n
        self.m = m

    @classmethod
    def upload(cls, offsets, indices, *, gpu_budget_bytes: int, threads: int = 8, stream=None) -> "HybridGraph":
        """offsets int64[n+1], indices int32[m] in host memory (numpy)."""
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        idx = np.ascontiguousarray(indices, dtype=np.int32)
        n, m = off.shape[0] - 1, idx.shape[0]
        h = ctypes.c_void_p()
        _check(_lib.dobfs_hybrid_upload(off.ctypes.data, idx.ctypes.data if m else None, n, m, int(gpu_budget_bytes),
                                        int(threads), _stream_ptr(stream), ctypes.byref(h)), "dobfs_hybrid_upload")
        return cls(h, n, m)

    def info(self) -> dict:
        v = [ctypes.c_int64() for _ in range(4)]
        _check(_lib.dobfs_hybrid_info(self._h, *[ctypes.byref(x) for x in v]), "dobfs_hybrid_info")
        return dict(zip(("split", "host_entries", "gpu_entries", "gpu_bytes"), (x.value for x in v)))

    def run(self, root: int, depth=None, parent=None, params: CParams | None = None, stats: bool = False,
            want_parent: bool = True, stream=None):
        """Returns (depth, parent|None, Stats|None): int32 device tensors in
        caller IDs, written when the call returns."""
        import torch
        if depth is None:
            depth = torch.empty(self.n, dtype=torch.int32, device="cuda")
        if parent is None and want_parent:
            parent = torch.empty(self.n, dtype=torch.int32, device="cuda")
        cs, log = _make_stats(stats)
        _check(_lib.dobfs_hybrid_run(self._h, int(root), _ptr(depth), _ptr(parent) if parent is not None else None,
                                     ctypes.byref(params) if params is not None else None,
                                     ctypes.byref(cs) if cs is not None else None, _stream_ptr(stream)),
               "dobfs_hybrid_run")
        return depth, parent, _read_stats(cs, log)

    def free(self) -> None:
        if self._h:
            _check(_lib.dobfs_hybrid_free(self._h), "dobfs_hybrid_free")
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.free()
