"""The C-ABI library loads and exports every entry point its header declares
(no device calls: runs without a GPU)."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in os.listdir(os.path.join(ROOT, "include")) if h.endswith(".h")]


def _declared_functions() -> list[str]:
    names = []
    for h in HEADERS:
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"\b(dobfs_[a-z_0-9]+)\s*\(", src):
            names.append(m.group(1))
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("dobfs_graph_upload", "dobfs_run", "dobfs_graph_free", "dobfs_strerror"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import __graft_entry__
    __graft_entry__.ensure_built()
    import torch  # noqa: F401  (its HIP runtime first, as the binding does)
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1503_04359_amd", "libdobfs.so"))
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_the_exports():
    import paper_1503_04359_amd as dobfs
    assert set(dobfs.EXPORTED) <= set(_declared_functions())


def test_host_only_entry_points():
    import paper_1503_04359_amd as dobfs
    p = dobfs.default_params()
    assert (p.policy, p.alpha, p.beta) == (dobfs.POLICY_EDGE, 14, 24)
    assert dobfs._lib.dobfs_strerror(dobfs.ERANGE) == b"vertex out of range"
    with pytest.raises(TypeError):
        dobfs.make_params("edge", nonsense=1)
