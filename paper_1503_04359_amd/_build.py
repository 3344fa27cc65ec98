"""Builds ``libdobfs.so`` (HIP for gfx950) in-tree from ``csrc/``.

Next to the library it writes ``libdobfs.so.stamp``: a SHA-256 digest of
the sources, the public header and the compiler flags it was built from.
:func:`is_current` compares it with the tree, so a library older than its
sources is rebuilt (``ensure_built``) or refused (the binding's import)
instead of being run.
"""
from __future__ import annotations

import glob
import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libdobfs.so")
STAMP = LIB + ".stamp"
SOURCES = ["api.hip", "bfs_kernels.hip", "graph_kernels.hip", "reindex.hip", "msbfs.hip", "hybrid.hip"]
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             f"-I{INCLUDE}", f"-I{CSRC}"]


def _inputs() -> list[str]:
    files = glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.h"))
    files += glob.glob(os.path.join(INCLUDE, "*.h"))
    return sorted(files)


def source_digest() -> str:
    h = hashlib.sha256()
    for f in _inputs():
        h.update(os.path.relpath(f, ROOT).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    h.update(" ".join(SOURCES).encode())
    h.update(" ".join(HIP_FLAGS[:-2]).encode())  # include paths are machine-specific
    return h.hexdigest()


def is_current() -> bool:
    if not os.path.exists(LIB) or not os.path.exists(STAMP):
        return False
    with open(STAMP) as fh:
        return fh.read().strip() == source_digest()


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    digest = source_digest()
    cmd = ["hipcc", *HIP_FLAGS, "-shared", *srcs, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    with open(STAMP + ".tmp", "w") as fh:
        fh.write(digest + "\n")
    os.replace(STAMP + ".tmp", STAMP)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
