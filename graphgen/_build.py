"""Builds the native graph generators in-tree.

* ``libgraphgen.so``      host builder (g++ + OpenMP), ``csrc/gg_cpu.cpp``
* ``libgraphgen_gpu.so``  device builder for graphs too large for the host
  builder (hipcc for gfx950), ``csrc/gg_gpu.hip``

Each library gets a ``.stamp`` file with the SHA-256 digest of the sources
and flags it was built from; :func:`is_current` compares it with the tree.
"""
from __future__ import annotations

import glob
import hashlib
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
HOST_LIB = os.path.join(HERE, "libgraphgen.so")
DEV_LIB = os.path.join(HERE, "libgraphgen_gpu.so")
HOST_FLAGS = ["-O3", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-Wall"]
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    subprocess.run(cmd, check=True)


def _digest(sources: list[str], flags: list[str]) -> str:
    h = hashlib.sha256()
    for f in sorted(sources):
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    h.update(" ".join(flags).encode())
    return h.hexdigest()


def _host_inputs() -> list[str]:
    return [os.path.join(CSRC, "gg_cpu.cpp")] + glob.glob(os.path.join(CSRC, "*.h"))


def _dev_inputs() -> list[str]:
    return [os.path.join(CSRC, "gg_gpu.hip")] + glob.glob(os.path.join(CSRC, "*.h"))


def _stamp(lib: str, digest: str) -> None:
    with open(lib + ".stamp.tmp", "w") as fh:
        fh.write(digest + "\n")
    os.replace(lib + ".stamp.tmp", lib + ".stamp")


def _current(lib: str, digest: str) -> bool:
    if not os.path.exists(lib) or not os.path.exists(lib + ".stamp"):
        return False
    with open(lib + ".stamp") as fh:
        return fh.read().strip() == digest


def is_current() -> bool:
    ok = _current(HOST_LIB, _digest(_host_inputs(), HOST_FLAGS))
    if os.path.exists(os.path.join(CSRC, "gg_gpu.hip")):
        ok = ok and _current(DEV_LIB, _digest(_dev_inputs(), HIP_FLAGS))
    return ok


def build_host() -> str:
    digest = _digest(_host_inputs(), HOST_FLAGS)
    _run(["g++", *HOST_FLAGS, os.path.join(CSRC, "gg_cpu.cpp"), "-o", HOST_LIB + ".tmp"])
    os.replace(HOST_LIB + ".tmp", HOST_LIB)
    _stamp(HOST_LIB, digest)
    return HOST_LIB


def build_device() -> str | None:
    src = os.path.join(CSRC, "gg_gpu.hip")
    if not os.path.exists(src):
        return None
    digest = _digest(_dev_inputs(), HIP_FLAGS)
    _run(["hipcc", *HIP_FLAGS, src, "-o", DEV_LIB + ".tmp"])
    os.replace(DEV_LIB + ".tmp", DEV_LIB)
    _stamp(DEV_LIB, digest)
    return DEV_LIB


def build() -> None:
    build_host()
    build_device()


if __name__ == "__main__":
    build()
