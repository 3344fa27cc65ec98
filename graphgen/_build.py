"""Builds the native graph generators in-tree.

* ``libgraphgen.so``      host builder (g++ + OpenMP), ``csrc/gg_cpu.cpp``
* ``libgraphgen_gpu.so``  device builder for graphs too large for the host
  builder (hipcc for gfx950), ``csrc/gg_gpu.hip``
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    subprocess.run(cmd, check=True)


def build_host() -> str:
    out = os.path.join(HERE, "libgraphgen.so")
    _run(["g++", "-O3", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-Wall",
          os.path.join(CSRC, "gg_cpu.cpp"), "-o", out + ".tmp"])
    os.replace(out + ".tmp", out)
    return out


def build_device() -> str | None:
    src = os.path.join(CSRC, "gg_gpu.hip")
    if not os.path.exists(src):
        return None
    out = os.path.join(HERE, "libgraphgen_gpu.so")
    _run(["hipcc", *HIP_FLAGS, src, "-o", out + ".tmp"])
    os.replace(out + ".tmp", out)
    return out


def build() -> None:
    build_host()
    build_device()


if __name__ == "__main__":
    build()
