"""The device graph builder reproduces the host builder bit for bit."""
from __future__ import annotations

import numpy as np
import pytest

import graphgen as gg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import __graft_entry__
    __graft_entry__.ensure_built()
    import torch
    torch.cuda.set_device(0)
    return torch


@pytest.mark.parametrize("scale,seed", [(1, 3), (4, 5), (10, 1), (14, 9), (16, 1), (18, 2)])
def test_device_builder_matches_host(torch_dev, scale, seed):
    print(f"[graphgen] scale {scale} seed {seed}", flush=True)
    host = gg.kronecker(scale, seed=seed)
    dev = gg.kronecker_device(scale, seed=seed)
    try:
        assert (dev.n, dev.m) == (host.n, host.m)
        got = dev.to_host()
        assert got.digest() == host.digest()
        if host.m > 0 and (host.degrees() > 0).sum() >= 4:
            k = min(8, int((host.degrees() > 0).sum()))
            assert np.array_equal(gg.sample_roots_device(dev, k, seed=77), gg.sample_roots(host, k, seed=77))
    finally:
        dev.free()
