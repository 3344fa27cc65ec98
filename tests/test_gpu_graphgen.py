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


@pytest.mark.parametrize("n_core,gamma,avg,mx,tails,tlen,seed", [
    (1000, 2.2, 20.0, 200.0, 3, 20, 5),
    (20000, 2.2, 20.0, 2000.0, 10, 50, 3),
    (200000, 2.2, 20.0, 2e4, 20, 100, 77),
    (100000, 2.5, 8.0, 1e3, 0, 0, 9),
    (1_000_000, 2.2, 20.0, 1e5, 50, 200, 3),
])
def test_device_chung_lu_matches_host(torch_dev, n_core, gamma, avg, mx, tails, tlen, seed):
    print(f"[graphgen] chung-lu {n_core} core, {tails} tails of {tlen}, seed {seed}", flush=True)
    host = gg.chung_lu(n_core, gamma, avg, mx, n_tails=tails, tail_len=tlen, seed=seed)
    dev = gg.chung_lu_device(n_core, gamma, avg, mx, n_tails=tails, tail_len=tlen, seed=seed)
    try:
        assert (dev.n, dev.m) == (host.n, host.m)
        assert dev.to_host().digest() == host.digest()
    finally:
        dev.free()
