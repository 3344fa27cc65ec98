"""The single-source level loop's completion protocol, replayed on the host
(``level_protocol_model.py``) under adversarial dispatch orders.  CPU only.

The earlier protocol, in which only the workgroups that hold queue entries
of a top-down level reported, is shown to go wrong when a workgroup is
dispatched after the level it was launched for has closed: it works on the
next level inside the wrong launch and leaves a completion ticket behind,
the next launch then closes a level while a workgroup still appends to it,
and a later level reads queue positions that were never written for it.
The protocol the kernels use survives every order tried."""
from __future__ import annotations

import random

import pytest

from level_protocol_model import Model, bfs_depths, broom, random_graph


def _broom():
    # level sizes 1, 1, 1, 12, 12, 12: one-workgroup levels, then a level
    # whose queue is handed on directly (the hub's 13 edges are within the
    # model's direct-queue cap of 16) and that needs every workgroup of the
    # grid (4 workgroups x 2 entries)
    return broom(handle=2, bristles=12, tail=2)


def test_unchecked_protocol_breaks_under_late_dispatch():
    adj = _broom()
    m = Model(adj, "unchecked", direct_cap=16)
    rng = random.Random(1)
    m.traverse(0, rng, late=frozenset({3}))
    assert "late-level" in m.violations
    assert "stale-ticket" in m.violations


def test_unchecked_protocol_reads_unwritten_queue_entries():
    # Several traversals on one control block (a reused workspace), each
    # workgroup held back with probability 0.3 per launch: a ticket left by
    # a late workgroup closes a later level early, while another workgroup
    # still appends to its queue, and a level then reads queue positions
    # that were not written for it (on the device, garbage vertex IDs used
    # as indices).
    adj = _broom()
    seen = set()
    for seed in range(40):
        m = Model(adj, "unchecked", direct_cap=16)
        rng = random.Random(seed)
        for _ in range(3):
            m.traverse(0, rng, resident=4, late_prob=0.3)
        seen.update(m.violations)
    assert {"closed-while-running", "stale-entry", "depth"} <= seen


@pytest.mark.parametrize("late", [frozenset(), frozenset({3}), frozenset({1, 3}), frozenset({0}), frozenset({0, 1, 2})])
def test_fixed_protocol_broom(late):
    adj = _broom()
    m = Model(adj, "fixed", direct_cap=16)
    for seed in range(30):
        rng = random.Random(seed)
        d = m.traverse(0, rng, late=late, resident=1 + seed % 4, late_prob=0.3 * (seed % 2))
        assert m.violations == [], (seed, m.violations)
        assert d == bfs_depths(adj, 0)


def test_fixed_protocol_random_graphs():
    for seed in range(60):
        rng = random.Random(1000 + seed)
        adj = random_graph(24, 0.08 + 0.02 * (seed % 5), rng)
        m = Model(adj, "fixed", grid=1 + seed % 5, block=1 + seed % 3, ngroups=1 + seed % 3,
                  direct_cap=seed % 9)
        late = frozenset(b for b in range(m.G) if rng.random() < 0.4)
        for root in (0, 5, 23):
            m.traverse(root, rng, late=late, resident=1 + seed % 3, late_prob=0.25)
            assert m.violations == [], (seed, root, m.violations)
