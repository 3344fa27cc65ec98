"""The autotuner's host logic (no GPU): tuning roots never include a
measurement root, the coordinate search finds the optimum of a known score
and ignores gains below its noise threshold, and tuned files load."""
from __future__ import annotations

import json

import numpy as np
import pytest

import graphgen as gg
from paper_1503_04359_amd import autotune


def test_tuning_roots_are_disjoint_from_measurement_roots():
    for scale, seed in ((12, 2), (14, 2), (16, 1)):
        g = gg.kronecker(scale, seed=seed)
        measure = gg.sample_roots(g, 16, seed=seed + autotune.MEASURE_ROOT_OFFSET)
        cand = gg.sample_roots(g, 8 + 16, seed=seed + autotune.TUNE_ROOT_OFFSET)
        tune = autotune.disjoint_roots(cand, measure, 8)
        assert len(tune) == 8 == len(set(tune))
        assert not set(tune) & set(int(x) for x in measure)
        deg = np.diff(g.offsets)
        assert all(deg[r] >= 1 for r in tune)


def test_disjoint_roots_keeps_order_and_refuses_shortfall():
    assert autotune.disjoint_roots([5, 3, 9, 1], [3], 2) == [5, 9]
    with pytest.raises(ValueError):
        autotune.disjoint_roots([1, 2], [1, 2], 1)


def test_coordinate_search_finds_separable_optimum():
    space = {"a": [1, 2, 3, 4], "b": [10, 20, 30]}
    target = {"a": 3, "b": 20}
    calls = []

    def score(p):
        calls.append(dict(p))
        return 100.0 - (p["a"] - target["a"]) ** 2 - ((p["b"] - target["b"]) / 10.0) ** 2

    best, sc, trials = autotune.coordinate_search(score, {"a": 1, "b": 30}, space, min_gain=0.0)
    assert best == target and sc == pytest.approx(100.0)
    assert len(calls) == len({tuple(sorted(c.items())) for c in calls})  # each set evaluated once
    assert max(t["score"] for t in trials) == sc


def test_coordinate_search_ignores_gains_below_threshold():
    space = {"a": [1, 2]}
    best, sc, _ = autotune.coordinate_search(lambda p: 100.0 + 0.1 * p["a"], {"a": 1}, space, min_gain=0.01)
    assert best == {"a": 1}  # 0.1% better is noise at a 1% threshold
    best, _, _ = autotune.coordinate_search(lambda p: 100.0 + 5.0 * p["a"], {"a": 1}, space, min_gain=0.01)
    assert best == {"a": 2}


def test_load_tuned(tmp_path):
    p = tmp_path / "t.json"
    assert autotune.load_tuned(str(p)) is None
    p.write_text(json.dumps({"params": {"alpha": 20, "beta": 24}}))
    assert autotune.load_tuned(str(p))["params"]["alpha"] == 20
    p.write_text(json.dumps({"params": {"nonsense": 1}}))
    with pytest.raises(ValueError):
        autotune.load_tuned(str(p))


def test_defaults_are_in_the_space_and_match_the_library():
    import paper_1503_04359_amd as dobfs
    d = dobfs.default_params()
    for k, v in autotune.DEFAULTS.items():
        assert v in autotune.SPACE[k]
        assert getattr(d, k) == v
