"""Host-side parts of the sweep-shape autotuner (no GPU needed)."""

import json

import pytest

from paper_2404_12134_amd import autotune


def test_length_signature_rounds_to_two_digits():
    n, p10, p50, p90 = autotune.length_signature([4000, 4100, 5000, 5900, 6000])
    assert n == 5
    assert p50 == 5000 and p10 == 4000 and p90 == 6000
    # batches differing only in detail share a signature
    assert autotune.length_signature([4012, 4991, 5988]) == autotune.length_signature([4009, 4990, 5991])


def test_cache_key_separates_shapes():
    k1 = autotune.cache_key("dev", "dba", 3, "f32", 4077, [5000] * 64)
    assert k1 == autotune.cache_key("dev", "dba", 3, "f32", 4077, [5000] * 64)
    assert k1 != autotune.cache_key("dev", "score", 3, "f32", 4077, [5000] * 64)
    assert k1 != autotune.cache_key("dev", "dba", 3, "f32", 4078, [5000] * 64)
    assert k1 != autotune.cache_key("dev", "dba", 3, "f32", 4077, [5000] * 65)


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    assert autotune.load_cache(path) == {}
    autotune.store_cache(path, "a", {"rho": 5, "grid": 0, "ms": 1.5, "table": [[5, 0, 1.5]]})
    autotune.store_cache(path, "b", {"rho": 4, "grid": 0, "ms": 2.0, "table": []})
    data = json.load(open(path))
    assert data["a"]["rho"] == 5 and data["b"]["rho"] == 4


def test_candidates_cover_the_supported_shapes():
    assert sorted(r for r, _ in autotune.candidates("dba")) == [2, 4, 5]
    assert sorted(r for r, _ in autotune.candidates("medoid")) == [2, 4, 5]


def test_tune_rejects_op_plan_mismatch_before_any_gpu_call():
    with pytest.raises(ValueError):
        autotune.tune([0, 5], 1, "f64", 0, op="dba")
    with pytest.raises(ValueError):
        autotune.tune([0, 5], 1, "f64", 4, op="medoid")
    with pytest.raises(ValueError):
        autotune.tune([0, 5], 1, "f64", 4, op="nope")
