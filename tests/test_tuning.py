"""Autotune cache (host logic only): problem signatures and the JSON file."""
import json
import os

import numpy as np

from paper_1911_02366_amd import tuning

CFG = ["64x64", "128x128"]


def test_signature_ignores_element_order_and_sees_every_field():
    n_i, n_c = np.array([320, 135, 320]), np.array([1200, 720, 1200])
    base = tuning.problem_signature(n_i, n_c, "fp64", "gpu", CFG)
    assert base == tuning.problem_signature(n_i[::-1], n_c[::-1], "fp64", "gpu", CFG)
    others = [tuning.problem_signature(n_i, n_c, "fp32", "gpu", CFG),
              tuning.problem_signature(n_i, n_c, "fp64", "other", CFG),
              tuning.problem_signature(n_i, n_c, "fp64", "gpu", CFG[:1]),
              tuning.problem_signature(n_i[:2], n_c[:2], "fp64", "gpu", CFG),
              tuning.problem_signature(np.array([320, 320, 135]), n_c, "fp64", "gpu", CFG)]
    assert len({base, *others}) == 6


def test_store_and_lookup_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "cache.json")
    assert tuning.lookup(path, "k1") is None                 # no file yet
    tuning.store(path, "k1", {"x": "64x64", "s": "128x128", "ms_x": {"64x64": 1.0}})
    tuning.store(path, "k2", {"x": "128x128", "s": "64x64"})
    assert tuning.lookup(path, "k1")["s"] == "128x128"
    assert tuning.lookup(path, "k2")["x"] == "128x128"
    assert sorted(json.load(open(path))) == ["k1", "k2"]
    assert [f for f in os.listdir(tmp_path / "sub") if f != "cache.json"] == []   # no temp files left


def test_unreadable_or_invalid_entries_count_as_missing(tmp_path):
    path = str(tmp_path / "cache.json")
    open(path, "w").write("{not json")
    assert tuning.lookup(path, "k") is None
    tuning.store(path, "k", {"x": "64x64", "s": "64x64"})     # a corrupt file is replaced
    assert tuning.lookup(path, "k") is not None
    json.dump({"k": {"x": 3}}, open(path, "w"))
    assert tuning.lookup(path, "k") is None
    assert tuning.lookup(None, "k") is None
    tuning.store(None, "k", {"x": "a", "s": "b"})            # no cache: nothing written
