"""Host logic of the schedule autotuner (no GPU): the structure key depends
on the structure and the optimizer settings but not on measurement values,
and the cache round-trips through its JSON file."""
import numpy as np

import synth
from paper_2207_09442_amd import autotune as A


def test_structure_key_ignores_values_and_sees_structure():
    p = synth.walk_se3(batch=2, n_poses=8, n_loops=3, seed=1)
    q = dict(p)
    q["edge_meas"] = p["edge_meas"] * 1.01
    assert A.structure_key(p, 5, 0.0, "fp64", 0) == A.structure_key(q, 5, 0.0, "fp64", 0)
    assert A.structure_key(p, 5, 0.0, "fp64", 0) != A.structure_key(p, 6, 0.0, "fp64", 0)
    assert A.structure_key(p, 5, 0.0, "fp64", 0) != A.structure_key(p, 5, 0.0, "mixed", 1)
    r = dict(p)
    r["edge_ij"] = p["edge_ij"].copy()
    r["edge_ij"][3] = r["edge_ij"][3][::-1]
    assert A.structure_key(p, 5, 0.0, "fp64", 0) != A.structure_key(r, 5, 0.0, "fp64", 0)


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "cache.json")
    assert A._load(path) == {}
    A._store(path, {"k": {"solver": "sparse", "ms": 1.5}})
    assert A._load(path) == {"k": {"solver": "sparse", "ms": 1.5}}
    dense = [c for c in A.CANDIDATES if c["solver"] == "dense"]
    assert len(dense) == 2 and sorted(c.get("pair", False) for c in dense) == [False, True]
