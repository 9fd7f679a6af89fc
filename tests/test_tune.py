"""Autotuner: database lookup (CPU) and a short tuning run that must keep
every output byte (GPU)."""
import numpy as np
import pytest

from paper_2108_04791_amd import tune


def test_length_bucket_and_lookup(tmp_path):
    assert tune.length_bucket(0) == 0 and tune.length_bucket(1) == 0
    assert tune.length_bucket(65536) == 16 and tune.length_bucket(65537) == 16
    db = {"entries": {"c2_mr64|24": {"config": {"mr_window": 3}},
                      "c2_mr64|16": {"config": {"mr_window": 2}},
                      "c1_uniform20|16": {"config": {"mr_window": 4}}}}
    assert tune.lookup(db, "c2_mr64", 1 << 23)["config"]["mr_window"] == 3
    assert tune.lookup(db, "c2_mr64", 1 << 15)["config"]["mr_window"] == 2
    assert tune.lookup(db, "c3_mixed", 100) is None
    p = str(tmp_path / "db.json")
    tune.save(db, p)
    assert tune.load(p) == db
    assert tune.load(str(tmp_path / "missing.json"))["entries"] == {}


def test_shipped_database_is_valid():
    db = tune.load()
    assert db["entries"], "the package ships a tuning database"
    keys = set(tune.SPACE) | {"sort_survivors", "rest_test", "wheel_log2"}
    for name, e in db["entries"].items():
        assert set(e["config"]) >= set(tune.SPACE), name
        assert set(e["config"]) <= keys, name
        assert e["ms"] <= e["default_ms"] * 1.0001


@pytest.mark.gpu
def test_tuning_run_keeps_bytes():
    import torch
    import paper_2108_04791_amd as isp
    import workloads as W
    a = torch.from_numpy(W.c3_mixed(200000, start=3).view(np.int64)).cuda()
    before = isp.get_config()
    res = tune.tune([a], reps=2, sweeps=1, log=lambda s: None)
    assert isp.get_config() == before
    assert res["ms"] <= res["default_ms"] and res["tried"] > 10
