"""The autotuner's host logic: cache keys, the choice rule, the cache file."""
import json

import numpy as np

from paper_0902_3092_amd import autotune as A
from paper_0902_3092_amd import workloads as W


def test_shape_key_separates_shapes_and_decades():
    d = W.small_disk(n_r=12, n_mu=8, n_lambda=16)
    k = A.shape_key(d, 100000, precision="fp32", mrw=True)
    assert k == A.shape_key(d, 120000, precision="fp32", mrw=True)
    assert k != A.shape_key(d, 1000000, precision="fp32", mrw=True)
    assert k != A.shape_key(d, 100000, precision="fp64", mrw=True)
    assert k != A.shape_key(W.small_disk(n_r=13, n_mu=8, n_lambda=16), 100000,
                            precision="fp32", mrw=True)
    heavy = W.small_disk(M_dust_msun=1e-1, n_r=12, n_mu=8, n_lambda=16)
    assert k != A.shape_key(heavy, 100000, precision="fp32", mrw=True)


def test_pick_keeps_default_within_margin_and_skips_failures():
    t = {"a": 1.00, "b": 0.98, "c": 0.50}
    assert A.pick(t, {"a": True, "b": True, "c": False}, "a") == "a"   # b within 3 %
    assert A.pick(t, {"a": True, "b": True, "c": True}, "a") == "c"
    assert A.pick(t, {"a": False, "b": True, "c": False}, "a") == "b"  # default failed
    assert A.pick(t, {}, "a") == "a"                                   # nothing ran
    assert A.pick({"a": float("nan"), "b": 2.0}, {"a": True, "b": True}, "a") == "b"


def test_cache_roundtrip(tmp_path):
    p = str(tmp_path / "sub" / "tune.json")
    d = W.small_disk()
    assert A.options_for(d, 1000, path=p, precision="fp32") == {}
    key = A.shape_key(d, 1000, precision="fp32")
    A.store(key, {"key": key, "options": {"wave_events": 512, "pda_solver": 2}}, p)
    A.store("other", {"key": "other", "options": {}}, p)
    assert A.options_for(d, 1000, path=p, precision="fp32") == {"wave_events": 512,
                                                                 "pda_solver": 2}
    with open(p) as fh:
        assert set(json.load(fh)) == {key, "other"}
    # a damaged file reads as empty
    with open(p, "w") as fh:
        fh.write("{not json")
    assert A.load(p) == {}
