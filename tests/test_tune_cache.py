"""The autotuner's on-disk cache (host logic only) and helm_autotune's argument checks
(rejected before any launch)."""
import ctypes
import json

import numpy as np
import pytest

from paper_1208_3956_amd import _lib as L
from paper_1208_3956_amd import tune


def test_key_separates_shapes():
    a = tune.key("MI355X", "mixed", "reduced", (2032, 2032, 1), [62, 61], 64)
    assert a != tune.key("MI355X", "mixed", "reduced", (2032, 2032, 1), [62, 61], 32)
    assert a != tune.key("MI355X", "c128", "reduced", (2032, 2032, 1), [62, 61], 64)
    assert a != tune.key("MI355X", "mixed", "reduced", (2032, 2032, 1), [61, 62], 64)


def test_store_and_lookup(tmp_path):
    p = str(tmp_path / "sub" / "tune.json")
    k = tune.key("dev", "mixed", "reduced", (10, 10, 1), [5], 2)
    assert tune.lookup(p, k) is None
    tune.store(p, k, 24, {16: 1.5, 24: 1.25})
    assert tune.lookup(p, k) == 24
    data = json.load(open(p))
    assert data[k]["ms_per_apply"] == {"16": 1.5, "24": 1.25}
    k2 = tune.key("dev", "c128", "reduced", (10, 10, 1), [5], 2)
    tune.store(p, k2, 32, {})
    assert tune.lookup(p, k) == 24 and tune.lookup(p, k2) == 32


def test_corrupt_cache_is_a_miss(tmp_path):
    p = tmp_path / "tune.json"
    p.write_text("{not json")
    assert tune.lookup(str(p), "x") is None
    p.write_text(json.dumps({"x": {"chunk_rows": 1}}))
    assert tune.lookup(str(p), "x") is None


def test_cache_path_default_and_env(monkeypatch):
    monkeypatch.delenv("HELM_TUNE_CACHE", raising=False)
    assert tune.cache_path(None) is None
    assert tune.cache_path("default").endswith("tune.json")
    monkeypatch.setenv("HELM_TUNE_CACHE", "/tmp/x.json")
    assert tune.cache_path("default") == "/tmp/x.json"
    assert tune.cache_path("/a/b.json") == "/a/b.json"


def test_autotune_null_handle_and_bad_arguments():
    lib = L.lib()
    cand = (ctypes.c_int * 2)(16, 32)
    assert lib.helm_autotune(None, 1, ctypes.c_void_p(1), cand, 2, 1, None, None) == L.HELM_EINVAL
    # a handle whose setup completed: bad candidate lists are rejected before any launch
    c = np.ones((12, 12))
    o = L.helm_default_opts(12, 12)
    o.pml_outer, o.pml_iface = 4, 3
    try:
        h = L.helm_setup(c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 2 * np.pi * 5, 0.05, o, 2)
    except L.HelmError as e:          # no GPU in this process: setup cannot upload the tables
        pytest.skip(f"setup needs a device: {e}")
    try:
        bad = (ctypes.c_int * 2)(16, 1)
        assert lib.helm_autotune(h, 1, ctypes.c_void_p(1), bad, 2, 1, None, None) == L.HELM_EINVAL
        assert lib.helm_autotune(h, 1, ctypes.c_void_p(1), cand, 0, 1, None, None) == L.HELM_EINVAL
        assert lib.helm_autotune(h, 0, ctypes.c_void_p(1), cand, 2, 1, None, None) == L.HELM_EINVAL
    finally:
        L.lib().helm_destroy(h)
