"""Host logic of the autotuner: keys, size buckets, cache round trip, choice."""
import os

from paper_2306_17263_amd import autotune as at


def test_size_bucket():
    assert at.size_bucket(8) == 16
    assert at.size_bucket(16) == 16
    assert at.size_bucket(17) == 32
    assert at.size_bucket(2048) == 2048


def test_key_is_order_independent():
    a = at.make_key("dev", "single", 2, 300, {"lap_mode": "tracked", "closure": "paper"})
    b = at.make_key("dev", "single", 2, 500, {"closure": "paper", "lap_mode": "tracked"})
    assert a == b                      # same bucket, same settings


def test_cache_round_trip(tmp_path, monkeypatch):
    path = str(tmp_path / "sub" / "cache.json")
    monkeypatch.setenv("C4M_TUNE_CACHE", path)
    assert at.load_cache() == {}
    at.store_cache("k1", {"tile_x": 2})
    at.store_cache("k2", {"tile_x": 0, "tile_y": 2})
    data = at.load_cache()
    assert data["k1"] == {"tile_x": 2} and data["k2"]["tile_y"] == 2
    with open(path, "w") as f:
        f.write("not json")
    assert at.load_cache() == {}
    assert os.path.exists(path)


def test_pick_best():
    assert at.pick_best({(0, 1): 3.0, (1, 1): 2.0, (2, 2): 2.5}) == (1, 1)
