"""The autotune cache's host side: keys group pools by device and size
class, and the JSON file survives missing, damaged and concurrent-looking
use (a missing or unreadable file is a miss; a write keeps other keys)."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import paper_2404_06359_amd as P  # noqa: E402


def test_keys_bucket_the_workload():
    k = P.tune_key("gfx950", 256, P.FORMAT_REUSE, 2000, 613847054, 7425035)
    assert k == "gfx950/cu256/reuse/m2^11/t2^29/tpm80"
    # within a bucket: the same key; across: different
    assert P.tune_key("gfx950", 256, P.FORMAT_REUSE, 1900, 600000000, 7300000) == k
    assert P.tune_key("gfx950", 256, P.FORMAT_GTS, 2000, 613847054, 7425035) != k
    assert P.tune_key("gfx950", 304, P.FORMAT_REUSE, 2000, 613847054, 7425035) != k
    assert P.tune_key("gfx942", 256, P.FORMAT_REUSE, 2000, 613847054, 7425035) != k
    assert P.tune_key("gfx950", 256, P.FORMAT_REUSE, 200, 613847054, 7425035) != k
    assert P.tune_key("gfx950", 256, P.FORMAT_REUSE, 2000, 77937631, 851612) != k
    assert P.tune_key("gfx950", 256, P.FORMAT_REUSE, 0, 0, 0) == "gfx950/cu256/reuse/m2^-1/t2^-1/tpm0"


def test_cache_file_round_trip(tmp_path):
    path = str(tmp_path / "tune.json")
    assert P.tune_cache_get(path, "a") is None                     # no file yet
    rec = {"target_tris": 1536, "cfg": {"waves_per_group": 1, "groups_per_cu": 512, "run_tris": 1280,
                                        "items_per_claim": 0}, "best": {"median_ms": 0.55}}
    P.tune_cache_put(path, "a", rec)
    assert P.tune_cache_get(path, "a") == rec
    assert P.tune_cache_get(path, "b") is None
    P.tune_cache_put(path, "b", dict(rec, target_tris=768))
    assert P.tune_cache_get(path, "a") == rec                       # other keys kept
    assert P.tune_cache_get(path, "b")["target_tris"] == 768
    data = json.load(open(path))
    assert data["version"] == 1 and set(data["entries"]) == {"a", "b"}
    assert [f for f in os.listdir(tmp_path)] == ["tune.json"]       # no temporary left behind


def test_damaged_cache_is_a_miss_and_is_replaced(tmp_path):
    path = str(tmp_path / "tune.json")
    for text in ("{not json", "[1, 2]", '{"entries": 5}', '{"entries": {"a": {"cfg": {}}}}'):
        with open(path, "w") as f:
            f.write(text)
        assert P.tune_cache_get(path, "a") is None
    rec = {"target_tris": 384, "cfg": {}, "best": {}}
    with open(path, "w") as f:
        f.write("{not json")
    P.tune_cache_put(path, "a", rec)
    assert P.tune_cache_get(path, "a") == rec
