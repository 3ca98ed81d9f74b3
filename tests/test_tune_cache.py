"""The batched plan's JSON autotune cache (host logic, no device)."""
import json
import os

import pytest

from paper_2006_06281_amd import tune_cache as tc


def test_bucket_is_ceil_log2():
    assert [tc.bucket(n) for n in (0, 1, 2, 3, 4, 5, 1024, 1025, 50000)] == \
        [0, 0, 1, 2, 2, 3, 10, 11, 16]


def test_batch_key_fields():
    k = tc.batch_key("gfx950", [500, 1500], [700, 700], 3, "fp32")
    # mean M 1000 -> 10, mean N 700 -> 10, two instances -> 1
    assert k == "gfx950|batch|M10|N10|D3|fp32|B1"
    assert tc.batch_key("gfx950", [3000] * 256, [6000] * 256) == "gfx950|batch|M12|N13|D3|fp32|B8"
    assert tc.batch_key("gfx942", [3000], [6000]) != tc.batch_key("gfx950", [3000], [6000])
    with pytest.raises(ValueError):
        tc.batch_key("gfx950", [1, 2], [3])
    with pytest.raises(ValueError):
        tc.batch_key("gfx950", [], [])


def test_round_trip_and_replace(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    c = tc.TuneCache(path)
    assert c.get("k") is None and len(c) == 0
    c.put("k", {"candidate": 3, "chunk": 2048, "tile": 512})
    c.put("j", {"candidate": 0})
    assert c.get("k") == {"candidate": 3, "chunk": 2048, "tile": 512}
    c.put("k", {"candidate": 5})
    assert tc.TuneCache(path).get("k") == {"candidate": 5} and len(c) == 2
    with open(path) as f:
        data = json.load(f)
    assert data["version"] == tc.VERSION and set(data["entries"]) == {"j", "k"}
    # no temporary files left beside it
    assert sorted(os.listdir(os.path.dirname(path))) == ["tune.json"]


def test_unreadable_or_foreign_file_is_ignored_then_rewritten(tmp_path):
    path = str(tmp_path / "tune.json")
    with open(path, "w") as f:
        f.write("{not json")
    c = tc.TuneCache(path)
    with pytest.warns(UserWarning):
        assert c.get("k") is None
    with pytest.warns(UserWarning):
        c.put("k", {"candidate": 1})
    assert c.get("k") == {"candidate": 1}
    with open(path, "w") as f:
        json.dump({"version": 999, "entries": {"k": {"candidate": 2}}}, f)
    with pytest.warns(UserWarning):
        assert c.get("k") is None
