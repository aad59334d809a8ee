"""Host logic of the tuning cache (no GPU): keys, round trip through the
JSON file, miss behaviour."""
import json

from paper_2004_11227_amd import tuning


def test_key_separates_classes():
    k1 = tuning.key((1024, 1024), None, model="potts", nlabels=4, storage="f32")
    k2 = tuning.key((1024, 1024), None, model="potts", nlabels=4, storage="bf16")
    k3 = tuning.key((1024, 1000), None, model="potts", nlabels=4, storage="f32")   # same size bucket
    k4 = tuning.key((2048, 2048), None, model="potts", nlabels=4, storage="f32")
    k5 = tuning.key((64, 64, 64), None, model="two")
    assert k1 != k2 and k1 == k3 and k1 != k4
    assert "|3d|" in k5 and "|2|" in k5


def test_store_lookup_round_trip(tmp_path, monkeypatch):
    path = tmp_path / "t.json"
    monkeypatch.setenv("MF_TUNING_CACHE", str(path))
    tuning.clear()
    assert tuning.lookup((512, 512), None, model="two") is None
    tuning.store((512, 512), None, 8, {8: 10.0, 16: 12.0, 32: 15.0}, model="two")
    assert tuning.lookup((512, 512), None, model="two") == 8
    d = json.loads(path.read_text())
    (k, v), = d.items()
    assert v["tile_rows"] == 8 and v["us_per_sweep"]["16"] == 12.0
    tuning.clear()   # re-read from the file
    assert tuning.lookup((500, 520), None, model="two") == 8
    assert tuning.lookup((512, 512), None, model="two", storage="bf16") is None
    tuning.clear()
