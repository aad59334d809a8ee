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
    k6 = tuning.key((64, 64, 64), None, model="two", slab_depth=16)
    k7 = tuning.key((64, 64), None, model="two", depth=1)
    assert k1 != k2 and k1 == k3 and k1 != k4
    assert "|3d|" in k5 and "|2|" in k5
    assert k5 != k6 and k7 != tuning.key((64, 64), None, model="two")


def test_store_lookup_round_trip(tmp_path, monkeypatch):
    path = tmp_path / "t.json"
    monkeypatch.setenv("MF_TUNING_CACHE", str(path))
    tuning.clear()
    assert tuning.lookup((512, 512), None, model="two") is None
    best = dict(tile_rows=16, depth=2, slab_depth=0)
    cands = [dict(tile_rows=8, depth=1, slab_depth=0, us_per_iter=30.0),
             dict(tile_rows=16, depth=2, slab_depth=0, us_per_iter=20.0)]
    tuning.store((512, 512), None, best, cands, model="two")
    assert tuning.lookup((512, 512), None, model="two") == best
    d = json.loads(path.read_text())
    (k, v), = d.items()
    assert v["choice"] == best and v["candidates"][1]["us_per_iter"] == 20.0
    tuning.clear()   # re-read from the file
    assert tuning.lookup((500, 520), None, model="two") == best
    assert tuning.lookup((512, 512), None, model="two", storage="bf16") is None
    tuning.clear()
