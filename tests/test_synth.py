"""Seeded generators: reproducible, right shapes and value structure."""
import numpy as np

from paper_2004_11227_amd import synth


def test_reproducible():
    a = synth.config_inputs("c0")["caps"]
    b = synth.config_inputs("c0")["caps"]
    assert np.array_equal(a, b)
    c = synth.config_inputs("c0", run=1)["caps"]
    assert not np.array_equal(a, c)


def test_shapes_and_structure():
    c0 = synth.config_inputs("c0")
    assert c0["caps"].shape == (2, 128, 128)
    assert np.all(c0["caps"] >= 0)
    img, truth = synth.voronoi_image(64, 80, 4, 0.0, 7)
    assert set(np.unique(truth)) <= {0, 1, 2, 3}
    assert np.allclose(img, truth / 3.0)
    caps = synth.potts_caps(img, 4)
    assert caps.shape == (4, 64, 80)
    assert np.array_equal(caps.argmin(0), truth)
    vol = synth.ellipsoid_volume(16, 16, 16, 5, 0.0, 3)
    assert set(np.unique(vol)) <= {0.2, 0.8}


def test_random_state_admissible():
    caps = synth.config_inputs("c0", size=(20, 24))["caps"]
    st = synth.random_state((20, 24), 2, "two", 0.5, caps, seed=5)
    nrm = np.sqrt((st["q"] ** 2).sum(1))
    assert nrm.max() <= 0.5 + 1e-12
    assert np.all(st["q"][:, 0, :, -1] == 0) and np.all(st["q"][:, 1, -1, :] == 0)
    assert np.all(st["ps"] <= caps[0]) and np.all(st["p"][0] <= caps[1])


def test_serving_trace():
    tr = synth.serving_trace(200, seed=1, rate=100.0)
    assert len(tr) == 200
    assert all(64 <= r.shape[0] <= 2048 for r in tr if r.ndim == 2)
    assert all(r.shape == (128, 128, 128) for r in tr if r.ndim == 3)
    arr = [r.arrival for r in tr]
    assert arr == sorted(arr)
