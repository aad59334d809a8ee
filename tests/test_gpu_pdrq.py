"""GPU parity of rPDRQ against the FP64 oracle: the fused tiled pass
(2-D, two-label and Potts) and the in-place red-black launches (the unfused
variant, 3-D and several sweeps); and the two giving the same bits."""
import numpy as np
import pytest
import torch

import oracle
from paper_2004_11227_amd import synth

from _gpu import banner, compare_run, gpu_fields, gpu_solver, need_gpu, oracle_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


@pytest.mark.parametrize("variant", ["fused", "unfused"])
@pytest.mark.parametrize("shape", [(128, 128), (77, 131), (1, 64), (64, 1), (2, 2)])
def test_two_label_2d(shape, variant):
    banner(f"pdrq two-label {shape} {variant}")
    caps = synth.config_inputs("c0", size=shape)["caps"]
    du, dis, g, st = compare_run(caps, 150, model="two", method="dr", alpha=0.5, variant=variant)
    print(f"max|du|={du:.3e} dis={dis:.2e}")
    assert du <= 1e-4 and dis <= 1e-3
    for f in ("zq", "zs", "zp"):
        assert np.max(np.abs(g[f] - getattr(st, f))) <= 1e-4


@pytest.mark.parametrize("variant", ["fused", "unfused"])
@pytest.mark.parametrize("n", [2, 3, 4, 8])
def test_potts_2d(n, variant):
    banner(f"pdrq potts n={n} {variant}")
    img, _ = synth.voronoi_image(90, 110, n, 0.15, 2100 + n, ncells=16)
    caps = synth.potts_caps(img, n)
    du, dis, g, st = compare_run(caps, 150, model="potts", nlabels=n, method="dr", alpha=0.3, variant=variant)
    print(f"max|du|={du:.3e} dis={dis:.2e}")
    assert du <= 1e-4 and dis <= 1e-3
    for f in ("zq", "zs", "zp"):
        assert np.max(np.abs(g[f] - getattr(st, f))) <= 1e-4


@pytest.mark.parametrize("model,n", [("two", 2), ("potts", 4)])
def test_3d(model, n):
    banner(f"pdrq 3d {model} n={n}")
    vol = synth.ellipsoid_volume(17, 24, 29, 4, 0.1, 3002)
    caps = synth.two_label_caps(vol) if model == "two" else synth.potts_caps(vol, n)
    du, dis, _, _ = compare_run(caps, 80, model=model, nlabels=n, method="dr", alpha=0.4)
    assert du <= 1e-4 and dis <= 1e-3


def test_solve_gap_on_resolvent_outputs():
    banner("pdrq solve")
    caps = synth.config_inputs("c0", size=(48, 64))["caps"].astype(np.float32).astype(np.float64)
    kw = dict(model="two", method="dr", alpha=0.5, tol=1e-3, max_iter=3000, check_every=10)
    s = gpu_solver(caps, **kw)
    res = s.solve()
    assert res["status"] == 0 and res["iter"] % 10 == 0
    k = res["iter"]
    s.close()
    pr = oracle_problem(caps.shape[1:], kw)
    st = oracle.init_state(pr, caps)
    oracle.step(pr, caps, st, k)
    e = oracle.energy(pr, caps, st)
    assert abs(res["rel_gap"] - e["rel_gap"]) < 1e-5
    assert e["rel_gap"] <= 1.5e-3


@pytest.mark.parametrize("storage", ["f32", "bf16"])
@pytest.mark.parametrize("shape", [(1, 1), (3, 70), (70, 3), (33, 130), (200, 333)])
@pytest.mark.parametrize("model,n", [("two", 2), ("potts", 3)])
def test_fused_equals_inplace_bitwise(model, n, storage, shape):
    """The tiled pass (ping-pong buffers) and the three in-place launches give
    the same bits: state and resolvent outputs, odd and even step counts,
    both tile heights."""
    banner(f"pdrq fused bitwise {model} n={n} {shape} {storage}")
    img = synth.ellipse_image(*shape, 3, 0.15, 3200)
    caps = synth.two_label_caps(img) if model == "two" else synth.potts_caps(img, n)
    kw = dict(model=model, nlabels=n, method="dr", alpha=0.5 if model == "two" else 0.3, storage=storage)
    ref = gpu_solver(caps, variant="unfused", **kw)
    runs = [gpu_solver(caps, variant="fused", tile_rows=tr, **kw) for tr in (16, 32)]
    for n in (1, 2, 5):
        ref.step(n)
        a = gpu_fields(ref)
        for s in runs:
            s.step(n)
            b = gpu_fields(s)
            for f in a:
                assert np.array_equal(a[f], b[f]), (n, s.params.tile_rows, f)
    for s in runs + [ref]:
        s.close()


@pytest.mark.parametrize("n", [2, 4, 8])
@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_potts_fused_equals_inplace_bitwise(n, storage):
    """Every Potts label count of the tiled pass against the in-place
    launches, on a ragged grid, with the resolvent outputs kept."""
    banner(f"pdrq potts fused bitwise n={n} {storage}")
    img, _ = synth.voronoi_image(75, 141, n, 0.15, 3300 + n, ncells=12)
    caps = synth.potts_caps(img, n)
    kw = dict(model="potts", nlabels=n, method="dr", alpha=0.3, storage=storage)
    ref = gpu_solver(caps, variant="unfused", **kw)
    runs = [gpu_solver(caps, variant="fused", tile_rows=tr, **kw) for tr in (16, 32)]
    for k in (1, 4, 9):
        ref.step(k)
        a = gpu_fields(ref)
        for s in runs:
            s.step(k)
            b = gpu_fields(s)
            for f in a:
                assert np.array_equal(a[f], b[f]), (k, s.params.tile_rows, f)
    for s in runs + [ref]:
        s.close()


@pytest.mark.parametrize("model,n", [("two", 2), ("potts", 4)])
def test_fused_solve_equals_inplace(model, n):
    banner(f"pdrq fused solve {model} n={n}")
    if model == "two":
        caps = synth.config_inputs("c0", size=(200, 170))["caps"]
        kw = dict(model="two", method="dr", alpha=0.5, tol=1e-3, max_iter=2000, check_every=10)
    else:
        img, _ = synth.voronoi_image(130, 170, n, 0.15, 3400, ncells=16)
        caps = synth.potts_caps(img, n)
        kw = dict(model="potts", nlabels=n, method="dr", alpha=0.3, tol=1e-3, max_iter=2000, check_every=10)
    out = []
    for variant in ("unfused", "fused"):
        s = gpu_solver(caps, variant=variant, **kw)
        r = s.solve()
        f = gpu_fields(s)
        s.step(3)
        out.append((r, f, gpu_fields(s)))
        s.close()
    (r1, f1, g1), (r2, f2, g2) = out
    assert r1["iter"] == r2["iter"] and r1["rel_gap"] == r2["rel_gap"] and r1["status"] == r2["status"]
    assert model != "two" or r1["status"] == 0
    for k in f1:
        assert np.array_equal(f1[k], f2[k]), k
        assert np.array_equal(g1[k], g2[k]), k
