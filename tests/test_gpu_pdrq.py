"""GPU parity of rPDRQ (in-place red-black half-sweeps) against the FP64 oracle."""
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


@pytest.mark.parametrize("shape", [(128, 128), (77, 131), (1, 64), (64, 1), (2, 2)])
def test_two_label_2d(shape):
    banner(f"pdrq two-label {shape}")
    caps = synth.config_inputs("c0", size=shape)["caps"]
    du, dis, g, st = compare_run(caps, 150, model="two", method="dr", alpha=0.5)
    print(f"max|du|={du:.3e} dis={dis:.2e}")
    assert du <= 1e-4 and dis <= 1e-3
    for f in ("zq", "zs", "zp"):
        assert np.max(np.abs(g[f] - getattr(st, f))) <= 1e-4


@pytest.mark.parametrize("n", [2, 3, 4, 8])
def test_potts_2d(n):
    banner(f"pdrq potts n={n}")
    img, _ = synth.voronoi_image(90, 110, n, 0.15, 2100 + n, ncells=16)
    caps = synth.potts_caps(img, n)
    du, dis, _, _ = compare_run(caps, 150, model="potts", nlabels=n, method="dr", alpha=0.3)
    print(f"max|du|={du:.3e} dis={dis:.2e}")
    assert du <= 1e-4 and dis <= 1e-3


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
