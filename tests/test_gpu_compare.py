"""GPU parity of the paper's comparison methods (pADMM-TY and ALG1, on the
element-wise kernels) against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
from paper_2004_11227_amd import synth

from _gpu import banner, compare_run, gpu_fields, gpu_solver, need_gpu, oracle_problem

pytestmark = pytest.mark.gpu

TOL_U = 1e-4      # max |u - u_oracle| after the same iterations (FP32 path)
TOL_LAB = 1e-3    # fraction of pixels whose label differs


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


@pytest.mark.parametrize("method", ["ty", "cp"])
@pytest.mark.parametrize("shape", [(128, 128), (77, 131), (1, 64), (64, 1)])
def test_two_label_2d(method, shape):
    banner(f"{method} two-label {shape}")
    caps = synth.config_inputs("c0", size=shape)["caps"]
    du, dis, _, _ = compare_run(caps, 200, model="two", method=method, alpha=0.5)
    print(f"max|du|={du:.3e} dis={dis:.2e}")
    assert du <= TOL_U and dis <= TOL_LAB


@pytest.mark.parametrize("method", ["ty", "cp"])
@pytest.mark.parametrize("n", [3, 4, 8])
def test_potts_2d(method, n):
    banner(f"{method} potts n={n}")
    img, _ = synth.voronoi_image(90, 110, n, 0.15, 2200 + n, ncells=16)
    caps = synth.potts_caps(img, n)
    du, dis, _, _ = compare_run(caps, 150, model="potts", nlabels=n, method=method, alpha=0.3)
    print(f"max|du|={du:.3e} dis={dis:.2e}")
    assert du <= TOL_U and dis <= TOL_LAB


@pytest.mark.parametrize("method", ["ty", "cp"])
@pytest.mark.parametrize("model,n", [("two", 2), ("potts", 3)])
def test_3d(method, model, n):
    banner(f"{method} 3d {model}")
    vol = synth.ellipsoid_volume(17, 24, 29, 4, 0.1, 3010)
    caps = synth.two_label_caps(vol) if model == "two" else synth.potts_caps(vol, n)
    du, dis, _, _ = compare_run(caps, 80, model=model, nlabels=n, method=method, alpha=0.4)
    assert du <= TOL_U and dis <= TOL_LAB


@pytest.mark.parametrize("method", ["ty", "cp"])
def test_solve_stops_and_resumes(method):
    """solve() stops at a checked iterate with the oracle's gap there; a
    checkpoint (ALG1's u-bar included) resumes bit for bit."""
    banner(f"{method} solve")
    caps = synth.config_inputs("c0", size=(48, 64))["caps"].astype(np.float32).astype(np.float64)
    kw = dict(model="two", method=method, alpha=0.5, tol=1e-3, max_iter=4000, check_every=10)
    s = gpu_solver(caps, **kw)
    res = s.solve()
    assert res["status"] == 0 and res["iter"] % 10 == 0
    pr = oracle_problem(caps.shape[1:], kw)
    st = oracle.init_state(pr, caps)
    oracle.step(pr, caps, st, res["iter"])
    e = oracle.energy(pr, caps, st)
    assert abs(res["rel_gap"] - e["rel_gap"]) < 1e-5
    blob = s.export_state()
    k = s.iter
    s.step(7)
    a = gpu_fields(s)
    t = gpu_solver(caps, **{**kw, "tol": 0.0})
    t.import_state(blob, k)
    t.step(7)
    b = gpu_fields(t)
    for f in a:
        assert np.array_equal(a[f], b[f]), f
    s.close()
    t.close()


def test_alg1_step_bound_rejected():
    from paper_2004_11227_amd import maxflow as mfx
    caps = torch.ones((2, 8, 8), device="cuda")
    with pytest.raises(mfx.MaxflowError):
        mfx.Solver(caps, model="two", method="cp", sigma=0.5, tau=0.5)
    with pytest.raises(mfx.MaxflowError):
        mfx.Solver(caps, model="two", method="ty", relax=1.5)
