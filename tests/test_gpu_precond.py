"""GPU parity of the preconditioner variants against the FP64 oracle:
several symmetric red-black Gauss-Seidel sweeps per rPDRQ iteration (M_n),
a non-decreasing relaxation schedule for rpADMMII, and preconditioner
parameters above their minimums (a > 4 ndim, a~ > 2, a1 > 2, a2 > 2n).

Bar (FP32 storage): max |u - u_oracle| <= 1e-4 and thresholded-label
disagreement <= 0.1 % after the same number of iterations.
"""
import numpy as np
import pytest
import torch

from paper_2004_11227_amd import maxflow, synth

from _gpu import banner, compare_run, gpu_fields, gpu_solver, need_gpu

pytestmark = pytest.mark.gpu

TOL_U = 1e-4
TOL_LAB = 1e-3


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


@pytest.mark.parametrize("sweeps", [2, 3, 4, 6])
@pytest.mark.parametrize("case", ["two-2d", "two-3d", "potts3-2d", "potts4-3d"])
def test_pdrq_gs_sweeps(case, sweeps):
    banner(f"pdrq M_{sweeps} {case}")
    if case == "two-2d":
        caps = synth.config_inputs("c0", size=(77, 131))["caps"]
        kw = dict(model="two", alpha=0.5)
    elif case == "two-3d":
        caps = synth.two_label_caps(synth.ellipsoid_volume(13, 17, 29, 3, 0.1, 3101))
        kw = dict(model="two", alpha=0.4)
    elif case == "potts3-2d":
        img, _ = synth.voronoi_image(66, 97, 3, 0.15, 3102, ncells=12)
        caps = synth.potts_caps(img, 3)
        kw = dict(model="potts", nlabels=3, alpha=0.3)
    else:
        caps = synth.potts_caps(synth.ellipsoid_volume(10, 12, 21, 4, 0.1, 3103), 4)
        kw = dict(model="potts", nlabels=4, alpha=0.3)
    du, dis, g, st = compare_run(caps, 80, method="dr", gs_sweeps=sweeps, **kw)
    print(f"max|du|={du:.3e} label disagreement={dis:.2e}")
    assert du <= TOL_U and dis <= TOL_LAB
    for f in ("zq", "zs", "zp"):
        err = np.max(np.abs(g[f] - getattr(st, f)))
        assert err <= 1e-3, (f, err)


@pytest.mark.parametrize("storage", ["f32", "bf16"])
@pytest.mark.parametrize("model,n,sweeps", [("two", 2, 2), ("two", 2, 3), ("two", 2, 4), ("potts", 3, 2),
                                            ("potts", 3, 3), ("potts", 8, 2), ("potts", 8, 3)])
def test_pdrq_fused_sweeps_equal_inplace_bitwise(sweeps, model, n, storage):
    """The fused 2-D pass with 2 to 4 sweeps (2 sweeps + 1 half-sweeps in LDS
    on shrinking regions; up to 4 for two labels, 3 for Potts) against the
    in-place launches: state and resolvent outputs bit for bit, on a ragged
    grid with edge and interior tiles."""
    banner(f"pdrq fused M_{sweeps} {model} n={n} {storage}")
    img = synth.ellipse_image(75, 141, 3, 0.15, 3106 + sweeps)
    caps = synth.two_label_caps(img) if model == "two" else synth.potts_caps(img, n)
    kw = dict(model=model, nlabels=n, method="dr", alpha=0.5 if model == "two" else 0.3, storage=storage,
              gs_sweeps=sweeps)
    ref = gpu_solver(caps, variant="unfused", **kw)
    fus = gpu_solver(caps, variant="fused", **kw)
    for k in (1, 4):
        ref.step(k)
        fus.step(k)
        a, b = gpu_fields(ref), gpu_fields(fus)
        for f in a:
            assert np.array_equal(a[f], b[f]), (k, f)
    ref.close()
    fus.close()


def test_pdrq_one_sweep_default_unchanged_and_fused():
    """gs_sweeps = 1 is the default and keeps the fused two-label 2-D pass;
    more sweeps give different iterates (the preconditioner is in effect)."""
    caps = synth.config_inputs("c0", size=(64, 96))["caps"]
    kw = dict(model="two", method="dr", alpha=0.5)
    a = gpu_solver(caps, **kw)
    b = gpu_solver(caps, gs_sweeps=1, **kw)
    c = gpu_solver(caps, gs_sweeps=2, **kw)
    for s in (a, b, c):
        s.step(9)
    torch.cuda.synchronize()
    fa, fb, fc = gpu_fields(a), gpu_fields(b), gpu_fields(c)
    for f in fa:
        assert np.array_equal(fa[f], fb[f]), f
    assert np.max(np.abs(fa["u"] - fc["u"])) > 1e-6
    for s in (a, b, c):
        s.close()


@pytest.mark.parametrize("variant", ["fused", "unfused"])
@pytest.mark.parametrize("model,n", [("two", 2), ("potts", 4)])
def test_eb_relaxation_schedule(model, n, variant):
    """rho_k rising from 0.6 to 1.9 over 25 iterations, 60 iterations; the
    two-label 2-D fused solver switches to depth-2 passes at k = 25."""
    banner(f"eb schedule {model} {variant}")
    if model == "two":
        caps = synth.config_inputs("c0", size=(90, 120))["caps"]
    else:
        img, _ = synth.voronoi_image(80, 100, n, 0.15, 3104, ncells=14)
        caps = synth.potts_caps(img, n)
    du, dis, _, _ = compare_run(caps, 60, model=model, nlabels=n, method="eb", relax=1.9, relax0=0.6,
                                relax_ramp=25, alpha=0.4, variant=variant)
    print(f"max|du|={du:.3e} label disagreement={dis:.2e}")
    assert du <= TOL_U and dis <= TOL_LAB


def test_eb_schedule_depth2_equals_depth1_bitwise():
    """Depth-2 passes begin once rho_k is constant, and give the depth-1
    iterates bit for bit, also across a stepwise run and a solve."""
    caps = synth.config_inputs("c0", size=(70, 133))["caps"]
    kw = dict(model="two", method="eb", relax=1.9, relax0=0.5, relax_ramp=7, alpha=0.5)
    ref = gpu_solver(caps, depth=1, **kw)
    ref.step(23)
    d2 = gpu_solver(caps, depth=2, **kw)
    for n in (3, 1, 6, 13):
        d2.step(n)
    a, b = gpu_fields(ref), gpu_fields(d2)
    for f in a:
        assert np.array_equal(a[f], b[f]), f
    ref.close()
    d2.close()
    s1 = gpu_solver(caps, depth=1, tol=0.0, max_iter=41, check_every=10, **kw)
    s2 = gpu_solver(caps, depth=2, tol=0.0, max_iter=41, check_every=10, **kw)
    r1, r2 = s1.solve(), s2.solve()
    assert r1["iter"] == r2["iter"] == 41 and r1["rel_gap"] == r2["rel_gap"]
    a, b = gpu_fields(s1), gpu_fields(s2)
    for f in a:
        assert np.array_equal(a[f], b[f]), f
    s1.close()
    s2.close()


@pytest.mark.parametrize("model,n,pre", [("two", 2, dict(a=12.0, a_tilde=3.0)),
                                         ("two", 2, dict(a=9.0)),
                                         ("potts", 3, dict(a=10.0, a1=2.5, a2=8.0))])
@pytest.mark.parametrize("method", ["fg", "eb"])
def test_larger_preconditioner_parameters(model, n, pre, method):
    banner(f"{method} {model} {pre}")
    if model == "two":
        caps = synth.config_inputs("c0", size=(80, 111))["caps"]
    else:
        img, _ = synth.voronoi_image(72, 90, n, 0.15, 3105, ncells=12)
        caps = synth.potts_caps(img, n)
    du, dis, _, _ = compare_run(caps, 80, model=model, nlabels=n, method=method, alpha=0.4, **pre)
    assert du <= TOL_U and dis <= TOL_LAB
