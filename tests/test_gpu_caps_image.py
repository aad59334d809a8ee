"""Capacities generated from one image plane (cap_source="image"):
C_k(x) = |I(x) - levels[k]|^power, evaluated in FP32 inside the kernels.

* With FP32 storage every path (fused depth 1 and 2, Potts, 3-D, unfused,
  rPDRQ fused and in place, pADMM-TY, ALG1) gives, bit for bit, the iterates
  of the same solver fed the capacity planes computed with the same FP32
  operations here (a subtraction, then abs or a product: IEEE-exact, so
  numpy float32 reproduces them).
* Against the FP64 oracle run on the capacities computed in FP64 from the
  same image: the FP32 bar; with BF16 storage (the image rounded to BF16)
  the BF16 bar of the precision tests.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2004_11227_amd import synth

from _gpu import banner, gpu_fields, gpu_solver, label_disagreement, need_gpu, oracle_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _caps32(img, levels, power):
    """The kernels' FP32 evaluation of |I - l|^power, plane by plane."""
    I = img.astype(np.float32)
    out = []
    for l in levels:
        d = I - np.float32(l)
        out.append(np.abs(d) if power == 1 else d * d)
    return np.stack(out).astype(np.float32)


def _caps64(img, levels, power):
    I = img.astype(np.float64)
    return np.stack([np.abs(I - l) ** power for l in levels])


CASES = [
    # (name, shape, model, n, kw)
    ("two 2d depth2 p1", (77, 131), "two", 2, dict(method="eb", relax=1.5, alpha=0.5)),
    ("two 2d depth1 p2", (77, 131), "two", 2, dict(method="fg", alpha=0.5, depth=1)),
    ("two 2d tile8", (65, 64), "two", 2, dict(method="eb", alpha=0.4, depth=1, tile_rows=8)),
    ("potts3 2d", (66, 97), "potts", 3, dict(method="eb", alpha=0.3)),
    ("potts8 2d", (40, 70), "potts", 8, dict(method="fg", alpha=0.2)),
    ("two 3d", (19, 21, 70), "two", 2, dict(method="eb", relax=1.5, alpha=0.4)),
    ("two 2d unfused", (50, 83), "two", 2, dict(method="eb", alpha=0.5, variant="unfused")),
    ("potts4 3d unfused", (9, 12, 21), "potts", 4, dict(method="eb", alpha=0.3)),
    ("dr two fused", (70, 133), "two", 2, dict(method="dr", alpha=0.5)),
    ("dr potts3", (48, 61), "potts", 3, dict(method="dr", alpha=0.3)),
    ("dr two M2", (48, 61), "two", 2, dict(method="dr", alpha=0.5, gs_sweeps=2)),
    ("ty potts3", (48, 61), "potts", 3, dict(method="ty", alpha=0.3)),
    ("cp two", (48, 61), "two", 2, dict(method="cp", alpha=0.5)),
]


@pytest.mark.parametrize("power", [1, 2])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_image_equals_planes_bitwise(case, power):
    name, shape, model, n, kw = case
    banner(f"image caps {name} power={power}")
    rng = np.random.default_rng(sum(shape) + 7 * n + power)
    if len(shape) == 3:
        img = synth.ellipsoid_volume(*shape, 4, 0.1, 4000)
    else:
        img = rng.uniform(0, 1, shape)
    img = img.astype(np.float32)
    levels = [0.2, 0.8] if model == "two" else list(np.linspace(0.0, 1.0, n))
    kw = dict(kw, model=model, nlabels=n, tol=0.0, max_iter=23, check_every=5)
    a = gpu_solver(_caps32(img, levels, power), **kw)
    b = gpu_solver(img[None], cap_source="image", cap_power=power, levels=levels, **kw)
    ra, rb = a.solve(), b.solve()
    torch.cuda.synchronize()
    assert ra["iter"] == rb["iter"] and ra["rel_gap"] == rb["rel_gap"] and ra["primal"] == rb["primal"]
    fa, fb = gpu_fields(a), gpu_fields(b)
    for f in fa:
        assert np.array_equal(fa[f], fb[f]), f
    ga, gb = a.gap(), b.gap()
    assert ga["rel_gap"] == gb["rel_gap"] and ga["dual"] == gb["dual"]
    a.close()
    b.close()


@pytest.mark.parametrize("model,n,power", [("two", 2, 1), ("potts", 4, 2)])
def test_image_mode_matches_oracle(model, n, power):
    banner(f"image caps vs oracle {model} n={n}")
    shape = (96, 130)
    if model == "two":
        img = synth.ellipse_image(*shape, 3, 0.1, 4001)
        levels = [0.2, 0.8]
    else:
        img, _ = synth.voronoi_image(*shape, n, 0.15, 4002, ncells=16)
        levels = list(np.linspace(0.0, 1.0, n))
    img = img.astype(np.float32)
    kw = dict(model=model, nlabels=n, method="eb", alpha=0.4)
    s = gpu_solver(img[None], cap_source="image", cap_power=power, levels=levels, **kw)
    s.step(200)
    g = gpu_fields(s)
    s.close()
    caps = _caps64(img, levels, power)
    pr = oracle_problem(shape, kw)
    st = oracle.init_state(pr, caps)
    oracle.step(pr, caps, st, 200)
    du = float(np.max(np.abs(g["u"] - st.u)))
    dis = label_disagreement(g["u"], st.u, model)
    print(f"max|du|={du:.3e} label disagreement={dis:.2e}")
    assert du <= 1e-4 and dis <= 1e-3


@pytest.mark.parametrize("model,n", [("two", 2), ("potts", 8)])
def test_image_mode_bf16(model, n):
    """BF16 storage rounds the image; the capacities are then evaluated in
    FP32 from the rounded image.  Objective error and label disagreement
    against the FP64 oracle on the capacities of the unrounded image."""
    banner(f"image caps bf16 {model} n={n}")
    shape = (160, 192)
    if model == "two":
        img = np.random.default_rng(4003).uniform(0, 1, shape)
        levels, alpha = [0.2, 0.8], 0.5
    else:
        img, _ = synth.voronoi_image(*shape, n, 0.15, 4004, ncells=24)
        levels, alpha = list(np.linspace(0.0, 1.0, n)), 0.3
    img = img.astype(np.float32)
    kw = dict(model=model, nlabels=n, method="eb", alpha=alpha)
    s = gpu_solver(img[None], storage="bf16", cap_source="image", cap_power=2, levels=levels, **kw)
    s.step(300)
    g = gpu_fields(s)
    s.close()
    caps = _caps64(img, levels, 2)
    pr = oracle_problem(shape, kw)
    st = oracle.init_state(pr, caps)
    oracle.step(pr, caps, st, 300)
    e = oracle.energy(pr, caps, st)
    eb = oracle.energy(pr, caps, oracle.state_from_arrays(pr, g["u"], st.q, st.ps, st.p))
    obj_err = abs(eb["primal"] - e["primal"]) / abs(e["primal"])
    dis = label_disagreement(g["u"], st.u, model)
    print(f"bf16 image objective rel err={obj_err:.3e} label disagreement={dis:.3e}")
    assert obj_err < 5e-3 and dis < 0.02
