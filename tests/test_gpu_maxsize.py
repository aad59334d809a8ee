"""Largest sizes: workspaces whose element offsets pass 2^31.

Two-label 16384^2 (12 planes of 2^28 elements: 3.2e9 elements, through
the depth-2 pass) and Potts n = 8 at 8192^2 (74 planes of 2^26: 5e9
elements).  The capacities tile a seeded 1024^2 stand-in image.  After a
few iterations from the initial point, sampled pixels (interior, edges,
corners) are compared with the FP64 oracle run on the window of radius 12
around each one, clipped to the image: the window's own edges lie farther
from the sample than the dependency cone of those iterations reaches
(at most 3 cells per iteration), so the sample's values are the whole-grid
values, and the clipped sides are the true image edges."""
import numpy as np
import pytest
import torch

import oracle
from paper_2004_11227_amd import synth

from _gpu import banner, gpu_solver, need_gpu, oracle_problem

pytestmark = pytest.mark.gpu

R = 12


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _samples(H, W, rng, n=24):
    pts = [(0, 0), (0, W - 1), (H - 1, 0), (H - 1, W - 1), (H // 2, 0), (0, W // 2), (H - 1, W // 2),
           (H // 2, W - 1), (H - 1, W - 3)]
    pts += [(int(rng.integers(0, H)), int(rng.integers(0, W))) for _ in range(n)]
    return pts


def _check(caps32, s, kw, iters, pts, model, n):
    H, W = caps32.shape[1:]
    u = s.read("u").cpu().numpy()
    q = s.read("q").cpu().numpy()
    ps = s.read("ps").cpu().numpy()
    p = s.read("p").cpu().numpy()
    L = u.shape[0]
    for (y, x) in pts:
        y0, y1 = max(0, y - R), min(H, y + R + 1)
        x0, x1 = max(0, x - R), min(W, x + R + 1)
        c = caps32[:, y0:y1, x0:x1].astype(np.float64)
        pr = oracle_problem(c.shape[1:], kw)
        st = oracle.init_state(pr, c)
        oracle.step(pr, c, st, iters)
        yy, xx = y - y0, x - x0
        assert abs(u[:, y, x] - st.u[:, yy, xx]).max() < 2e-5, (y, x, "u")
        assert abs(q.reshape(L, 2, H, W)[:, :, y, x] - st.q[:, :, yy, xx]).max() < 2e-5, (y, x, "q")
        assert abs(ps[0, y, x] - st.ps[yy, xx]) < 2e-5, (y, x, "ps")
        assert abs(p[:, y, x] - st.p[:, yy, xx]).max() < 2e-5, (y, x, "p")


def test_two_label_16384():
    banner("max size: two-label 16384^2, depth 2, 4 iterations")
    tile = synth.config_inputs("c1", size=(1024, 1024))["caps"].astype(np.float32)
    caps = np.tile(tile, (1, 16, 16))
    kw = dict(model="two", method="eb", relax=1.5, alpha=0.5, depth=2)
    s = gpu_solver(caps, **kw)
    s.step(4)
    torch.cuda.synchronize()
    _check(caps, s, kw, 4, _samples(16384, 16384, np.random.default_rng(5)), "two", 2)
    s.close()
    torch.cuda.empty_cache()


def test_potts8_8192():
    banner("max size: Potts n=8 8192^2, 3 iterations")
    img, _ = synth.voronoi_image(1024, 1024, 8, 0.15, 2008)
    tile = synth.potts_caps(img, 8).astype(np.float32)
    caps = np.tile(tile, (1, 8, 8))
    kw = dict(model="potts", nlabels=8, method="eb", relax=1.5, alpha=0.3)
    s = gpu_solver(caps, **kw)
    s.step(3)
    torch.cuda.synchronize()
    _check(caps, s, kw, 3, _samples(8192, 8192, np.random.default_rng(6)), "potts", 8)
    s.close()
    torch.cuda.empty_cache()
