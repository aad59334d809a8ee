"""rPDRQ at the benchmark sizes, in the launch configurations the benchmark
times: the fused 2-D pass on the two-label 2048^2 workload and the Potts
n = 4 1024^2 workload, and the in-place launches on the 256^3 volume.

After a few iterations from the initial point, sampled cells (interior,
edges, corners) are compared with the FP64 oracle run on a window around
each one, clipped to the grid.  One rPDRQ iteration moves information at
most 5 cells (b: 1, three half-sweeps: 3, flows: 1), so a window of radius
R > 5 x iterations gives the sample its whole-grid values.  The red-black
colouring follows the parity of the global coordinates, so every window
starts at even coordinates."""
import numpy as np
import pytest
import torch

import oracle
from paper_2004_11227_amd import synth

from _gpu import banner, gpu_solver, need_gpu, oracle_problem

pytestmark = pytest.mark.gpu

TOL = 5e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _points(shape, rng, n=16):
    corners = [tuple(0 if b == 0 else s - 1 for b, s in zip(bits, shape))
               for bits in np.ndindex(*(2,) * len(shape))]
    mids = [tuple(s // 2 for s in shape)]
    rand = [tuple(int(rng.integers(0, s)) for s in shape) for _ in range(n)]
    return corners + mids + rand


def _check(caps32, s, kw, iters, pts, R):
    shape = caps32.shape[1:]
    nd = len(shape)
    u = s.read("u").cpu().numpy()
    q = s.read("q").cpu().numpy()
    ps = s.read("ps").cpu().numpy()
    p = s.read("p").cpu().numpy()
    L = u.shape[0]
    q = q.reshape((L, nd) + shape)
    ps = ps.reshape(shape)
    worst = 0.0
    for pt in pts:
        lo = [max(0, c - R) & ~1 for c in pt]   # even origin: the colouring of the whole grid
        hi = [min(n, c + R + 1) for c, n in zip(pt, shape)]
        win = tuple(slice(a, b) for a, b in zip(lo, hi))
        c = caps32[(slice(None),) + win].astype(np.float64)
        pr = oracle_problem(c.shape[1:], kw)
        st = oracle.init_state(pr, c)
        oracle.step(pr, c, st, iters)
        loc = tuple(c_ - a for c_, a in zip(pt, lo))
        errs = [np.abs(u[(slice(None),) + pt] - st.u[(slice(None),) + loc]).max(),
                np.abs(q[(slice(None), slice(None)) + pt] - st.q[(slice(None), slice(None)) + loc]).max(),
                abs(ps[pt] - st.ps[loc]),
                np.abs(p[(slice(None),) + pt] - st.p[(slice(None),) + loc]).max()]
        worst = max(worst, max(errs))
        assert max(errs) < TOL, (pt, errs)
    print(f"worst |gpu - oracle| over {len(pts)} samples: {worst:.2e}")


def test_two_label_2048_fused():
    banner("pdrq full size: two-label 2048^2, fused pass, 3 iterations")
    caps = synth.config_inputs("c1")["caps"].astype(np.float32)
    kw = dict(model="two", method="dr", alpha=0.5)
    s = gpu_solver(caps, **kw)
    s.step(3)
    torch.cuda.synchronize()
    _check(caps, s, kw, 3, _points(caps.shape[1:], np.random.default_rng(21)), R=18)
    s.close()


def test_potts4_1024_fused():
    banner("pdrq full size: Potts n=4 1024^2, fused pass, 3 iterations")
    caps = synth.config_inputs("c2n4")["caps"].astype(np.float32)
    kw = dict(model="potts", nlabels=4, method="dr", alpha=0.3)
    s = gpu_solver(caps, **kw)
    s.step(3)
    torch.cuda.synchronize()
    _check(caps, s, kw, 3, _points(caps.shape[1:], np.random.default_rng(22)), R=18)
    s.close()


def test_two_label_3d_256_inplace():
    banner("pdrq full size: two-label 256^3, in-place launches, 2 iterations")
    caps = synth.config_inputs("c3")["caps"].astype(np.float32)
    kw = dict(model="two", method="dr", alpha=0.4)
    s = gpu_solver(caps, **kw)
    s.step(2)
    torch.cuda.synchronize()
    _check(caps, s, kw, 2, _points(caps.shape[1:], np.random.default_rng(23), n=10), R=12)
    s.close()
    torch.cuda.empty_cache()
