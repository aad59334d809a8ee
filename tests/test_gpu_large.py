"""Parity at the largest sizes, beyond the 2-D rpADMM cases of
test_gpu_maxsize.py: element offsets past 2^31 and byte offsets past 2^32.

* two-label 768^3 (4.5e8 voxels; the six state fields of a buffer span
  2.7e9 elements), the fused 3-D sweep, 2 iterations;
* two-label 16384^2 (working set 11 GB: the streaming tile order and
  non-temporal stores), the fused rPDRQ pass, 2 iterations;
* Potts n = 8 at 8192^2 (the 33 planes of a state buffer span 2.2e9
  elements): the gap fused into the sweep, against its closed form.

Sampled cells (corners, the centre, seeded random ones) are compared with
the FP64 oracle run on a window around each one (clipped to the grid); one
rpADMM iteration moves information at most 3 cells (an rPDRQ one 5), so a
window of radius R > 3 (5) x iterations gives a sample its whole-grid
value.  The label kernel is checked at the same cells.  Capacities are
|I - l_k| (two labels, l = 0.2, 0.8) or |I - l_k|^2 (Potts, l_k evenly
spaced) of a seeded smooth pattern plus Gaussian noise (cheap to draw at
this size)."""
import numpy as np
import pytest
import torch

import oracle

from _gpu import banner, gpu_solver, need_gpu, oracle_problem, progress

pytestmark = pytest.mark.gpu

TOL = 5e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _caps(shape, seed, nlabels=0):
    rng = np.random.default_rng(seed)
    axes = np.meshgrid(*[np.linspace(0.0, 1.0, n, dtype=np.float32) for n in shape], indexing="ij", sparse=True)
    img = np.full(shape, 0.5, dtype=np.float32)
    img += np.float32(0.3) * np.sin(np.float32(6.3) * sum(axes[1:])) * np.cos(np.float32(5.1) * axes[0])
    img += rng.standard_normal(shape, dtype=np.float32) * np.float32(0.1)
    if not nlabels:
        caps = np.empty((2,) + shape, dtype=np.float32)
        np.abs(img - np.float32(0.2), out=caps[0])
        np.abs(img - np.float32(0.8), out=caps[1])
        return caps
    caps = np.empty((nlabels,) + shape, dtype=np.float32)
    for k in range(nlabels):
        np.subtract(img, np.float32((k + 0.5) / nlabels), out=caps[k])
        np.square(caps[k], out=caps[k])
    return caps


def _points(shape, rng, n=12):
    corners = [tuple(0 if b == 0 else s - 1 for b, s in zip(bits, shape))
               for bits in np.ndindex(*(2,) * len(shape))]
    return corners + [tuple(s // 2 for s in shape)] + [tuple(int(rng.integers(0, s)) for s in shape)
                                                        for _ in range(n)]


def _check(caps, s, kw, iters, pts, R):
    shape = caps.shape[1:]
    nd = len(shape)
    fields = {f: s.read(f) for f in ("u", "q", "ps", "p")}
    fields["q"] = fields["q"].view((s.L, nd) + shape)
    fields["ps"] = fields["ps"].view(shape)
    lab = s.labels()
    worst = 0.0
    for pt in pts:
        lo = [max(0, c - R) & ~1 for c in pt]   # even origin: rPDRQ's red-black colouring of the whole grid
        hi = [min(n, c + R + 1) for c, n in zip(pt, shape)]
        win = tuple(slice(a, b) for a, b in zip(lo, hi))
        c = caps[(slice(None),) + win].astype(np.float64)
        pr = oracle_problem(c.shape[1:], kw)
        st = oracle.init_state(pr, c)
        oracle.step(pr, c, st, iters)
        loc = tuple(c_ - a for c_, a in zip(pt, lo))
        g = {"u": fields["u"][(slice(None),) + pt].cpu().numpy(),
             "q": fields["q"][(slice(None), slice(None)) + pt].cpu().numpy(),
             "ps": float(fields["ps"][pt]), "p": fields["p"][(slice(None),) + pt].cpu().numpy()}
        errs = [np.abs(g["u"] - st.u[(slice(None),) + loc]).max(),
                np.abs(g["q"] - st.q[(slice(None), slice(None)) + loc]).max(),
                abs(g["ps"] - st.ps[loc]), np.abs(g["p"] - st.p[(slice(None),) + loc]).max()]
        worst = max(worst, max(errs))
        assert max(errs) < TOL, (pt, errs)
        assert int(lab[pt]) == int(oracle.labels(pr, st.u)[loc]), pt
    progress(f"worst |gpu - oracle| over {len(pts)} samples: {worst:.2e}")


def test_two_label_768_cubed():
    banner("large: two-label 768^3 fused 3-D sweep, 2 iterations")
    caps = _caps((768, 768, 768), 9100)
    kw = dict(model="two", method="eb", relax=1.5, alpha=0.4)
    s = gpu_solver(caps, **kw)
    s.step(2)
    torch.cuda.synchronize()
    _check(caps, s, kw, 2, _points(caps.shape[1:], np.random.default_rng(91)), R=8)
    s.close()
    del caps
    torch.cuda.empty_cache()


def test_two_label_16384_squared_pdrq():
    banner("large: two-label 16384^2, fused rPDRQ pass, 2 iterations")
    caps = _caps((16384, 16384), 9300)
    kw = dict(model="two", method="dr", alpha=0.5)
    s = gpu_solver(caps, **kw)
    s.step(2)
    torch.cuda.synchronize()
    _check(caps, s, kw, 2, _points(caps.shape[1:], np.random.default_rng(93)), R=12)
    s.close()
    del caps
    torch.cuda.empty_cache()


def test_potts8_8192_fused_gap_at_iterate_0():
    """The gap check fused into the Potts sweep at iterate 0, where it has a
    closed form: u = 0 projects to 1/n per label, so the primal is the mean
    data term and the TV term vanishes; q = 0, so the dual is the sum of the
    minimum capacities."""
    banner("large: Potts n=8 8192^2, the fused gap at iterate 0")
    n = 8
    caps = _caps((8192, 8192), 9400, nlabels=n)
    kw = dict(model="potts", nlabels=n, method="eb", relax=1.5, alpha=0.3)
    s = gpu_solver(caps, tol=10.0, max_iter=10, check_every=10, **kw)
    r = s.solve()
    s.close()
    assert r["iter"] == 0 and r["status"] == 0, r
    primal = sum(float(caps[k].sum(dtype=np.float64)) for k in range(n)) / n
    dual = float(caps.min(axis=0).sum(dtype=np.float64))
    progress(f"gap at iterate 0: primal {r['primal']:.10e} vs {primal:.10e}, dual {r['dual']:.10e} vs {dual:.10e}")
    assert abs(r["primal"] - primal) <= 1e-9 * primal and abs(r["dual"] - dual) <= 1e-9 * dual
    del caps
    torch.cuda.empty_cache()
