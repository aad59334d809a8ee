"""Seeded synthetic inputs shaped like the paper's segmentation workloads.

The paper's experiments (Section 4, Tables 1-2) segment natural images that are
not distributed with it, and it does not state image sizes or how the data
capacities were built.  These generators stand in for them:

* two-label images: a union of random ellipses (value 0.8) on a 0.2
  background plus Gaussian noise; capacities C_s = |I - 0.2|, C_t = |I - 0.8|
  (the data term of the relaxed min-cut model, eq. ``seg:chanvese``);
* 3-D volumes: the same with random ellipsoids;
* multi-label images: a Voronoi partition whose cells carry a random label k
  with intensity c_k = k/(L-1), plus noise; Potts data costs
  C_k = (I - c_k)^2 (the rho(l_i, x) of eq. ``potts-model``);
* random admissible iterates (flows inside their constraint sets) for
  one-step tests.

This module holds no arithmetic of the solver: it only draws numbers.  Both
the FP64 oracle (under ``oracle/``) and the GPU path consume its arrays.  All
randomness comes from numpy's PCG64 with an explicit seed.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "ellipse_image", "ellipsoid_volume", "voronoi_image",
    "two_label_caps", "potts_caps", "voronoi_two_label_caps",
    "config_inputs", "random_state", "serving_trace", "Request",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def ellipse_image(h: int, w: int, k: int, sigma: float, seed: int,
                  bg: float = 0.2, fg: float = 0.8) -> np.ndarray:
    """Union of ``k`` random filled ellipses on a constant background + noise.

    Centres are uniform over the image, semi-axes U[0.04, 0.20] * S * sqrt(3/k)
    with S = min(h, w), orientation U[0, pi).  Pixel centres sit at integer
    coordinates.  Noise is N(0, sigma^2), not clipped.  Returns float64 (h, w).
    """
    rng = _rng(seed)
    img = np.full((h, w), bg, dtype=np.float64)
    s = float(min(h, w))
    scale = math.sqrt(3.0 / max(k, 1))
    for _ in range(k):
        cy = rng.uniform(0, h)
        cx = rng.uniform(0, w)
        ra = rng.uniform(0.04, 0.20) * s * scale
        rb = rng.uniform(0.04, 0.20) * s * scale
        th = rng.uniform(0, math.pi)
        rmax = max(ra, rb)
        y0, y1 = max(0, int(cy - rmax) - 1), min(h, int(cy + rmax) + 2)
        x0, x1 = max(0, int(cx - rmax) - 1), min(w, int(cx + rmax) + 2)
        if y0 >= y1 or x0 >= x1:
            continue
        yy, xx = np.mgrid[y0:y1, x0:x1]
        dy = yy - cy
        dx = xx - cx
        ct, st = math.cos(th), math.sin(th)
        e1 = (dx * ct + dy * st) / ra
        e2 = (-dx * st + dy * ct) / rb
        inside = e1 * e1 + e2 * e2 <= 1.0
        img[y0:y1, x0:x1][inside] = fg
    img += rng.normal(0.0, sigma, size=(h, w))
    return img


def ellipsoid_volume(d: int, h: int, w: int, k: int, sigma: float, seed: int,
                     bg: float = 0.2, fg: float = 0.8) -> np.ndarray:
    """Union of ``k`` random ellipsoids (random rotation) + noise; (d, h, w)."""
    rng = _rng(seed)
    vol = np.full((d, h, w), bg, dtype=np.float64)
    s = float(min(d, h, w))
    scale = (3.0 / max(k, 1)) ** (1.0 / 3.0)
    for _ in range(k):
        c = np.array([rng.uniform(0, d), rng.uniform(0, h), rng.uniform(0, w)])
        radii = rng.uniform(0.04, 0.20, size=3) * s * scale
        g = rng.normal(size=(3, 3))
        qm, rm = np.linalg.qr(g)
        qm = qm * np.sign(np.diag(rm))[None, :]
        rmax = float(radii.max())
        lo = [max(0, int(c[i] - rmax) - 1) for i in range(3)]
        hi = [min(n, int(c[i] + rmax) + 2) for i, n in enumerate((d, h, w))]
        if any(lo[i] >= hi[i] for i in range(3)):
            continue
        zz, yy, xx = np.mgrid[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]]
        pts = np.stack([zz - c[0], yy - c[1], xx - c[2]], axis=-1)
        loc = pts @ qm
        inside = ((loc / radii) ** 2).sum(-1) <= 1.0
        vol[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]][inside] = fg
    vol += rng.normal(0.0, sigma, size=vol.shape)
    return vol


def voronoi_image(h: int, w: int, nlabels: int, sigma: float, seed: int,
                  ncells: int = 64):
    """Voronoi partition with ``ncells`` uniform seeds (Euclidean nearest seed,
    ties to the lower seed index); each cell gets label k ~ U{0..L-1} with
    intensity c_k = k/(L-1).  Returns (image + noise, truth labels int32)."""
    rng = _rng(seed)
    sy = rng.uniform(0, h, size=ncells)
    sx = rng.uniform(0, w, size=ncells)
    cell_label = rng.integers(0, nlabels, size=ncells)
    truth = np.empty((h, w), dtype=np.int32)
    xs = np.arange(w, dtype=np.float64)
    rows = max(1, (1 << 22) // max(1, w * ncells))
    for y0 in range(0, h, rows):
        y1 = min(h, y0 + rows)
        ys = np.arange(y0, y1, dtype=np.float64)
        d2 = ((ys[:, None, None] - sy[None, None, :]) ** 2
              + (xs[None, :, None] - sx[None, None, :]) ** 2)
        truth[y0:y1] = cell_label[np.argmin(d2, axis=-1)]
    levels = np.arange(nlabels, dtype=np.float64) / max(1, nlabels - 1)
    img = levels[truth] + rng.normal(0.0, sigma, size=(h, w))
    return img, truth


def two_label_caps(img: np.ndarray, lo: float = 0.2, hi: float = 0.8) -> np.ndarray:
    """Stack [C_s, C_t] = [|I - lo|, |I - hi|]; shape (2,) + img.shape."""
    return np.stack([np.abs(img - lo), np.abs(img - hi)]).astype(np.float64)


def potts_caps(img: np.ndarray, nlabels: int) -> np.ndarray:
    """Stack of C_k = (I - k/(L-1))^2 for k = 0..L-1; shape (L,) + img.shape."""
    levels = np.arange(nlabels, dtype=np.float64) / max(1, nlabels - 1)
    return np.stack([(img - c) ** 2 for c in levels]).astype(np.float64)


def voronoi_two_label_caps(img: np.ndarray) -> np.ndarray:
    """Two-label capacities for a two-level Voronoi image: C_s=(I-0)^2, C_t=(I-1)^2."""
    return np.stack([(img - 0.0) ** 2, (img - 1.0) ** 2]).astype(np.float64)


def config_inputs(name: str, run: int = 0, size=None):
    """Named workloads.  Returns dict(model, shape, caps, alpha, iters, ...).

    * ``c0``: two-label 128x128, 3 ellipses, sigma 0.1, alpha 0.5, 300 its
    * ``c1``: two-label 2048x2048, 40 ellipses, sigma 0.15, alpha 0.5, 500 its
    * ``c2n4`` / ``c2n8``: Potts 1024x1024 Voronoi, L = 4 / 8, sigma 0.15,
      alpha 0.3, 800 its
    * ``c3``: two-label 3-D 256^3, 20 ellipsoids, sigma 0.1, alpha 0.4

    ``size`` overrides the spatial shape (same generator, e.g. a smaller
    version for CPU tests or 4096^2 for a working set above the last-level
    cache).  Seed = config index * 1000 + run.
    """
    if name == "c0":
        h, w = size or (128, 128)
        img = ellipse_image(h, w, 3, 0.1, 0 * 1000 + run)
        return dict(model="two", shape=(h, w), caps=two_label_caps(img), alpha=0.5,
                    iters=300, nlabels=2, image=img)
    if name == "c1":
        h, w = size or (2048, 2048)
        img = ellipse_image(h, w, 40, 0.15, 1 * 1000 + run)
        return dict(model="two", shape=(h, w), caps=two_label_caps(img), alpha=0.5,
                    iters=500, nlabels=2, image=img)
    if name in ("c2n4", "c2n8"):
        n = 4 if name == "c2n4" else 8
        h, w = size or (1024, 1024)
        img, truth = voronoi_image(h, w, n, 0.15, 2 * 1000 + run)
        return dict(model="potts", shape=(h, w), caps=potts_caps(img, n), alpha=0.3,
                    iters=800, nlabels=n, image=img, truth=truth)
    if name == "c3":
        d, h, w = size or (256, 256, 256)
        vol = ellipsoid_volume(d, h, w, 20, 0.1, 3 * 1000 + run)
        return dict(model="two", shape=(d, h, w), caps=two_label_caps(vol), alpha=0.4,
                    iters=1000, nlabels=2, image=vol)
    raise KeyError(name)


def random_state(shape, nlabels: int, model: str, alpha: float, caps: np.ndarray,
                 seed: int, spread: float = 1.0):
    """A random admissible iterate for one-step tests.

    Flows q have |q(x)|_2 <= alpha pointwise (uniform radius fraction and
    random direction) and a zero component wherever the forward neighbour along
    that axis is outside the grid; the source/sink flows lie below their
    capacities; u is uniform in [-0.25, 1.25].  Returns a dict of float64
    arrays: u (L, *shape), q (L, ndim, *shape), ps (*shape), p (L, *shape),
    where L = 1 for the two-label model (p holds p_t).
    """
    rng = _rng(seed)
    ndim = len(shape)
    nl = 1 if model == "two" else nlabels
    dirs = rng.normal(size=(nl, ndim) + tuple(shape))
    nrm = np.sqrt((dirs ** 2).sum(axis=1, keepdims=True)) + 1e-30
    rad = rng.uniform(0.0, 1.0, size=(nl, 1) + tuple(shape)) * alpha
    q = dirs / nrm * rad
    for k in range(ndim):
        axis = ndim - 1 - k          # component k is the k-th fastest axis
        sl = [slice(None)] * ndim
        sl[axis] = -1
        q[(slice(None), k) + tuple(sl)] = 0.0
    u = rng.uniform(-0.25, 1.25, size=(nl,) + tuple(shape))
    if model == "two":
        cs, ct = caps[0], caps[1]
        ps = cs - rng.uniform(0, spread, size=shape)
        p = (ct - rng.uniform(0, spread, size=shape))[None]
    else:
        p = caps - rng.uniform(0, spread, size=caps.shape)
        ps = caps.min(axis=0) + rng.normal(0, spread, size=shape)
    return dict(u=u, q=q, ps=ps, p=p)


@dataclass
class Request:
    rid: int
    arrival: float
    ndim: int
    shape: tuple
    model: str
    nlabels: int
    kind: str
    sigma: float
    alpha: float
    seed: int


def serving_trace(nreq: int = 2048, seed: int = 4000, rate: float | None = None,
                  lo: int = 64, hi: int = 2048, frac3d: float = 0.1, side3d: int = 128):
    """Request mix for the serving workload: 2-D square sides log-uniform on
    [lo, hi] (integers, not tile aligned), ``frac3d`` of requests 3-D
    side3d^3 (two-label), L uniform on {2,3,4,8}, image kind ellipse/Voronoi
    50/50, sigma ~ U[0.05, 0.2], alpha ~ U[0.2, 0.6].  Arrival times are a
    Poisson process of the given rate (all zero when rate is None)."""
    rng = _rng(seed)
    out = []
    t = 0.0
    for i in range(nreq):
        if rate is not None:
            t += rng.exponential(1.0 / rate)
        is3d = rng.uniform() < frac3d
        n = int(rng.choice([2, 3, 4, 8]))
        kind = "ellipse" if rng.uniform() < 0.5 else "voronoi"
        sig = float(rng.uniform(0.05, 0.2))
        alp = float(rng.uniform(0.2, 0.6))
        if is3d:
            shape = (side3d, side3d, side3d)
            n = 2
            kind = "ellipse"
        else:
            side = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
            shape = (side, side)
        model = "two" if n == 2 else "potts"
        out.append(Request(i, t, len(shape), shape, model, n, kind, sig, alp,
                           int(rng.integers(0, 2**31 - 1))))
    return out


def request_caps(req: Request) -> np.ndarray:
    """Capacities for one serving request (float64)."""
    if req.ndim == 3:
        vol = ellipsoid_volume(*req.shape, 20, req.sigma, req.seed)
        return two_label_caps(vol)
    h, w = req.shape
    if req.kind == "ellipse":
        img = ellipse_image(h, w, 10, req.sigma, req.seed)
        if req.model == "two":
            return two_label_caps(img)
        return potts_caps(img, req.nlabels)
    img, _ = voronoi_image(h, w, req.nlabels, req.sigma, req.seed, ncells=32)
    if req.model == "two":
        return voronoi_two_label_caps(img)
    return potts_caps(img, req.nlabels)
