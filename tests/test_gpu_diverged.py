"""The divergence status through the C ABI: a non-finite gap (NaN or Inf
capacities) or a negative gap beyond what rounding of the stored flows
explains stops a solve with MF_EDIVERGED, and a diverging solve in the pool
retires with that status without changing any other solve's bits.

Weak duality (Section 2.1: the relaxed primal min-cut and the max-flow dual,
eqs. seg:chanvese / two-label-mf) gives P(u) >= D(q) whenever |q| <= alpha,
so a clearly negative gap means the flows left their constraint set."""
import numpy as np
import pytest
import torch

from paper_2004_11227_amd import maxflow as mfx
from paper_2004_11227_amd import synth

from _gpu import banner, gpu_solver, need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _caps(model, n, shape, seed):
    rng = np.random.default_rng(seed)
    img = rng.uniform(0, 1, size=shape)
    return synth.two_label_caps(img) if model == "two" else synth.potts_caps(img, n)


@pytest.mark.parametrize("bad", [np.nan, np.inf])
@pytest.mark.parametrize("model,n,method,variant,storage", [
    ("two", 2, "eb", "fused", "f32"), ("two", 2, "fg", "unfused", "f32"), ("two", 2, "eb", "fused", "bf16"),
    ("potts", 4, "eb", "fused", "f32"), ("potts", 3, "dr", "fused", "f32"), ("two", 2, "dr", "unfused", "f32")])
def test_non_finite_capacities_diverge(model, n, method, variant, storage, bad):
    banner(f"diverged {model} n={n} {method} {variant} {storage} {bad}")
    shape = (40, 70)
    caps = _caps(model, n, shape, 3).astype(np.float32)
    caps[0, 17, 33] = bad
    s = gpu_solver(caps, model=model, nlabels=n, method=method, variant=variant, storage=storage, alpha=0.3,
                   tol=1e-4, max_iter=200, check_every=10)
    g = s.solve()
    s.close()
    assert g["status"] == mfx.MF_EDIVERGED and g["iter"] == 0, g


def _infeasible_state(shape, alpha):
    """A step labeling u (0 on the left half, 1 on the right) with capacities
    that favour it, and a flux of magnitude 0.8 >> alpha pushed across the
    step: then sum min(C_s, C_t + div q) exceeds P(u) by about (0.8 - alpha)
    per row."""
    H, W = shape
    c = W // 2
    cs = np.where(np.arange(W)[None, :] < c, 0.2, 1.0) * np.ones(shape)
    ct = np.where(np.arange(W)[None, :] < c, 1.0, 0.2) * np.ones(shape)
    u = np.zeros((1,) + shape, np.float32)
    u[0, :, c:] = 1.0
    q = np.zeros((1, 2) + shape, np.float32)
    q[0, 0, :, c - 1] = -0.8          # x-flux between columns c-1 and c
    caps = np.stack([cs, ct]).astype(np.float32)
    # P and D of this state in numpy (isotropic TV of the step = H * 1)
    P = float(cs[:, :c].sum() + ct[:, c:].sum() + alpha * H)
    div = np.zeros(shape)
    div[:, c - 1] += q[0, 0, :, c - 1]
    div[:, c] -= q[0, 0, :, c - 1]
    D = float(np.minimum(cs, ct + div).sum())
    return caps, u, q, (P - D) / max(abs(P), abs(D))


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_negative_gap_diverges(storage):
    banner(f"negative gap {storage}")
    shape, alpha = (32, 32), 0.1
    caps, u, q, rel = _infeasible_state(shape, alpha)
    assert rel < -0.05
    s = gpu_solver(caps, model="two", alpha=alpha, storage=storage, tol=1e-4, max_iter=100, check_every=10)
    s.write("u", torch.from_numpy(u))
    s.write("q", torch.from_numpy(q.reshape(2, *shape)))
    g = s.gap()
    assert g["status"] == mfx.MF_EDIVERGED and g["rel_gap"] < -0.05, g
    assert abs(g["rel_gap"] - rel) < 2e-2 * abs(rel)
    r = s.solve()
    s.close()
    assert r["status"] == mfx.MF_EDIVERGED and r["iter"] == 0, r


def test_feasible_states_do_not_diverge():
    """The same step labeling with a flux inside the ball (|q| = alpha): the gap
    is non-negative, and a solve from the initial point converges."""
    banner("feasible state not diverged")
    shape, alpha = (32, 32), 0.1
    caps, u, q, _ = _infeasible_state(shape, alpha)
    q = np.clip(q, -alpha, alpha)
    s = gpu_solver(caps, model="two", alpha=alpha, tol=1e-4, max_iter=400, check_every=10)
    s.write("u", torch.from_numpy(u))
    s.write("q", torch.from_numpy(q.reshape(2, *shape)))
    g = s.gap()
    assert g["status"] == 0 and g["rel_gap"] >= -1e-7, g
    s.reset()
    r = s.solve()
    s.close()
    assert r["status"] in (0, 1) and r["rel_gap"] >= -1e-5, r


def _run(items):
    pool = mfx.Pool(1 << 28, max_slots=16, max_tiles=1 << 14, steps_per_advance=10)
    ids = [pool.admit(c, **kw) for c, kw in items]
    assert all(i is not None for i in ids)
    res = {}
    while len(res) < len(ids):
        pool.advance()
        for sid, g in pool.poll():
            u, lab = pool.retire(sid)
            res[sid] = (g, u.cpu().numpy(), lab.cpu().numpy())
    pool.close()
    return [res[i] for i in ids]


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_pool_diverging_solve_leaves_the_others_unchanged(storage):
    banner(f"pool diverged solve {storage}")
    items = []
    for i, (shape, model, n) in enumerate([((64, 96), "two", 2), ((70, 130), "potts", 4), ((20, 24, 37), "two", 2),
                                           ((90, 97), "potts", 3)]):
        caps = _caps(model, n, shape, 60 + i).astype(np.float32)
        kw = dict(model=model, nlabels=n, method="eb", alpha=0.35, storage=storage, tol=1e-4, max_iter=300,
                  check_every=10)
        items.append((torch.from_numpy(caps).cuda(), kw))
    bad = []
    for model, n, shape in (("two", 2, (50, 60)), ("potts", 4, (40, 70))):
        caps = _caps(model, n, shape, 9).astype(np.float32)
        caps[1, 5, 7] = np.nan
        bad.append((torch.from_numpy(caps).cuda(), dict(model=model, nlabels=n, method="eb", alpha=0.35,
                                                        storage=storage, tol=1e-4, max_iter=300, check_every=10)))
    mixed = _run(items[:2] + bad[:1] + items[2:] + bad[1:])
    order = [0, 1, None, 2, 3, None]
    for k, m in enumerate(mixed):
        if order[k] is None:
            assert m[0]["status"] == mfx.MF_EDIVERGED and m[0]["iter"] == 0, m[0]
            continue
        alone = _run([items[order[k]]])[0]
        assert m[0]["iter"] == alone[0]["iter"] and m[0]["status"] == alone[0]["status"]
        assert np.array_equal(m[1], alone[1]) and np.array_equal(m[2], alone[2])
