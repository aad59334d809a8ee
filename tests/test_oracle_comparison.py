"""Pins for the oracle's comparison methods (CPU only): the classical
sequential ADMM pADMM-TY (eqs. ADMM:Tai_yuan, mADMM:Tai_yuan) and the
Chambolle-Pock primal-dual algorithm ALG1 (appendix, eqs. iteration:pd:seg,
alg1:4labels).

What fixes the answers is independent of these two iterations:
* a saddle point of the max-flow problem, reached by the pinned rpADMMII
  iteration, is a fixed point of every one of these schemes (the KKT
  conditions: q* = P_alpha(q* - t grad u*) for t > 0, p_s* = min(C_s, p_s* +
  t (1 - u*)), p_i* = min(C_i, p_i* + t u_i*), conservation), so one step
  from it must not move it; a dropped term or a flipped sign moves it by
  O(1/c) or O(sigma);
* exhaustive minimisation over all labelings on tiny grids;
* the step-size bound of ALG1 (sigma tau |K^*K| < 1) checked with the
  oracle's own operators.
"""
import numpy as np
import pytest

import oracle
from paper_2004_11227_amd import synth


def _rand_caps(shape, seed, model="two", n=2):
    rng = np.random.default_rng(seed)
    img = rng.uniform(0, 1, size=shape)
    return synth.two_label_caps(img) if model == "two" else synth.potts_caps(img, n)


def _saddle(shape, caps, model, n, tv, alpha):
    """A saddle point: rpADMMII iterated until one more of its own steps moves
    no field by more than 1e-12 (a small gap alone is not enough: the gap can
    close while the conservation residual is still 1e-4)."""
    pr = oracle.Problem(shape, model=model, nlabels=n, method="eb", tv=tv, alpha=alpha)
    st = oracle.init_state(pr, caps)
    for _ in range(80):
        oracle.step(pr, caps, st, 5000)
        s1 = st.copy()
        oracle.step(pr, caps, s1, 1)
        if max(float(np.max(np.abs(getattr(st, f) - getattr(s1, f)))) for f in ("u", "q", "ps", "p")) < 1e-12:
            return st
    raise AssertionError("rpADMMII did not reach a fixed point")


@pytest.mark.parametrize("model,n,tv,shape", [("two", 2, "aniso", (5, 6)), ("two", 2, "iso", (6, 7)),
                                              ("potts", 3, "iso", (4, 5)), ("potts", 4, "aniso", (3, 5)),
                                              ("two", 2, "iso", (3, 3, 4))])
@pytest.mark.parametrize("method", ["ty", "cp"])
def test_saddle_point_is_a_fixed_point(model, n, tv, shape, method):
    caps = _rand_caps(shape, 11, model, n)
    alpha = 0.2
    st = _saddle(shape, caps, model, n, tv, alpha)
    pr = oracle.Problem(shape, model=model, nlabels=n, method=method, tv=tv, alpha=alpha)
    s1 = oracle.state_from_arrays(pr, st.u, st.q, st.ps, st.p)
    oracle.step(pr, caps, s1, 1)
    for f in ("u", "q", "ps", "p"):
        a, b = getattr(st, f), getattr(s1, f)
        assert np.max(np.abs(a - b)) < 1e-9 * max(1.0, np.max(np.abs(a))), f


@pytest.mark.parametrize("method", ["ty", "cp"])
@pytest.mark.parametrize("shape", [(4, 4), (2, 8), (2, 2, 4)])
def test_two_label_exact_vs_brute_force(shape, method):
    for seed, alpha in [(1, 0.15), (2, 0.3)]:
        caps = _rand_caps(shape, seed)
        best, blab, second = oracle.brute_force_binary(caps, alpha)
        pr = oracle.Problem(shape, model="two", method=method, tv="aniso", alpha=alpha)
        st, hist = oracle.solve(pr, caps, 60000, check_every=25, tol=1e-11)
        assert hist[-1][1]["rel_gap"] < 1e-10
        lab = oracle.labels(pr, st.u[0])
        assert abs(oracle.labeling_energy(caps, lab, alpha, "two") - best) < 1e-8
        if second > best + 1e-9:
            assert np.array_equal(lab, blab)


@pytest.mark.parametrize("method", ["ty", "cp"])
@pytest.mark.parametrize("L,shape", [(3, (2, 4)), (4, (2, 3))])
def test_potts_sandwich_vs_brute_force(L, shape, method):
    caps = _rand_caps(shape, 5, "potts", L)
    alpha = 0.1
    best = oracle.brute_force_potts(caps, alpha)[0]
    pr = oracle.Problem(shape, model="potts", nlabels=L, method=method, tv="aniso", alpha=alpha)
    st, hist = oracle.solve(pr, caps, 60000, check_every=25, tol=1e-11)
    e = hist[-1][1]
    assert e["rel_gap"] < 1e-9
    lab = oracle.labels(pr, st.u)
    assert e["primal"] <= best + 1e-8
    assert oracle.labeling_energy(caps, lab, alpha, "potts") >= best - 1e-8


@pytest.mark.parametrize("model,n", [("two", 2), ("potts", 4)])
def test_alg1_step_sizes_satisfy_the_bound(model, n):
    """sigma tau |K^*K| < 1 at the default steps, with |K^*K| from power
    iteration on K^*K u = -div grad u + (2 or n+1) u (the oracle's own
    grad/div)."""
    shape = (16, 16)
    pr = oracle.Problem(shape, model=model, nlabels=n, method="cp")
    m = 2.0 if model == "two" else n + 1.0
    rng = np.random.default_rng(3)
    u = rng.normal(size=shape)
    lam = 0.0
    for _ in range(400):
        v = -oracle.div(oracle.grad(u)) + m * u
        lam = float(np.sqrt((v * v).sum() / (u * u).sum()))
        u = v / np.linalg.norm(v)
    assert pr.sigma == 0.4
    assert pr.sigma * pr.tau * lam < 1.0
    assert pr.sigma * pr.tau * (8.0 + m) == pytest.approx(1.0)


def test_ty_potts_converges_on_a_voronoi_image():
    """The sequential pADMM-TY converges on a 4-label synthetic stand-in
    (with the old p_i in the p_s step the iterates grow without bound)."""
    img, _ = synth.voronoi_image(40, 50, 4, 0.15, 2204, ncells=16)
    caps = synth.potts_caps(img, 4)
    pr = oracle.Problem((40, 50), model="potts", nlabels=4, method="ty", alpha=0.3)
    st = oracle.init_state(pr, caps)
    oracle.step(pr, caps, st, 600)
    e = oracle.energy(pr, caps, st)
    assert e["rel_gap"] < 1e-3 and np.abs(st.u).max() < 2.0


def test_alg1_iterates_feasible_and_gap_nonnegative():
    shape = (9, 11)
    caps = _rand_caps(shape, 4)
    pr = oracle.Problem(shape, model="two", method="cp", alpha=0.3)
    st = oracle.init_state(pr, caps)
    for _ in range(60):
        oracle.step(pr, caps, st, 1)
        assert np.all(np.sqrt((st.q ** 2).sum(axis=1)) <= 0.3 * (1 + 1e-12))
        assert np.all(st.p[0] <= caps[1] + 1e-15) and np.all(st.ps <= caps[0] + 1e-15)
        assert oracle.energy(pr, caps, st)["rel_gap"] >= -1e-12


def _argmax_1d(f, lo, hi):
    """Maximiser of a concave scalar function on [lo, hi] by bounded Brent
    search (no closed form)."""
    from scipy.optimize import minimize_scalar
    r = minimize_scalar(lambda x: -f(x), bounds=(lo, hi), method="bounded", options={"xatol": 1e-12})
    return r.x


def test_ty_two_label_blocks_maximise_the_augmented_lagrangian():
    """pADMM-TY is block-sequential maximisation of the augmented Lagrangian
    L = <1, p_s> + <u, p_t - p_s + div q> - c/2 |p_t - p_s + div q|^2 (remark
    after eq. rpADMMI): p_s' maximises L over p_s <= C_s with p_t at p_t^k;
    p_t' maximises L over p_t <= C_t with p_s at p_s'.  Checked per pixel
    against a numerical maximiser, from a random admissible state."""
    shape = (4, 5)
    caps = _rand_caps(shape, 7)
    pr = oracle.Problem(shape, model="two", method="ty", alpha=0.3)
    rs = synth.random_state(shape, 2, "two", 0.3, caps, seed=8)
    st = oracle.state_from_arrays(pr, rs["u"], rs["q"], rs["ps"], rs["p"])
    s1 = st.copy()
    oracle.step(pr, caps, s1, 1)
    d = oracle.div(s1.q[0])
    c = pr.c
    cs, ct = caps
    for idx in np.ndindex(shape):
        u, pt0, dd = st.u[0][idx], st.p[0][idx], d[idx]
        lag = lambda ps, pt: ps + u * (pt - ps + dd) - 0.5 * c * (pt - ps + dd) ** 2
        ps1 = _argmax_1d(lambda x: lag(x, pt0), cs[idx] - 50.0, cs[idx])
        pt1 = _argmax_1d(lambda x: lag(ps1, x), ct[idx] - 50.0, ct[idx])
        assert abs(ps1 - s1.ps[idx]) < 1e-6 and abs(pt1 - s1.p[0][idx]) < 1e-6, idx


def test_ty_potts_blocks_maximise_the_augmented_lagrangian():
    """n labels (eq. mADMM:Tai_yuan, blocks q, p_i, p_s, u in sequence):
    p_i' maximises L = <1, p_s> + sum_i <u_i, div q_i + p_i - p_s> - c/2 sum_i
    |div q_i + p_i - p_s|^2 over p_i <= C_i with p_s at p_s^k, and p_s'
    maximises it over p_s with every p_i at its new value p_i'."""
    shape, n = (3, 4), 3
    caps = _rand_caps(shape, 9, "potts", n)
    pr = oracle.Problem(shape, model="potts", nlabels=n, method="ty", alpha=0.3)
    rs = synth.random_state(shape, n, "potts", 0.3, caps, seed=10)
    st = oracle.state_from_arrays(pr, rs["u"], rs["q"], rs["ps"], rs["p"])
    s1 = st.copy()
    oracle.step(pr, caps, s1, 1)
    d = np.stack([oracle.div(s1.q[i]) for i in range(n)])
    c = pr.c
    for idx in np.ndindex(shape):
        u = st.u[(slice(None),) + idx]
        p0 = st.p[(slice(None),) + idx]
        dd = d[(slice(None),) + idx]
        ps0 = st.ps[idx]

        def lag(p, ps):
            r = dd + p - ps
            return ps + float(np.dot(u, r)) - 0.5 * c * float(np.dot(r, r))
        for i in range(n):
            def f(x, i=i):
                p = p0.copy()
                p[i] = x
                return lag(p, ps0)
            pi = _argmax_1d(f, caps[(i,) + idx] - 50.0, caps[(i,) + idx])
            assert abs(pi - s1.p[(i,) + idx]) < 1e-6, (idx, i)
        p1 = s1.p[(slice(None),) + idx]
        ps1 = _argmax_1d(lambda x: lag(p1, x), ps0 - 50.0, ps0 + 50.0)
        assert abs(ps1 - s1.ps[idx]) < 1e-6, idx
