"""Pins for the oracle's iterations (CPU only).

What fixes the answers here is independent of the oracle:
* exhaustive minimisation over all binary / Potts labelings on tiny grids
  (anisotropic TV counts cut edges, and thresholding a relaxed two-label
  minimiser is exact, remark after eq. seg:chanvese);
* a graph max-flow computed by scipy on larger grids (max-flow = min-cut);
* closed forms (alpha = 0; alpha above the total data imbalance);
* algebraic identities between methods (EB with rho = 1 equals FG with r = 1;
  Potts with two labels equals the two-label model with 2 alpha);
* the invariants of every iterate (|q| <= alpha, p <= C, weak duality).
"""
import numpy as np
import pytest

import oracle
from paper_2004_11227_amd import synth

METHODS = ["fg", "eb", "dr"]


def _rand_caps(shape, seed, model="two", n=2):
    rng = np.random.default_rng(seed)
    if model == "two":
        img = rng.uniform(0, 1, size=shape)
        return synth.two_label_caps(img)
    img = rng.uniform(0, 1, size=shape)
    return synth.potts_caps(img, n)


@pytest.mark.parametrize("shape", [(4, 4), (2, 8), (1, 16), (2, 2, 4)])
@pytest.mark.parametrize("method", METHODS)
def test_two_label_exact_vs_brute_force(shape, method):
    for seed, alpha in [(1, 0.15), (2, 0.3)]:
        caps = _rand_caps(shape, seed)
        best, blab, second = oracle.brute_force_binary(caps, alpha)
        pr = oracle.Problem(shape, model="two", method=method, tv="aniso", alpha=alpha)
        st, hist = oracle.solve(pr, caps, 40000, check_every=25, tol=1e-11)
        e = hist[-1][1]
        assert e["rel_gap"] < 1e-10
        lab = oracle.labels(pr, st.u[0])
        assert abs(oracle.labeling_energy(caps, lab, alpha, "two") - best) < 1e-8
        assert abs(e["dual"] - best) < 1e-8
        if second > best + 1e-9:
            assert np.array_equal(lab, blab)


def _scipy_maxflow_value(caps_int, alpha_int):
    """s-t max flow on the 4-neighbour grid graph: s->x (C_s), x->t (C_t),
    x<->y (alpha each way); integer capacities."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import maximum_flow
    cs, ct = caps_int
    shape = cs.shape
    n = cs.size
    s, t = n, n + 1
    rows, cols, vals = [], [], []
    idx = np.arange(n).reshape(shape)
    rows += [s] * n; cols += list(range(n)); vals += list(cs.ravel())
    rows += list(range(n)); cols += [t] * n; vals += list(ct.ravel())
    for ax in range(len(shape)):
        a = np.take(idx, np.arange(shape[ax] - 1), axis=ax).ravel()
        b = np.take(idx, np.arange(1, shape[ax]), axis=ax).ravel()
        rows += list(a) + list(b); cols += list(b) + list(a); vals += [alpha_int] * (2 * len(a))
    m = csr_matrix((np.array(vals, dtype=np.int32), (rows, cols)), shape=(n + 2, n + 2))
    return maximum_flow(m, s, t).flow_value


@pytest.mark.parametrize("shape", [(32, 32), (17, 23)])
def test_two_label_matches_graph_maxflow(shape):
    # capacities on a 1/1000 lattice so that the integer graph is exact
    rng = np.random.default_rng(11)
    img = rng.uniform(0, 1, size=shape)
    smooth = img.copy()
    caps = np.round(synth.two_label_caps(smooth) * 1000) / 1000
    alpha = 0.25
    value = _scipy_maxflow_value(np.round(caps * 1000).astype(np.int64), 250) / 1000.0
    for method in ["eb", "dr"]:
        pr = oracle.Problem(shape, model="two", method=method, tv="aniso", alpha=alpha)
        st, hist = oracle.solve(pr, caps, 60000, check_every=50, tol=1e-10)
        e = hist[-1][1]
        assert abs(e["dual"] - value) < 1e-6 * value
        lab = oracle.labels(pr, st.u[0])
        assert abs(oracle.labeling_energy(caps, lab, alpha, "two") - value) < 1e-6 * value


@pytest.mark.parametrize("L,shape", [(3, (2, 5)), (4, (2, 4)), (8, (1, 5)), (8, (2, 2)), (2, (4, 4))])
@pytest.mark.parametrize("method", METHODS)
def test_potts_sandwich_vs_brute_force(L, shape, method):
    for seed, alpha in [(21, 0.05), (22, 0.12)]:
        caps = _rand_caps(shape, seed, "potts", L)
        best, blab, second = oracle.brute_force_potts(caps, alpha)
        pr = oracle.Problem(shape, model="potts", nlabels=L, method=method, tv="aniso", alpha=alpha)
        st, hist = oracle.solve(pr, caps, 40000, check_every=25, tol=1e-11)
        e = hist[-1][1]
        assert e["rel_gap"] < 1e-9
        relaxed = e["primal"]
        lab = oracle.labels(pr, st.u)
        e_lab = oracle.labeling_energy(caps, lab, alpha, "potts")
        # relaxed optimum <= integral optimum <= energy of the rounded labeling
        assert relaxed <= best + 1e-8
        assert best <= e_lab + 1e-12
        integral = np.all(np.abs(st.u - np.round(st.u)) < 1e-6)
        if integral:
            assert abs(e_lab - best) < 1e-8
            assert abs(relaxed - best) < 1e-8


def test_potts_two_labels_equals_two_label_model_with_double_alpha():
    shape = (12, 10)
    rng = np.random.default_rng(31)
    img = rng.uniform(0, 1, size=shape)
    caps_p = synth.potts_caps(img, 2)                  # [C_1, C_2]
    caps_t = np.stack([caps_p[1], caps_p[0]])         # C_s = C_2, C_t = C_1
    alpha = 0.2
    pp = oracle.Problem(shape, model="potts", nlabels=2, method="eb", alpha=alpha)
    pt = oracle.Problem(shape, model="two", method="eb", alpha=2 * alpha)
    _, hp = oracle.solve(pp, caps_p, 30000, check_every=50, tol=1e-11)
    _, ht = oracle.solve(pt, caps_t, 30000, check_every=50, tol=1e-11)
    Pp, Pt = hp[-1][1]["primal"], ht[-1][1]["primal"]
    assert abs(Pp - Pt) < 1e-8 * abs(Pt)


@pytest.mark.parametrize("model", ["two", "potts"])
def test_eb_rho1_equals_fg_r1(model):
    shape = (9, 13)
    caps = _rand_caps(shape, 41, model, 3)
    kw = dict(model=model, nlabels=3, alpha=0.4, relax=1.0)
    a = oracle.Problem(shape, method="eb", **kw)
    b = oracle.Problem(shape, method="fg", **kw)
    sa, _ = oracle.solve(a, caps, 57)
    sb, _ = oracle.solve(b, caps, 57)
    for f in ("u", "q", "ps", "p"):
        assert np.max(np.abs(getattr(sa, f) - getattr(sb, f))) < 1e-12


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("model", ["two", "potts"])
def test_feasibility_and_weak_duality_every_iterate(method, model):
    shape = (14, 11)
    caps = _rand_caps(shape, 51, model, 4)
    pr = oracle.Problem(shape, model=model, nlabels=4, method=method, alpha=0.3)
    st = oracle.init_state(pr, caps)
    for k in range(60):
        oracle.step(pr, caps, st, 1)
        q = st.zq if method == "dr" else st.q
        nrm = np.sqrt((q ** 2).sum(1))
        assert nrm.max() <= pr.alpha * (1 + 1e-12)
        if method != "dr":
            if model == "two":
                assert np.all(st.ps <= caps[0] + 1e-15) and np.all(st.p[0] <= caps[1] + 1e-15)
            else:
                assert np.all(st.p <= caps + 1e-15)
        else:
            if model == "two":
                assert np.all(st.zs <= caps[0] + 1e-15) and np.all(st.zp[0] <= caps[1] + 1e-15)
            else:
                assert np.all(st.zp <= caps + 1e-15)
        e = oracle.energy(pr, caps, st)
        assert e["rel_gap"] >= -1e-12


@pytest.mark.parametrize("method", METHODS)
def test_cross_method_same_optimum_iso(method):
    shape = (32, 32)
    inp = synth.config_inputs("c0", size=shape)
    caps = inp["caps"]
    pr = oracle.Problem(shape, model="two", method=method, alpha=0.5)
    st, hist = oracle.solve(pr, caps, 60000, check_every=50, tol=1e-10)
    e = hist[-1][1]
    ref = oracle.Problem(shape, model="two", method="eb", alpha=0.5)
    _, h2 = oracle.solve(ref, caps, 60000, check_every=50, tol=1e-11)
    assert abs(e["primal"] - h2[-1][1]["primal"]) < 1e-8 * abs(h2[-1][1]["primal"])


@pytest.mark.parametrize("method", ["fg", "eb", "dr"])
def test_kkt_at_convergence(method):
    shape = (10, 12)
    caps = _rand_caps(shape, 61)
    pr = oracle.Problem(shape, model="two", method=method, tv="aniso", alpha=0.2)
    st, hist = oracle.solve(pr, caps, 200000, check_every=100, tol=1e-13)
    # continue until the conservation residual is small as well
    for _ in range(200):
        if oracle.energy(pr, caps, st)["resid_rms"] < 1e-9:
            break
        oracle.step(pr, caps, st, 200)
    e = oracle.energy(pr, caps, st)
    assert e["rel_gap"] < 1e-10 and e["resid_rms"] < 1e-8
    u = st.u[0]
    ps, pt = (st.zs, st.zp[0]) if method == "dr" else (st.ps, st.p[0])
    assert u.min() > -1e-6 and u.max() < 1 + 1e-6
    assert np.all(np.abs(pt[u > 1e-6] - caps[1][u > 1e-6]) < 1e-6)
    assert np.all(np.abs(ps[u < 1 - 1e-6] - caps[0][u < 1 - 1e-6]) < 1e-6)
    assert abs(e["flow"] - e["dual"]) < 1e-6 * e["dual"]


@pytest.mark.parametrize("method", METHODS)
def test_closed_form_alpha_zero(method):
    shape = (7, 9)
    caps = _rand_caps(shape, 71)
    pr = oracle.Problem(shape, model="two", method=method, alpha=0.0)
    st, hist = oracle.solve(pr, caps, 20000, check_every=20, tol=1e-12)
    e = hist[-1][1]
    pstar = np.minimum(caps[0], caps[1]).sum()
    assert abs(e["primal"] - pstar) < 1e-9 * pstar
    lab = oracle.labels(pr, st.u[0])
    assert np.array_equal(lab, (caps[1] < caps[0]).astype(np.int32))


@pytest.mark.parametrize("method", METHODS)
def test_closed_form_huge_alpha(method):
    # alpha >= sqrt(2) * sum |C_s - C_t|: every non-constant labeling pays
    # more in TV than it can save in data, so u* is constant.
    shape = (6, 5)
    caps = _rand_caps(shape, 81)
    alpha = np.sqrt(2) * np.abs(caps[0] - caps[1]).sum() * 1.01
    pr = oracle.Problem(shape, model="two", method=method, alpha=alpha)
    st, hist = oracle.solve(pr, caps, 60000, check_every=50, tol=1e-11)
    e = hist[-1][1]
    pstar = min(caps[0].sum(), caps[1].sum())
    assert abs(e["primal"] - pstar) < 1e-8 * pstar


def test_one_pixel_grid():
    caps = np.array([[[0.3]], [[0.9]]])
    pr = oracle.Problem((1, 1), model="two", method="eb", alpha=0.5)
    st, hist = oracle.solve(pr, caps, 5000, check_every=10, tol=1e-13)
    assert abs(hist[-1][1]["primal"] - 0.3) < 1e-12
    assert oracle.labels(pr, st.u[0])[0, 0] == 0


def _np_div(q):
    """Divergence of a flux field q (ndim, *shape) written with numpy: the
    backward difference of the forward-difference flux with zero flux through
    the boundary (so <grad u, q> = -<u, div q>)."""
    nd = q.shape[0]
    out = np.zeros(q.shape[1:])
    for k in range(nd):
        ax = nd - 1 - k   # component k belongs to the k-th fastest axis
        f = np.moveaxis(q[k], ax, 0).copy()
        f[-1] = 0.0
        d = f.copy()
        d[1:] -= f[:-1]
        out += np.moveaxis(d, 0, ax)
    return out


@pytest.mark.parametrize("method", ["fg", "eb", "dr", "ty", "cp"])
@pytest.mark.parametrize("model,n,shape", [("two", 2, (9, 13)), ("two", 2, (3, 4, 5)),
                                           ("potts", 3, (8, 11)), ("potts", 8, (6, 7))])
def test_initial_point_is_the_largest_flow_at_zero_q(method, model, n, shape):
    """The initial point (the paper states none; reading A10): u = 0, q = 0,
    and source/sink flows on the constraint set with zero conservation
    residual.  With q = 0 the constraints decouple per pixel: two labels
    p_t - p_s = 0, p_s <= C_s, p_t <= C_t; Potts p_i - p_s = 0, p_i <= C_i.
    The largest total source flow there (the dual objective sum p_s of eqs.
    two-label-mf / potts-mf restricted to q = 0) is reached exactly when p_s
    is the pointwise minimum capacity, so the point must be feasible, have
    zero residual, and carry that flow pixel by pixel."""
    caps = _rand_caps(shape, 81 + n, model, n)
    pr = oracle.Problem(shape, model=model, nlabels=n, method=method, alpha=0.3)
    st = oracle.init_state(pr, caps)
    L = 1 if model == "two" else n
    assert np.all(st.u == 0.0) and np.all(st.q == 0.0)
    cmin = caps.min(axis=0)
    if model == "two":
        assert np.all(st.ps <= caps[0]) and np.all(st.p[0] <= caps[1])
        resid = [st.p[0] - st.ps + _np_div(st.q[0])]
    else:
        assert np.all(st.p <= caps)
        resid = [_np_div(st.q[i]) + st.p[i] - st.ps for i in range(L)]
    assert max(float(np.abs(r).max()) for r in resid) == 0.0
    # the source flow is the largest one compatible with q = 0
    assert np.array_equal(st.ps, cmin)
    assert abs(st.ps.sum() - cmin.sum()) <= 1e-12 * cmin.sum()
    # and the oracle's own residual and dual agree with it
    e = oracle.energy(pr, caps, st)
    assert e["resid_rms"] == 0.0
    assert abs(e["flow"] - cmin.sum()) <= 1e-12 * cmin.sum()
    assert abs(e["dual"] - cmin.sum()) <= 1e-12 * cmin.sum()


@pytest.mark.parametrize("model,n,tv,shape", [("potts", 3, "iso", (4, 5)), ("potts", 4, "aniso", (3, 5)),
                                              ("two", 2, "iso", (6, 7))])
def test_eb_step_keeps_a_saddle_point_found_by_fg(model, n, tv, shape):
    """Reading A5 (coefficient 1 on p_i^{k+1} - p_s^{k+1} in the multi-label EB
    multiplier step, as in the general EB update): a saddle point reached by
    the FG scheme (r = 1, whose multiplier step has no such term) must be a
    fixed point of one EB step with rho = 1.9.  With the printed coefficient
    rho the multiplier would move by c (1 - rho)(p_i - p_s), which is not zero
    at a saddle point (there p_i - p_s = -div q_i)."""
    caps = _rand_caps(shape, 12, model, n)
    alpha = 0.2
    fg = oracle.Problem(shape, model=model, nlabels=n, method="fg", relax=1.0, tv=tv, alpha=alpha)
    st = oracle.init_state(fg, caps)
    for _ in range(40):
        oracle.step(fg, caps, st, 5000)
        s1 = st.copy()
        oracle.step(fg, caps, s1, 1)
        if max(float(np.max(np.abs(getattr(st, f) - getattr(s1, f)))) for f in ("u", "q", "ps", "p")) < 1e-13:
            break
    else:
        raise AssertionError("FG did not reach a fixed point")
    assert float(np.max(np.abs(st.p - st.ps))) > 1e-3   # the A5 term would be visible
    eb = oracle.Problem(shape, model=model, nlabels=n, method="eb", relax=1.9, tv=tv, alpha=alpha)
    s2 = oracle.state_from_arrays(eb, st.u, st.q, st.ps, st.p)
    oracle.step(eb, caps, s2, 1)
    for f in ("u", "q", "ps", "p"):
        a, b = getattr(st, f), getattr(s2, f)
        assert np.max(np.abs(a - b)) < 1e-9 * max(1.0, np.max(np.abs(a))), f
