"""Pins for the oracle's preconditioner variants (CPU only).

* M_n, several symmetric red-black Gauss-Seidel sweeps per rPDRQ iteration
  (the sRBGS preconditioner applied n times, the construction the rPDRQ
  section builds on): checked against n explicit preconditioned steps
  u <- u + M^{-1}(b - T u) with M the symmetric Gauss-Seidel matrix of T, all
  built here from difference matrices of this file (not the oracle's
  operators); against a direct linear solve of T u = b as n grows; for the
  feasibility M_n >= T that the convergence result needs; and by the method
  still reaching the exhaustive minimum cut.
* A non-decreasing relaxation sequence rho_k in (0, 2) for rpADMMII (the EB
  scheme allows any such sequence): the schedule's end points and
  monotonicity; that a scheduled run is the composition of constant-rho
  steps at rho_0, rho_1, ... (also across split calls, so the iteration
  index is carried); and convergence to the exhaustive minimum.
"""
import numpy as np
import pytest

import oracle
from paper_2004_11227_amd import synth


# ---- difference matrices, written from the definitions --------------------------

def _fwd_diff(n):
    """Forward difference on a line of n cells with zero flux at the end."""
    D = np.zeros((n, n))
    for i in range(n - 1):
        D[i, i] = -1.0
        D[i, i + 1] = 1.0
    return D


def _grad_matrix(shape):
    """grad u stacked component by component; component k differentiates the
    k-th fastest axis (x first), on C-ordered cells."""
    axes = list(range(len(shape)))[::-1]
    blocks = []
    for ax in axes:
        mats = [np.eye(s) for s in shape]
        mats[ax] = _fwd_diff(shape[ax])
        M = mats[0]
        for m in mats[1:]:
            M = np.kron(M, m)
        blocks.append(M)
    return np.vstack(blocks)


def _red_black_perm(shape):
    par = np.indices(shape).reshape(len(shape), -1).sum(0) % 2
    return np.concatenate([np.where(par == 0)[0], np.where(par == 1)[0]])


def _sgs_matrix(T, perm):
    """Symmetric Gauss-Seidel matrix of T in the ordering perm (forward sweep
    then backward sweep): M = (D - L) D^{-1} (D - U), in permuted indices."""
    Tp = T[np.ix_(perm, perm)]
    D = np.diag(np.diag(Tp))
    Lo = -np.tril(Tp, -1)
    Up = -np.triu(Tp, 1)
    return (D - Lo) @ np.linalg.inv(D) @ (D - Up), Tp


def _n_steps(T, perm, b, u, n):
    M, Tp = _sgs_matrix(T, perm)
    up = u[perm].copy()
    for _ in range(n):
        up = up + np.linalg.solve(M, b[perm] - Tp @ up)
    out = np.empty_like(u)
    out[perm] = up
    return out


def _dr_problem_and_b(shape, model, n, seed):
    """Random rPDRQ iterate; returns (problem, caps, state, b per label, T per label)."""
    rng = np.random.default_rng(seed)
    L = 1 if model == "two" else n
    N = int(np.prod(shape))
    caps = synth.two_label_caps(rng.uniform(0, 1, shape)) if model == "two" else \
        synth.potts_caps(rng.uniform(0, 1, shape), n)
    pr = oracle.Problem(shape, model=model, nlabels=n, method="dr", alpha=0.3)
    u = rng.normal(size=(L,) + shape)
    q = rng.normal(scale=0.2, size=(L, len(shape)) + shape)
    ps = rng.normal(size=shape)
    p = rng.normal(size=(L,) + shape)
    st = oracle.state_from_arrays(pr, u, q, ps, p)
    G = _grad_matrix(shape)
    Dv = -G.T                                  # div = -grad^*
    lap = G.T @ G                              # -Delta with zero-flux boundary
    sg, tau = pr.sigma, pr.tau
    m = 2.0 if model == "two" else n + 1.0
    bs = []
    for l in range(L):
        bl = -sg * (Dv @ q[l].reshape(-1) + p[l].ravel() - ps.ravel())
        if model != "two":
            # b_i = ... + st ((n-1) u_i - sum_{j != i} u_j)
            bl = bl + sg * tau * ((n - 1) * u[l].ravel() - (u.reshape(L, N).sum(0) - u[l].ravel()))
        bs.append(bl)
    T = sg * tau * (lap + m * np.eye(N))
    return pr, caps, st, bs, T


@pytest.mark.parametrize("shape,model,n", [((5, 6), "two", 2), ((4, 7), "potts", 3), ((3, 3, 4), "two", 2)])
@pytest.mark.parametrize("sweeps", [1, 2, 3])
def test_gs_sweeps_are_n_preconditioned_steps(shape, model, n, sweeps):
    pr, caps, st, bs, T = _dr_problem_and_b(shape, model, n, seed=11 + sweeps)
    perm = _red_black_perm(shape)
    u0 = st.u.copy()
    pr.gs_sweeps = sweeps
    oracle.step(pr, caps, st, 1)
    for l in range(len(bs)):
        expect = _n_steps(T, perm, bs[l], u0[l].ravel(), sweeps)
        assert np.max(np.abs(st.u[l].ravel() - expect)) < 1e-11


def test_many_sweeps_solve_the_linear_system():
    """As the sweep count grows, the u-step becomes the exact solve of
    T u = b (here 400 sweeps on 6 x 7 cells, contraction factor < 0.9)."""
    shape = (6, 7)
    pr, caps, st, bs, T = _dr_problem_and_b(shape, "two", 2, seed=5)
    pr.gs_sweeps = 400
    oracle.step(pr, caps, st, 1)
    assert np.max(np.abs(st.u[0].ravel() - np.linalg.solve(T, bs[0]))) < 1e-10


@pytest.mark.parametrize("shape,m", [((4, 5), 2.0), ((3, 3, 3), 4.0)])
def test_n_fold_preconditioner_is_feasible(shape, m):
    """n steps of the symmetric GS iteration are one step of the
    preconditioner M_n = T (I - (I - M^{-1} T)^n)^{-1}; it is symmetric and
    M_n >= T (the feasibility condition), and M_1 = M."""
    N = int(np.prod(shape))
    G = _grad_matrix(shape)
    T = 0.2 * (G.T @ G + m * np.eye(N))
    M, Tp = _sgs_matrix(T, _red_black_perm(shape))
    E = np.eye(N) - np.linalg.solve(M, Tp)
    for n in range(1, 5):
        Mn = Tp @ np.linalg.inv(np.eye(N) - np.linalg.matrix_power(E, n))
        if n == 1:
            assert np.allclose(Mn, M, atol=1e-10)
        assert np.allclose(Mn, Mn.T, atol=1e-9)
        assert np.linalg.eigvalsh(0.5 * (Mn + Mn.T) - Tp).min() >= -1e-9


@pytest.mark.parametrize("shape", [(4, 4), (2, 2, 4)])
@pytest.mark.parametrize("sweeps", [2, 4])
def test_dr_with_more_sweeps_reaches_the_minimum_cut(shape, sweeps):
    for seed, alpha in [(1, 0.15), (2, 0.3)]:
        rng = np.random.default_rng(seed)
        caps = synth.two_label_caps(rng.uniform(0, 1, size=shape))
        best, blab, second = oracle.brute_force_binary(caps, alpha)
        pr = oracle.Problem(shape, model="two", method="dr", tv="aniso", alpha=alpha, gs_sweeps=sweeps)
        st, hist = oracle.solve(pr, caps, 40000, check_every=25, tol=1e-11)
        e = hist[-1][1]
        assert e["rel_gap"] < 1e-10
        lab = oracle.labels(pr, st.u[0])
        assert abs(oracle.labeling_energy(caps, lab, alpha, "two") - best) < 1e-8
        if second > best + 1e-9:
            assert np.array_equal(lab, blab)


# ---- non-decreasing relaxation ------------------------------------------------

def test_rho_schedule_end_points_and_monotone():
    pr = oracle.Problem((4, 4), method="eb", relax=1.9, relax0=0.5, relax_ramp=20)
    r = [pr.rho_at(k) for k in range(40)]
    assert r[0] == 0.5 and r[20] == 1.9 and all(x == 1.9 for x in r[20:])
    assert all(b >= a for a, b in zip(r, r[1:]))
    assert all(0.0 < x < 2.0 for x in r)
    assert abs(r[10] - 1.2) < 1e-15
    const = oracle.Problem((4, 4), method="eb", relax=1.7)
    assert all(const.rho_at(k) == 1.7 for k in (0, 5, 1000))


@pytest.mark.parametrize("model", ["two", "potts"])
def test_scheduled_run_is_the_composition_of_constant_rho_steps(model):
    shape = (9, 11)
    rng = np.random.default_rng(17)
    caps = synth.two_label_caps(rng.uniform(0, 1, shape)) if model == "two" else \
        synth.potts_caps(rng.uniform(0, 1, shape), 3)
    kw = dict(model=model, nlabels=3, alpha=0.35, method="eb")
    sched = oracle.Problem(shape, relax=1.8, relax0=0.6, relax_ramp=6, **kw)
    a = oracle.init_state(sched, caps)
    oracle.step(sched, caps, a, 9)
    b = oracle.init_state(sched, caps)
    oracle.step(sched, caps, b, 4)
    oracle.step(sched, caps, b, 5)
    c = oracle.init_state(sched, caps)
    for k in range(9):
        oracle.step(oracle.Problem(shape, relax=sched.rho_at(k), **kw), caps, c, 1)
    for f in ("u", "q", "ps", "p"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
        assert np.array_equal(getattr(a, f), getattr(c, f)), f
    # and it differs from the constant-rho run (the schedule is in effect)
    d = oracle.init_state(sched, caps)
    oracle.step(oracle.Problem(shape, relax=1.8, **kw), caps, d, 9)
    assert np.max(np.abs(a.u - d.u)) > 1e-6


@pytest.mark.parametrize("shape", [(4, 4), (2, 8)])
def test_scheduled_eb_reaches_the_minimum_cut(shape):
    for seed, alpha in [(3, 0.15), (4, 0.3)]:
        rng = np.random.default_rng(seed)
        caps = synth.two_label_caps(rng.uniform(0, 1, size=shape))
        best, blab, second = oracle.brute_force_binary(caps, alpha)
        pr = oracle.Problem(shape, model="two", method="eb", tv="aniso", alpha=alpha, relax=1.9,
                            relax0=0.5, relax_ramp=200)
        st, hist = oracle.solve(pr, caps, 40000, check_every=25, tol=1e-11)
        e = hist[-1][1]
        assert e["rel_gap"] < 1e-10
        lab = oracle.labels(pr, st.u[0])
        assert abs(oracle.labeling_energy(caps, lab, alpha, "two") - best) < 1e-8
        if second > best + 1e-9:
            assert np.array_equal(lab, blab)
