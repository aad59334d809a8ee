"""Pins for the oracle's discrete operators (CPU only).

Each check is fixed by mathematics, not by re-typing the oracle's formulas:
adjointness of grad and -div, the operator-norm bounds of Theorem 1 and of
the 3-D extension, the matrix inequalities of Theorem 2 and Lemma 1 on the
oracle's own dense operators, the sRBGS sweep as an explicit preconditioned
step, and the defining properties of the two projections.
"""
import numpy as np
import pytest

import oracle

SHAPES = [(7, 5), (1, 9), (9, 1), (16, 16), (3, 4, 5), (1, 1, 6), (5, 1, 1)]


def _dense(op, shape, nin):
    """Matrix of a linear operator by applying it to unit vectors."""
    cols = []
    for j in range(nin):
        e = np.zeros(nin)
        e[j] = 1.0
        cols.append(op(e).ravel())
    return np.stack(cols, 1)


@pytest.mark.parametrize("shape", SHAPES)
def test_grad_div_adjoint(shape):
    rng = np.random.default_rng(0)
    u = rng.normal(size=shape)
    q = rng.normal(size=(len(shape),) + shape)
    lhs = (oracle.grad(u) * q).sum()
    rhs = -(u * oracle.div(q)).sum()
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_grad_of_constant_and_linear_ramp():
    # Neumann forward differences: constant -> 0; ramp along x -> 1 except the
    # last column, which is 0 by the boundary condition.
    f = np.ones((4, 6)) * 3.5
    assert np.all(oracle.grad(f) == 0.0)
    ramp = np.tile(np.arange(6.0), (4, 1))
    g = oracle.grad(ramp)
    assert np.all(g[0][:, :-1] == 1.0) and np.all(g[0][:, -1] == 0.0)
    assert np.all(g[1] == 0.0)


def _power_norm(shape, iters=3000):
    rng = np.random.default_rng(1)
    nd = len(shape)
    q = rng.normal(size=(nd,) + shape)
    lam = 0.0
    for _ in range(iters):
        v = -oracle.grad(oracle.div(q))      # div^* div q
        lam = np.sqrt((v * v).sum() / (q * q).sum())
        q = v / np.sqrt((v * v).sum())
    return lam


def test_div_star_div_bound_2d():
    # Theorem 1: ||div^* div|| <= 8 in 2-D; the bound is asymptotically sharp,
    # so on a 16x16 grid the norm must be close to (but below) 8.
    lam = _power_norm((16, 16))
    assert 7.5 < lam < 8.0


def test_div_star_div_bound_3d():
    # 3-D extension: each 1-D forward difference has squared norm < 4, so
    # ||div^* div|| < 12 (preconditioner a = 4 * ndim = 12).
    lam = _power_norm((8, 8, 8))
    assert 10.5 < lam < 12.0


def test_theorem1_a_tilde():
    # 2 I_2 - A^*A >= 0 with A = [I, -I]  (Theorem 1)
    n = 5
    I = np.eye(n)
    A = np.hstack([I, -I])
    assert np.linalg.eigvalsh(2 * np.eye(2 * n) - A.T @ A).min() >= -1e-12


@pytest.mark.parametrize("n", [2, 3, 4, 8])
def test_theorem2_block_preconditioner(n):
    # diag(a1 I, ..., a1 I, a2 I) - A^*A >= 0 with a1 = 2, a2 = 2n, A = [I_n, -L_n]
    A = np.hstack([np.eye(n), -np.ones((n, 1))])
    At = np.diag([2.0] * n + [2.0 * n])
    assert np.linalg.eigvalsh(At - A.T @ A).min() >= -1e-12
    # a1 below 1 violates the inequality already on the p_i block
    At_bad = np.diag([0.9] * n + [2.0 * n])
    assert np.linalg.eigvalsh(At_bad - A.T @ A).min() < 0


@pytest.mark.parametrize("n", [2, 3, 4])
def test_lemma1_T0_dominates_KstarK(n):
    # K = [B^*; A^*] with B^* = diag(-grad), A^* u = (u_1..u_n, -sum u_i).
    # K^*K u_i = -Delta u_i + u_i + sum_j u_j;  T_0 = diag(-Delta + (n+1) I).
    shape = (3, 4)
    N = 12

    def neg_lap(v):
        return -oracle.div(oracle.grad(v.reshape(shape)))

    Lm = _dense(neg_lap, shape, N)                     # -Delta (Neumann), from the oracle ops
    KK = np.kron(np.eye(n), Lm + np.eye(N)) + np.kron(np.ones((n, n)), np.eye(N))
    T0 = np.kron(np.eye(n), Lm + (n + 1) * np.eye(N))
    assert np.linalg.eigvalsh(T0 - KK).min() >= -1e-10
    # -Delta from the oracle is symmetric PSD with the constant in its kernel
    assert np.allclose(Lm, Lm.T)
    assert abs(np.linalg.eigvalsh(Lm).min()) < 1e-10


@pytest.mark.parametrize("shape,m", [((4, 4), 2.0), ((3, 5), 5.0), ((2, 3, 3), 2.0)])
def test_rbgs_sweep_is_symmetric_gs_preconditioned_step(shape, m):
    """u + M^{-1}(b - T u) with M the symmetric Gauss-Seidel matrix of
    T = st(-Delta + m I) in red-black ordering equals the oracle's in-place
    red, black, red sweep."""
    rng = np.random.default_rng(3)
    N = int(np.prod(shape))
    st = 0.37
    Lm = _dense(lambda v: -oracle.div(oracle.grad(v.reshape(shape))), shape, N)
    T = st * (Lm + m * np.eye(N))
    coords = np.indices(shape).reshape(len(shape), -1).sum(0)
    perm = np.concatenate([np.where(coords % 2 == 0)[0], np.where(coords % 2 == 1)[0]])
    Tp = T[np.ix_(perm, perm)]
    D = np.diag(np.diag(Tp))
    Lo = -np.tril(Tp, -1)
    Up = -np.triu(Tp, 1)
    M = (D - Lo) @ np.linalg.inv(D) @ (D - Up)
    # M - T = Lo D^{-1} Up >= 0 (feasibility M >= T_Q of Proposition 1)
    assert np.linalg.eigvalsh(0.5 * (M + M.T) - Tp).min() >= -1e-10
    b = rng.normal(size=N)
    u = rng.normal(size=N)
    up = u[perm] + np.linalg.solve(M, b[perm] - Tp @ u[perm])
    expect = np.empty(N)
    expect[perm] = up
    got = oracle.rbgs_sweep(b.reshape(shape), u.reshape(shape), m, st).ravel()
    assert np.max(np.abs(got - expect)) < 1e-12


def test_project_alpha_iso_properties():
    rng = np.random.default_rng(4)
    alpha = 0.7
    q = rng.normal(size=(2, 9, 11)) * 2
    p = oracle.project_alpha(q, alpha, "iso")
    nrm = np.sqrt((p ** 2).sum(0))
    assert nrm.max() <= alpha * (1 + 1e-14)
    # idempotent (up to the last-bit rounding of |q| = alpha)
    assert np.allclose(oracle.project_alpha(p, alpha, "iso"), p, rtol=4e-16, atol=0)
    # identity inside the ball, radial scaling outside
    qn = np.sqrt((q ** 2).sum(0))
    inside = qn <= alpha
    assert np.array_equal(p[:, inside], q[:, inside])
    ratio = p[:, ~inside] / q[:, ~inside]
    assert np.allclose(ratio[0], ratio[1]) and np.allclose(nrm[~inside], alpha)
    # nonexpansive
    q2 = q + rng.normal(size=q.shape) * 0.3
    p2 = oracle.project_alpha(q2, alpha, "iso")
    assert np.all(np.sqrt(((p - p2) ** 2).sum(0)) <= np.sqrt(((q - q2) ** 2).sum(0)) + 1e-14)
    # alpha = 0 maps everything to zero
    assert np.all(oracle.project_alpha(q, 0.0, "iso") == 0.0)


def test_project_alpha_aniso_is_clamp():
    rng = np.random.default_rng(5)
    q = rng.normal(size=(3, 4, 4, 4))
    p = oracle.project_alpha(q, 0.5, "aniso")
    assert np.array_equal(p, np.minimum(0.5, np.maximum(-0.5, q)))


@pytest.mark.parametrize("n", [2, 3, 4, 8])
def test_simplex_projection_kkt(n):
    rng = np.random.default_rng(6 + n)
    for _ in range(200):
        v = rng.normal(size=n) * rng.uniform(0.1, 3)
        w = oracle.simplex_project(v)
        assert abs(w.sum() - 1.0) < 1e-12 and w.min() >= 0.0
        # KKT: v - w = theta on the support, v <= theta off the support
        sup = w > 0
        theta = (v - w)[sup]
        assert np.ptp(theta) < 1e-12
        assert np.all(v[~sup] <= theta[0] + 1e-12)
    # points of the simplex are fixed
    p = rng.dirichlet(np.ones(n))
    assert np.allclose(oracle.simplex_project(p), p, atol=1e-15)
