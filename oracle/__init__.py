"""FP64 CPU oracle for the continuous max-flow methods (TEST INFRASTRUCTURE).

Only the test suite, the smoke check and the CPU-baseline leg of ``bench.py``
may import this package.  The solver never does: it shares no
code with this oracle.  The arithmetic lives in ``oracle.c`` (plain C loops in
double precision, following the paper's equations); this module only
marshals numpy arrays through ctypes and adds the pure-Python brute-force
references used to pin the oracle.

Array conventions (numpy, C order, float64):
    caps: (2, *shape) = [C_s, C_t] for the two-label model,
          (n, *shape) = [C_1..C_n] for the Potts model
    state: u (L, *shape), q (L, ndim, *shape), ps (*shape), p (L, *shape)
           where L = 1 for two-label (p holds p_t) and L = n for Potts;
           shape = (ny, nx) or (nz, ny, nx); flow component k belongs to the
           k-th fastest axis (k = 0 is x).
"""
from __future__ import annotations

import ctypes
import itertools
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MODELS = {"two": 0, "potts": 1}
METHODS = {"fg": 0, "eb": 1, "dr": 2, "ty": 3, "cp": 4}
TVS = {"iso": 0, "aniso": 1}


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain -O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-fno-fast-math", "-ffp-contract=off", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd, cwd=_HERE)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Grid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("nx", ctypes.c_long), ("ny", ctypes.c_long),
                ("nz", ctypes.c_long)]


class _Params(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int), ("method", ctypes.c_int), ("tv", ctypes.c_int),
                ("nlabels", ctypes.c_int), ("alpha", ctypes.c_double), ("c", ctypes.c_double),
                ("relax", ctypes.c_double), ("sigma", ctypes.c_double), ("tau", ctypes.c_double),
                ("a", ctypes.c_double), ("a_tilde", ctypes.c_double), ("a1", ctypes.c_double),
                ("a2", ctypes.c_double), ("gs_sweeps", ctypes.c_int), ("relax0", ctypes.c_double),
                ("relax_ramp", ctypes.c_long)]


_lib = None


def _L():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        P = ctypes.POINTER(ctypes.c_double)
        G, PR = ctypes.POINTER(_Grid), ctypes.POINTER(_Params)
        _lib.or_grad.argtypes = [G, P, P]
        _lib.or_div.argtypes = [G, P, P]
        _lib.or_project_alpha.argtypes = [G, ctypes.c_int, ctypes.c_double, P]
        _lib.or_simplex_project.argtypes = [ctypes.c_int, P, P]
        _lib.or_rbgs_sweep.argtypes = [G, ctypes.c_double, ctypes.c_double, P, P]
        _lib.or_init.argtypes = [G, PR, P, P, P, P, P]
        _lib.or_admm_iter.argtypes = [G, PR, P, P, P, P, P]
        _lib.or_pdrq_iter.argtypes = [G, PR, P, P, P, P, P, P, P, P]
        _lib.or_run.argtypes = [G, PR, P, ctypes.c_long, ctypes.c_long, P, P, P, P, P, P, P, P]
        _lib.or_rho_at.argtypes = [PR, ctypes.c_long]
        _lib.or_rho_at.restype = ctypes.c_double
        _lib.or_energy.argtypes = [G, PR, P, P, P, P, P, P]
        _lib.or_labels.argtypes = [G, PR, P, ctypes.POINTER(ctypes.c_int)]
        _lib.or_num_threads.restype = ctypes.c_int
        _lib.or_set_threads.argtypes = [ctypes.c_int]
    return _lib


def num_threads() -> int:
    return int(_L().or_num_threads())


def set_threads(n: int):
    """Threads of the oracle's parallel loops (results do not depend on it)."""
    _L().or_set_threads(int(n))


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _grid(shape) -> _Grid:
    if len(shape) == 2:
        return _Grid(2, shape[1], shape[0], 1)
    if len(shape) == 3:
        return _Grid(3, shape[2], shape[1], shape[0])
    raise ValueError("shape must be 2-D or 3-D")


@dataclass
class Problem:
    """Model + method + parameters.  Zero parameters take the paper's values:
    c = 0.3; relax = 1.618 (FG r), 1.9 (EB rho, DR rho); a = 4*ndim,
    a_tilde = 2, a1 = 2, a2 = 2n; rPDRQ (sigma, tau) = (0.2, 1.0) two-label,
    (5, 0.4) Potts; ALG1 sigma = 0.4, tau = 1 / (L^2 sigma) with the bound
    L^2 = 4 ndim + 2 (two labels) or 4 ndim + n + 1 (n labels) on |K^* K|.
    Methods: fg (rpADMMI), eb (rpADMMII), dr (rPDRQ), ty (pADMM-TY), cp
    (ALG1).  Preconditioner variants: gs_sweeps symmetric red-black
    Gauss-Seidel sweeps per rPDRQ iteration (M_n; 0 -> 1); for rpADMMII a
    non-decreasing relaxation rising linearly from relax0 to relax over
    relax_ramp iterations (relax0 = 0: constant)."""
    shape: tuple
    model: str = "two"
    method: str = "eb"
    tv: str = "iso"
    nlabels: int = 2
    alpha: float = 0.5
    c: float = 0.0
    relax: float = 0.0
    sigma: float = 0.0
    tau: float = 0.0
    a: float = 0.0
    a_tilde: float = 0.0
    a1: float = 0.0
    a2: float = 0.0
    gs_sweeps: int = 0
    relax0: float = 0.0
    relax_ramp: int = 0

    def __post_init__(self):
        self.shape = tuple(int(s) for s in self.shape)
        nd = len(self.shape)
        if self.model == "two":
            self.nlabels = 2
        self.c = self.c or 0.3
        self.relax = self.relax or {"fg": 1.618, "eb": 1.9, "dr": 1.9, "ty": 1.0, "cp": 1.0}[self.method]
        if self.method == "cp":
            self.sigma = self.sigma or 0.4
            l2 = 4.0 * nd + (2.0 if self.model == "two" else self.nlabels + 1.0)
            self.tau = self.tau or 1.0 / (l2 * self.sigma)
        elif self.model == "two":
            self.sigma = self.sigma or 0.2
            self.tau = self.tau or 1.0
        else:
            self.sigma = self.sigma or 5.0
            self.tau = self.tau or 0.4
        self.a = self.a or 4.0 * nd
        self.a_tilde = self.a_tilde or 2.0
        self.a1 = self.a1 or 2.0
        self.a2 = self.a2 or 2.0 * self.nlabels

    @property
    def L(self) -> int:
        return 1 if self.model == "two" else self.nlabels

    @property
    def ndim(self) -> int:
        return len(self.shape)

    def _params(self) -> _Params:
        return _Params(MODELS[self.model], METHODS[self.method], TVS[self.tv], self.nlabels,
                       self.alpha, self.c, self.relax, self.sigma, self.tau, self.a,
                       self.a_tilde, self.a1, self.a2, int(self.gs_sweeps), float(self.relax0),
                       int(self.relax_ramp))

    def rho_at(self, k: int) -> float:
        """rpADMMII relaxation of the step from iterate k to k+1."""
        return float(_L().or_rho_at(ctypes.byref(self._params()), int(k)))


@dataclass
class State:
    u: np.ndarray
    q: np.ndarray
    ps: np.ndarray
    p: np.ndarray
    # rPDRQ resolvent outputs of the last iteration (the feasible dual point)
    zq: np.ndarray = None
    zs: np.ndarray = None
    zp: np.ndarray = None
    iters: int = 0
    # ALG1 extrapolated primal variable u-bar
    ub: np.ndarray = None

    def copy(self) -> "State":
        c = lambda a: None if a is None else a.copy()
        return State(c(self.u), c(self.q), c(self.ps), c(self.p), c(self.zq), c(self.zs),
                     c(self.zp), self.iters, c(self.ub))


def _caps(prob: Problem, caps) -> np.ndarray:
    caps = np.ascontiguousarray(caps, dtype=np.float64)
    ncap = 2 if prob.model == "two" else prob.nlabels
    if caps.shape != (ncap,) + prob.shape:
        raise ValueError(f"caps shape {caps.shape} != {(ncap,) + prob.shape}")
    return caps


def init_state(prob: Problem, caps) -> State:
    caps = _caps(prob, caps)
    L, sh, nd = prob.L, prob.shape, prob.ndim
    u = np.zeros((L,) + sh)
    q = np.zeros((L, nd) + sh)
    ps = np.zeros(sh)
    p = np.zeros((L,) + sh)
    _L().or_init(ctypes.byref(_grid(sh)), ctypes.byref(prob._params()), _ptr(caps),
                 _ptr(u), _ptr(q), _ptr(ps), _ptr(p))
    st = State(u, q, ps, p)
    if prob.method == "dr":
        st.zq, st.zs, st.zp = q.copy(), ps.copy(), p.copy()
    if prob.method == "cp":
        st.ub = u.copy()
    return st


def state_from_arrays(prob: Problem, u, q, ps, p) -> State:
    f = lambda a: np.ascontiguousarray(a, dtype=np.float64).copy()
    st = State(f(u), f(q), f(ps), f(p))
    if prob.method == "dr":
        st.zq, st.zs, st.zp = st.q.copy(), st.ps.copy(), st.p.copy()
    if prob.method == "cp":
        st.ub = st.u.copy()
    return st


def step(prob: Problem, caps, st: State, iters: int = 1) -> State:
    """Advance ``st`` in place by ``iters`` iterations of the chosen method."""
    caps = _caps(prob, caps)
    if prob.method == "dr" and st.zq is None:
        st.zq, st.zs, st.zp = st.q.copy(), st.ps.copy(), st.p.copy()
    z = st.zq if st.zq is not None else np.zeros(1)
    zs = st.zs if st.zs is not None else np.zeros(1)
    zp = st.zp if st.zp is not None else np.zeros(1)
    if prob.method == "cp" and st.ub is None:
        st.ub = st.u.copy()
    ub = st.ub if st.ub is not None else np.zeros(1)
    _L().or_run(ctypes.byref(_grid(prob.shape)), ctypes.byref(prob._params()), _ptr(caps),
                int(st.iters), int(iters), _ptr(st.u), _ptr(st.q), _ptr(st.ps), _ptr(st.p),
                _ptr(z), _ptr(zs), _ptr(zp), _ptr(ub))
    st.iters += iters
    return st


def energy(prob: Problem, caps, st: State) -> dict:
    """FP64 primal, dual, relative gap, residual RMS and total source flow.

    For rPDRQ the dual point is the last resolvent output (zq, zs, zp)."""
    caps = _caps(prob, caps)
    out = (ctypes.c_double * 5)()
    if prob.method == "dr":
        q, ps, p = st.zq, st.zs, st.zp
    else:
        q, ps, p = st.q, st.ps, st.p
    _L().or_energy(ctypes.byref(_grid(prob.shape)), ctypes.byref(prob._params()), _ptr(caps),
                   _ptr(st.u), _ptr(q), _ptr(ps), _ptr(p), out)
    data, tv, dual, r2, flow = list(out)
    primal = data + prob.alpha * tv
    n = int(np.prod(prob.shape)) * prob.L
    return dict(primal=primal, dual=dual,
                rel_gap=(primal - dual) / max(abs(primal), abs(dual), 1e-300),
                resid_rms=float(np.sqrt(r2 / n)), flow=flow, data=data, tv=tv)


def labels(prob: Problem, u) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64)
    lab = np.zeros(prob.shape, dtype=np.int32)
    _L().or_labels(ctypes.byref(_grid(prob.shape)), ctypes.byref(prob._params()), _ptr(u),
                   lab.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return lab


def solve(prob: Problem, caps, iters: int, check_every: int = 0, tol: float = 0.0):
    """Run ``iters`` iterations from the initial point.  With check_every > 0,
    stop at the first multiple of check_every whose relative gap <= tol.
    Returns (state, history) with history = [(k, energy dict), ...]."""
    st = init_state(prob, caps)
    hist = []
    if check_every <= 0:
        step(prob, caps, st, iters)
        return st, hist
    k = 0
    while True:
        e = energy(prob, caps, st)
        hist.append((k, e))
        if e["rel_gap"] <= tol or k >= iters:
            break
        n = min(check_every, iters - k)
        step(prob, caps, st, n)
        k += n
    return st, hist


# ---- operators exposed for the pins ---------------------------------------------------

def grad(f: np.ndarray) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros((f.ndim,) + f.shape)
    _L().or_grad(ctypes.byref(_grid(f.shape)), _ptr(f), _ptr(out))
    return out


def div(q: np.ndarray) -> np.ndarray:
    q = np.ascontiguousarray(q, dtype=np.float64)
    out = np.zeros(q.shape[1:])
    _L().or_div(ctypes.byref(_grid(q.shape[1:])), _ptr(q), _ptr(out))
    return out


def project_alpha(q: np.ndarray, alpha: float, tv: str = "iso") -> np.ndarray:
    q = np.ascontiguousarray(q, dtype=np.float64).copy()
    _L().or_project_alpha(ctypes.byref(_grid(q.shape[1:])), TVS[tv], alpha, _ptr(q))
    return q


def simplex_project(v) -> np.ndarray:
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.zeros_like(v)
    _L().or_simplex_project(len(v), _ptr(v), _ptr(out))
    return out


def rbgs_sweep(b: np.ndarray, u: np.ndarray, m: float, st: float) -> np.ndarray:
    b = np.ascontiguousarray(b, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64).copy()
    _L().or_rbgs_sweep(ctypes.byref(_grid(b.shape)), m, st, _ptr(b), _ptr(u))
    return u


# ---- brute-force references (tiny grids) ------------------------------------------------

def _edges(shape):
    """Forward-neighbour pairs (i, j) of the 4/6-neighbour grid, flattened."""
    idx = np.arange(int(np.prod(shape))).reshape(shape)
    out = []
    for ax in range(len(shape)):
        a = np.take(idx, np.arange(shape[ax] - 1), axis=ax).ravel()
        b = np.take(idx, np.arange(1, shape[ax]), axis=ax).ravel()
        out.append(np.stack([a, b], 1))
    return np.concatenate(out, 0) if out else np.zeros((0, 2), int)


def brute_force_binary(caps, alpha: float):
    """Exhaustive minimum of sum (1-l) C_s + l C_t + alpha * #cut edges over all
    binary labelings l (anisotropic TV of a binary field counts cut edges).
    Returns (best energy, best labeling, second-best energy)."""
    cs, ct = caps[0].ravel(), caps[1].ravel()
    n = cs.size
    if n > 20:
        raise ValueError("too many pixels for brute force")
    e = _edges(caps.shape[1:])
    labs = ((np.arange(1 << n)[:, None] >> np.arange(n)[None, :]) & 1).astype(np.float64)
    data = (1 - labs) @ cs + labs @ ct
    cut = np.abs(labs[:, e[:, 0]] - labs[:, e[:, 1]]).sum(1) if len(e) else 0.0
    en = data + alpha * cut
    order = np.argsort(en, kind="stable")
    best = order[0]
    second = en[order[1]] if len(order) > 1 else np.inf
    return float(en[best]), labs[best].reshape(caps.shape[1:]).astype(np.int32), float(second)


def brute_force_potts(caps, alpha: float):
    """Exhaustive minimum over all L^N labelings of sum_x C_{l(x)}(x) +
    alpha * sum_i TV_aniso(1[l = i]) = data + 2 alpha * #edges with l(x) != l(y)."""
    L = caps.shape[0]
    shape = caps.shape[1:]
    n = int(np.prod(shape))
    if L ** n > 70000:
        raise ValueError("too many labelings")
    c = caps.reshape(L, n)
    e = _edges(shape)
    labs = np.array(list(itertools.product(range(L), repeat=n)), dtype=np.int64)
    data = c[labs, np.arange(n)[None, :]].sum(1)
    cut = (labs[:, e[:, 0]] != labs[:, e[:, 1]]).sum(1) if len(e) else 0
    en = data + 2.0 * alpha * cut
    order = np.argsort(en, kind="stable")
    second = en[order[1]] if len(order) > 1 else np.inf
    return float(en[order[0]]), labs[order[0]].reshape(shape).astype(np.int32), float(second)


def labeling_energy(caps, lab, alpha: float, model: str) -> float:
    """Energy of an integral labeling under anisotropic TV."""
    e = _edges(lab.shape)
    a, b = lab.ravel()[e[:, 0]], lab.ravel()[e[:, 1]]
    if model == "two":
        l = lab.ravel().astype(np.float64)
        return float(((1 - l) * caps[0].ravel() + l * caps[1].ravel()).sum()
                     + alpha * np.abs(a - b).sum())
    n = lab.size
    data = caps.reshape(caps.shape[0], n)[lab.ravel(), np.arange(n)].sum()
    return float(data + 2.0 * alpha * (a != b).sum())
