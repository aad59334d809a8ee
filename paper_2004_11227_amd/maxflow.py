"""Python binding of the C ABI in include/maxflow.h (argument marshalling only).

Every step of the solver runs in the HIP library ``libmaxflow.so`` built
in-tree by ``paper_2004_11227_amd.build``; importing this module on a machine
without it raises immediately -- there is no CPU fallback.  PyTorch supplies
device memory (the workspace and all input/output tensors) and streams.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmaxflow.so")

MF_OK, MF_ENOTCONV, MF_EINVAL, MF_ENOMEM, MF_EDEVICE, MF_EDIVERGED = 0, 1, -1, -2, -3, -4
MODELS = {"two": 0, "potts": 1}
METHODS = {"fg": 0, "eb": 1, "dr": 2, "ty": 3, "cp": 4}
TVS = {"iso": 0, "aniso": 1}
STORAGES = {"f32": 0, "bf16": 1}
VARIANTS = {"fused": 0, "unfused": 1}
CAP_SOURCES = {"planes": 0, "image": 1}
FIELDS = {"u": 0, "q": 1, "ps": 2, "p": 3, "zq": 4, "zs": 5, "zp": 6}
STATUS = {0: "converged", 1: "cap", -4: "diverged"}


class MaxflowError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"maxflow status {status}: {msg}")
        self.status = status


class mf_params(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("shape", ctypes.c_int64 * 3),
                ("model", ctypes.c_int32), ("method", ctypes.c_int32), ("tv", ctypes.c_int32),
                ("storage", ctypes.c_int32), ("variant", ctypes.c_int32), ("nlabels", ctypes.c_int32),
                ("alpha", ctypes.c_double), ("c", ctypes.c_double), ("relax", ctypes.c_double),
                ("sigma", ctypes.c_double), ("tau", ctypes.c_double), ("a", ctypes.c_double),
                ("a_tilde", ctypes.c_double), ("a1", ctypes.c_double), ("a2", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("tol", ctypes.c_double),
                ("check_every", ctypes.c_int32), ("tile_rows", ctypes.c_int32),
                ("promote_gap", ctypes.c_double), ("promote_iter", ctypes.c_int32), ("depth", ctypes.c_int32),
                ("slab_depth", ctypes.c_int32), ("gs_sweeps", ctypes.c_int32), ("relax0", ctypes.c_double),
                ("relax_ramp", ctypes.c_int32), ("cap_source", ctypes.c_int32), ("cap_power", ctypes.c_int32),
                ("levels", ctypes.c_double * 8)]


class mf_tune_cand(ctypes.Structure):
    _fields_ = [("tile_rows", ctypes.c_int32), ("depth", ctypes.c_int32), ("slab_depth", ctypes.c_int32),
                ("us_per_iter", ctypes.c_double)]


class mf_tuning(ctypes.Structure):
    _fields_ = [("tile_rows", ctypes.c_int32), ("depth", ctypes.c_int32), ("slab_depth", ctypes.c_int32),
                ("ncand", ctypes.c_int32), ("cand", mf_tune_cand * 16)]


MF_TUNE_TILE, MF_TUNE_DEPTH, MF_TUNE_SLAB = 1, 2, 4


class mf_gap(ctypes.Structure):
    _fields_ = [("iter", ctypes.c_int64), ("primal", ctypes.c_double), ("dual", ctypes.c_double),
                ("rel_gap", ctypes.c_double), ("resid_rms", ctypes.c_double),
                ("flow", ctypes.c_double), ("status", ctypes.c_int32)]

    def as_dict(self):
        return dict(iter=int(self.iter), primal=self.primal, dual=self.dual, rel_gap=self.rel_gap,
                    resid_rms=self.resid_rms, flow=self.flow, status=int(self.status))


_lib = None

#: names declared in include/maxflow.h that the library must export
EXPORTS = ["maxflow_workspace_bytes", "maxflow_create", "maxflow_reset", "maxflow_step",
           "maxflow_gap", "maxflow_solve", "maxflow_iter", "maxflow_read_u", "maxflow_labels",
           "maxflow_read_field", "maxflow_write_field", "maxflow_state_bytes",
           "maxflow_export_state", "maxflow_import_state", "maxflow_destroy",
           "maxflow_last_error", "maxflow_tune", "maxflow_solve_static"]


def lib():
    """Load libmaxflow.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} not built: run `python -m paper_2004_11227_amd.build` "
                           "(there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    P, V, S = ctypes.POINTER(mf_params), ctypes.c_void_p, ctypes.c_int32
    G = ctypes.POINTER(mf_gap)
    sig = {
        "maxflow_workspace_bytes": (ctypes.c_size_t, [P]),
        "maxflow_create": (S, [P, V, V, ctypes.c_size_t, V, ctypes.POINTER(V)]),
        "maxflow_reset": (S, [V]),
        "maxflow_step": (S, [V, ctypes.c_int32]),
        "maxflow_gap": (S, [V, G]),
        "maxflow_solve": (S, [V, G]),
        "maxflow_iter": (ctypes.c_int64, [V]),
        "maxflow_read_u": (S, [V, V]),
        "maxflow_labels": (S, [V, V]),
        "maxflow_read_field": (S, [V, ctypes.c_int32, V]),
        "maxflow_write_field": (S, [V, ctypes.c_int32, V]),
        "maxflow_state_bytes": (ctypes.c_size_t, [V]),
        "maxflow_export_state": (S, [V, V]),
        "maxflow_import_state": (S, [V, V, ctypes.c_int64]),
        "maxflow_destroy": (S, [V]),
        "maxflow_last_error": (ctypes.c_char_p, []),
        "maxflow_tune": (S, [V, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(mf_tuning)]),
        "maxflow_solve_static": (S, [P, V, V, V, G, V]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def last_error() -> str:
    return lib().maxflow_last_error().decode()


def _check(status, allow=(MF_OK,)):
    if status not in allow:
        raise MaxflowError(status, last_error())
    return status


def make_params(shape, model="two", method="eb", tv="iso", storage="f32", variant="fused",
                nlabels=2, alpha=0.5, c=0.0, relax=0.0, sigma=0.0, tau=0.0, a=0.0, a_tilde=0.0,
                a1=0.0, a2=0.0, max_iter=1000, tol=1e-4, check_every=10, tile_rows=0,
                promote_gap=0.0, promote_iter=0, depth=0, slab_depth=0, gs_sweeps=0, relax0=0.0,
                relax_ramp=0, cap_source="planes", cap_power=0, levels=()) -> mf_params:
    shape = tuple(int(s) for s in shape)
    p = mf_params()
    p.ndim = len(shape)
    for i, s in enumerate(shape):
        p.shape[i] = s
    p.model = MODELS[model]
    p.method = METHODS[method]
    p.tv = TVS[tv]
    p.storage = STORAGES[storage]
    p.variant = VARIANTS[variant]
    p.nlabels = 2 if model == "two" else int(nlabels)
    p.alpha, p.c, p.relax, p.sigma, p.tau = alpha, c, relax, sigma, tau
    p.a, p.a_tilde, p.a1, p.a2 = a, a_tilde, a1, a2
    p.max_iter, p.tol, p.check_every, p.tile_rows = int(max_iter), float(tol), int(check_every), int(tile_rows)
    p.promote_gap, p.promote_iter = float(promote_gap), int(promote_iter)
    p.depth = int(depth)
    p.slab_depth = int(slab_depth)
    p.gs_sweeps, p.relax0, p.relax_ramp = int(gs_sweeps), float(relax0), int(relax_ramp)
    p.cap_source = CAP_SOURCES[cap_source]
    p.cap_power = int(cap_power)
    if len(levels) > 8:
        raise ValueError("at most 8 levels")
    for i, v in enumerate(levels):
        p.levels[i] = float(v)
    return p


def workspace_bytes(params: mf_params) -> int:
    n = lib().maxflow_workspace_bytes(ctypes.byref(params))
    if n == 0:
        raise MaxflowError(MF_EINVAL, last_error())
    return int(n)


class Solver:
    """One solve on the current CUDA/HIP device.

    ``caps`` is a float32 device tensor of shape (2, *shape) = [C_s, C_t] for
    the two-label model or (n, *shape) = [C_1..C_n] for Potts; with
    ``cap_source="image"`` it is the image, shape (1, *shape), and the
    capacities are |I - levels[k]|^cap_power.  Keyword
    arguments follow ``make_params``.  ``stream`` is a torch stream (default:
    the current stream).  The workspace is a torch uint8 tensor owned here.
    """

    def __init__(self, caps: torch.Tensor, stream: torch.cuda.Stream | None = None, **kw):
        shape = tuple(caps.shape[1:])
        auto = kw.get("tile_rows") == "auto"
        what = 0
        if auto:
            # tile_rows="auto": the launch shape is autotuned (the tile height,
            # and the fusion depth and 3-D slab depth unless given); a cached
            # choice for this shape class, else the defaults now and the
            # autotuner below
            from . import tuning
            what = MF_TUNE_TILE | (MF_TUNE_DEPTH if not kw.get("depth") else 0) | \
                (MF_TUNE_SLAB if not kw.get("slab_depth") else 0)
            cached = tuning.lookup(shape, caps.device, **kw)
            kw = {**kw, "tile_rows": 0}
            if cached:
                kw["tile_rows"] = cached["tile_rows"]
                if what & MF_TUNE_DEPTH:
                    kw["depth"] = cached["depth"]
                if what & MF_TUNE_SLAB:
                    kw["slab_depth"] = cached["slab_depth"]
            auto = cached is None
        self.params = make_params(shape, **kw)
        self.shape = shape
        self.model = kw.get("model", "two")
        self.L = 1 if self.model == "two" else int(kw.get("nlabels", 2))
        self.ndim = len(shape)
        if caps.dtype != torch.float32 or not caps.is_cuda or not caps.is_contiguous():
            raise ValueError("caps must be a contiguous float32 device tensor")
        ncap = 2 if self.model == "two" else self.L
        if kw.get("cap_source", "planes") == "image":
            ncap = 1
        if caps.shape[0] != ncap:
            raise ValueError(f"caps must have {ncap} planes")
        self.device = caps.device
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        # create() reads `caps` on the solver stream
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        nbytes = workspace_bytes(self.params)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        _check(lib().maxflow_create(ctypes.byref(self.params), ctypes.c_void_p(caps.data_ptr()),
                                    ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                    ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self._kw = kw
        if auto:
            from . import tuning
            best, cands = self.tune(what=what)
            tuning.store(shape, caps.device, best, cands, **kw)

    # -- lifecycle
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().maxflow_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def tune(self, sweeps: int = 20, what: int = MF_TUNE_TILE | MF_TUNE_DEPTH | MF_TUNE_SLAB):
        """Time the candidate launch shapes on this solver (state unchanged)
        and keep the fastest.  Returns (choice, candidates): the chosen
        dict(tile_rows, depth, slab_depth) and a list of
        dict(tile_rows, depth, slab_depth, us_per_iter)."""
        t = mf_tuning()
        _check(lib().maxflow_tune(self._h, int(sweeps), int(what), ctypes.byref(t)))
        self.params.tile_rows, self.params.depth, self.params.slab_depth = t.tile_rows, t.depth, t.slab_depth
        best = dict(tile_rows=int(t.tile_rows), depth=int(t.depth), slab_depth=int(t.slab_depth))
        cands = [dict(tile_rows=int(c.tile_rows), depth=int(c.depth), slab_depth=int(c.slab_depth),
                      us_per_iter=float(c.us_per_iter)) for c in t.cand[:t.ncand]]
        return best, cands

    # -- iteration
    @property
    def iter(self) -> int:
        return int(lib().maxflow_iter(self._h))

    def reset(self):
        _check(lib().maxflow_reset(self._h))

    def step(self, iters: int = 1):
        _check(lib().maxflow_step(self._h, int(iters)))

    def gap(self) -> dict:
        g = mf_gap()
        _check(lib().maxflow_gap(self._h, ctypes.byref(g)), allow=(MF_OK, MF_EDIVERGED))
        return g.as_dict()

    def solve(self) -> dict:
        g = mf_gap()
        _check(lib().maxflow_solve(self._h, ctypes.byref(g)), allow=(MF_OK, MF_ENOTCONV, MF_EDIVERGED))
        return g.as_dict()

    # -- results
    def _planes(self, field: str) -> int:
        L, d = self.L, self.ndim
        return {"u": L, "q": L * d, "ps": 1, "p": L, "zq": L * d, "zs": 1, "zp": L}[field]

    def read(self, field: str) -> torch.Tensor:
        out = torch.empty((self._planes(field),) + self.shape, dtype=torch.float32, device=self.device)
        _check(lib().maxflow_read_field(self._h, FIELDS[field], ctypes.c_void_p(out.data_ptr())))
        return out

    def write(self, field: str, t: torch.Tensor):
        t = t.to(device=self.device, dtype=torch.float32).contiguous()
        if t.numel() != self._planes(field) * int(torch.tensor(self.shape).prod()):
            raise ValueError("wrong field size")
        _check(lib().maxflow_write_field(self._h, FIELDS[field], ctypes.c_void_p(t.data_ptr())))

    def u(self) -> torch.Tensor:
        return self.read("u")

    def labels(self) -> torch.Tensor:
        out = torch.empty(self.shape, dtype=torch.int32, device=self.device)
        _check(lib().maxflow_labels(self._h, ctypes.c_void_p(out.data_ptr())))
        return out

    def export_state(self) -> torch.Tensor:
        n = int(lib().maxflow_state_bytes(self._h))
        out = torch.empty(n, dtype=torch.uint8, device=self.device)
        _check(lib().maxflow_export_state(self._h, ctypes.c_void_p(out.data_ptr())))
        return out

    def import_state(self, blob: torch.Tensor, iter: int):
        _check(lib().maxflow_import_state(self._h, ctypes.c_void_p(blob.data_ptr()), int(iter)))


#: bytes of the static device workspace of solve_static (per device)
STATIC_SCRATCH_BYTES = 64 << 20


def solve_static(caps: torch.Tensor, stream: torch.cuda.Stream | None = None, want_u: bool = True,
                 want_labels: bool = True, **kw):
    """One complete solve through maxflow_solve_static, the entry point that
    allocates nothing inside the library (its workspace is a static device
    array of STATIC_SCRATCH_BYTES).  ``caps`` and keywords as for Solver.
    Returns (gap dict, u or None, labels or None); the output tensors are
    allocated here, by the caller's side of the boundary."""
    shape = tuple(caps.shape[1:])
    p = make_params(shape, **kw)
    if caps.dtype != torch.float32 or not caps.is_cuda or not caps.is_contiguous():
        raise ValueError("caps must be a contiguous float32 device tensor")
    L = 1 if kw.get("model", "two") == "two" else int(kw.get("nlabels", 2))
    stream = stream if stream is not None else torch.cuda.current_stream(caps.device)
    stream.wait_stream(torch.cuda.current_stream(caps.device))
    u = torch.empty((L,) + shape, dtype=torch.float32, device=caps.device) if want_u else None
    lab = torch.empty(shape, dtype=torch.int32, device=caps.device) if want_labels else None
    g = mf_gap()
    _check(lib().maxflow_solve_static(ctypes.byref(p), ctypes.c_void_p(caps.data_ptr()),
                                      ctypes.c_void_p(u.data_ptr() if u is not None else 0),
                                      ctypes.c_void_p(lab.data_ptr() if lab is not None else 0),
                                      ctypes.byref(g), ctypes.c_void_p(stream.cuda_stream)),
           allow=(MF_OK, MF_ENOTCONV, MF_EDIVERGED))
    return g.as_dict(), u, lab


# ---------------------------------------------------------------------------- pool

_POOL_SIG = {
    "mf_pool_footprint": (ctypes.c_size_t, [ctypes.POINTER(mf_params)]),
    "mf_pool_table_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32]),
    "mf_pool_create": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                        ctypes.POINTER(ctypes.c_void_p)]),
    "mf_pool_admit": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(mf_params), ctypes.c_void_p,
                                       ctypes.POINTER(ctypes.c_int64)]),
    "mf_pool_advance": (ctypes.c_int32, [ctypes.c_void_p]),
    "mf_pool_poll": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(mf_gap),
                                      ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "mf_pool_retire": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]),
    "mf_pool_stats": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]),
    "mf_pool_destroy": (ctypes.c_int32, [ctypes.c_void_p]),
    "mf_pool_promotions": (ctypes.c_int64, [ctypes.c_void_p]),
}
EXPORTS += list(_POOL_SIG)


def _pool_lib():
    L = lib()
    if not getattr(L, "_pool_ready", False):
        for name, (res, args) in _POOL_SIG.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        L._pool_ready = True
    return L


def pool_footprint(shape, **kw) -> int:
    p = make_params(shape, **kw)
    n = _pool_lib().mf_pool_footprint(ctypes.byref(p))
    if n == 0:
        raise MaxflowError(MF_EINVAL, last_error())
    return int(n)


class Pool:
    """Continuous-batching pool over one device arena (a torch uint8 tensor
    owned here).  admit() returns a solve id, or None when the arena, the slot
    table or the class work list is full (MF_ENOMEM).  ``depth``: iterations
    per two-label 2-D pass (0: 2 when steps_per_advance is even, else 1)."""

    def __init__(self, arena_bytes: int, max_slots: int = 256, max_tiles: int = 1 << 16,
                 steps_per_advance: int = 10, device=None, stream: torch.cuda.Stream | None = None,
                 depth: int = 0):
        L = _pool_lib()
        self.device = torch.device(device or "cuda")
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        _check(L.mf_pool_create(ctypes.c_void_p(self.arena.data_ptr()), int(arena_bytes), int(max_slots),
                                int(max_tiles), int(steps_per_advance), int(depth),
                                ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self.max_slots = max_slots
        self.meta = {}
        self._ids = (ctypes.c_int64 * max_slots)()
        self._gaps = (mf_gap * max_slots)()

    def admit(self, caps: torch.Tensor, **kw):
        shape = tuple(caps.shape[1:])
        p = make_params(shape, **kw)
        if caps.dtype != torch.float32 or not caps.is_cuda or not caps.is_contiguous():
            raise ValueError("caps must be a contiguous float32 device tensor")
        sid = ctypes.c_int64()
        # the admission copies read `caps` on the pool stream
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        st = _pool_lib().mf_pool_admit(self._h, ctypes.byref(p), ctypes.c_void_p(caps.data_ptr()),
                                       ctypes.byref(sid))
        if st == MF_ENOMEM:
            return None
        _check(st)
        L = 1 if kw.get("model", "two") == "two" else int(kw.get("nlabels", 2))
        self.meta[int(sid.value)] = (shape, L)
        return int(sid.value)

    def advance(self):
        _check(_pool_lib().mf_pool_advance(self._h))

    def poll(self):
        n = ctypes.c_int32()
        _check(_pool_lib().mf_pool_poll(self._h, self._ids, self._gaps, self.max_slots, ctypes.byref(n)))
        return [(int(self._ids[i]), self._gaps[i].as_dict()) for i in range(n.value)]

    def retire(self, sid: int, want_u: bool = True, want_labels: bool = True):
        shape, L = self.meta.pop(sid)
        u = torch.empty((L,) + shape, dtype=torch.float32, device=self.device) if want_u else None
        lab = torch.empty(shape, dtype=torch.int32, device=self.device) if want_labels else None
        _check(_pool_lib().mf_pool_retire(self._h, int(sid), ctypes.c_void_p(u.data_ptr() if u is not None else 0),
                                          ctypes.c_void_p(lab.data_ptr() if lab is not None else 0)))
        return u, lab

    def stats(self):
        a, used, free = ctypes.c_int32(), ctypes.c_size_t(), ctypes.c_size_t()
        _check(_pool_lib().mf_pool_stats(self._h, ctypes.byref(a), ctypes.byref(used), ctypes.byref(free)))
        return dict(active=a.value, bytes_in_use=used.value, largest_free=free.value,
                    promotions=int(_pool_lib().mf_pool_promotions(self._h)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _pool_lib().mf_pool_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
