"""Continuous-batching serving loop for segmentation solves.

Requests (arrival time, grid, model, labels, alpha, capacities) are admitted
FIFO into a resident pool as soon as they have arrived and the pool has room
(HBM footprint and a free slot); every resident solve advances together on
the GPU; a solve retires as soon as its gap converges (or it hits the
iteration cap), its u and labels are copied out, and its memory and slot are
reused by the next request.  Latency is arrival -> result.

The loop talks to a backend with four calls (admit / advance / poll /
retire), so the scheduling logic is testable on the CPU with a fake backend;
``PoolBackend`` is the real one (the HIP pool through the C ABI).
``run_sequential`` is the one-solve-at-a-time baseline through the
single-solve API.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Record:
    rid: int
    arrival: float
    admitted: float = float("nan")
    finished: float = float("nan")
    iters: int = -1
    status: int = 99
    rel_gap: float = float("nan")

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclass
class Report:
    records: list
    wall: float
    solves_per_s: float
    p50: float
    p99: float
    mean_latency: float
    extra: dict = field(default_factory=dict)

    def as_dict(self):
        return dict(solves=len(self.records), wall_s=self.wall, solves_per_s=self.solves_per_s,
                    p50_latency_s=self.p50, p99_latency_s=self.p99, mean_latency_s=self.mean_latency,
                    **self.extra)


def summarize(records, wall, **extra) -> Report:
    lat = np.array([r.latency for r in records], dtype=np.float64)
    return Report(records, wall, len(records) / wall if wall > 0 else float("inf"),
                  float(np.percentile(lat, 50)) if len(lat) else float("nan"),
                  float(np.percentile(lat, 99)) if len(lat) else float("nan"),
                  float(lat.mean()) if len(lat) else float("nan"), extra)


def serve(requests, backend, clock=time.perf_counter, advances_per_poll: int = 1,
          idle_sleep: float = 0.0, working_set: int | None = None) -> Report:
    """Run the request list (objects with .rid and .arrival seconds) to
    completion through `backend`.  Returns per-request records and totals.

    `working_set` (bytes, optional) bounds the summed footprint of the solves
    advanced together, so that they stay resident in the last-level cache
    between advances; a request larger than the bound is admitted only
    into an empty pool (it then runs alone, like the one-at-a-time path).
    The backend's own arena bound still applies."""
    pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
    waiting = collections.deque()
    active = {}
    recs = {r.rid: Record(r.rid, r.arrival) for r in requests}
    t0 = clock()
    peak_active = 0
    resident = 0
    fp = {}
    while pending or waiting or active:
        now = clock() - t0
        while pending and pending[0].arrival <= now:
            waiting.append(pending.popleft())
        # FIFO admission while the pool has room; the head blocks the queue
        while waiting:
            need = backend.footprint(waiting[0]) if working_set is not None else 0
            if working_set is not None and active and resident + need > working_set:
                break
            sid = backend.admit(waiting[0])
            if sid is None:
                break
            req = waiting.popleft()
            active[sid] = req
            fp[sid] = need
            resident += need
            recs[req.rid].admitted = clock() - t0
        peak_active = max(peak_active, len(active))
        if not active:
            if waiting:
                raise RuntimeError(f"request {waiting[0].rid} does not fit in an empty pool")
            if pending:
                wait = pending[0].arrival - (clock() - t0)
                if wait > 0 and idle_sleep:
                    time.sleep(min(wait, idle_sleep))
            continue
        for _ in range(advances_per_poll):
            backend.advance()
        for sid, gap in backend.poll():
            req = active.pop(sid)
            resident -= fp.pop(sid)
            backend.retire(sid)
            r = recs[req.rid]
            r.finished = clock() - t0
            r.iters = gap["iter"]
            r.status = gap["status"]
            r.rel_gap = gap["rel_gap"]
    wall = clock() - t0
    return summarize(list(recs.values()), wall, peak_active=peak_active)


class PoolBackend:
    """The HIP pool.  `caps_of(req)` returns the request's FP32 capacities as
    a device tensor; `kw_of(req)` its solver keyword arguments."""

    def __init__(self, pool, caps_of, kw_of, keep_results: bool = False):
        self.pool = pool
        self.caps_of = caps_of
        self.kw_of = kw_of
        self.keep = keep_results
        self.results = {}
        self.rid_of = {}

    def footprint(self, req):
        from . import maxflow
        return maxflow.pool_footprint(tuple(self.caps_of(req).shape[1:]), **self.kw_of(req))

    def admit(self, req):
        sid = self.pool.admit(self.caps_of(req), **self.kw_of(req))
        if sid is not None:
            self.rid_of[sid] = req.rid
        return sid

    def advance(self):
        self.pool.advance()

    def poll(self):
        return self.pool.poll()

    def retire(self, sid):
        u, lab = self.pool.retire(sid, want_u=self.keep, want_labels=True)
        rid = self.rid_of.pop(sid)
        if self.keep:
            self.results[rid] = (u, lab)


def run_sequential(requests, caps_of, kw_of, stream=None, clock=time.perf_counter,
                   keep_results: bool = False) -> Report:
    """One solve at a time through the single-solve API, in arrival order;
    a request starts when it has arrived and the previous one finished."""
    import torch

    from . import maxflow
    reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
    recs = []
    results = {}
    t0 = clock()
    for req in reqs:
        while clock() - t0 < req.arrival:
            pass
        rec = Record(req.rid, req.arrival, admitted=clock() - t0)
        s = maxflow.Solver(caps_of(req), stream=stream, **kw_of(req))
        g = s.solve()
        lab = s.labels()
        if keep_results:
            results[req.rid] = (s.u(), lab)
        s.close()
        rec.finished = clock() - t0
        rec.iters, rec.status, rec.rel_gap = g["iter"], g["status"], g["rel_gap"]
        recs.append(rec)
    wall = clock() - t0
    rep = summarize(recs, wall)
    rep.extra["results"] = results if keep_results else None
    return rep


def _caps32(req):
    from . import synth
    return synth.request_caps(req).astype(np.float32)


def draw_requests(nreq: int = 2048, seed: int = 4000, workers: int | None = None) -> dict:
    """The serving trace and every request's FP32 capacities, drawn on the
    host cores by worker processes (forked: call this before the GPU is
    initialised).  Returns dict(requests, caps, seed)."""
    import os
    from concurrent.futures import ProcessPoolExecutor

    from . import synth
    base = synth.serving_trace(nreq, seed=seed)
    workers = workers or max(1, min(16, os.cpu_count() or 1))
    if workers == 1:
        caps = [_caps32(r) for r in base]
    else:
        with ProcessPoolExecutor(max_workers=workers) as ex:
            caps = list(ex.map(_caps32, base, chunksize=4))
    return {"requests": base, "caps": caps, "seed": seed}


def benchmark(nreq: int = 128, seed: int = 4000, pool_storage: str = "bf16", tol: float = 1e-4,
              max_iter: int = 1000, arena_bytes: int = 48 << 30, max_slots: int = 256,
              steps_per_advance: int = 10, latency_load: float = 0.7, promote_gap: float = 2e-3,
              promote_iter: int = 400, working_set: int | None = None, drawn: dict | None = None,
              latency: bool = True, log=None) -> dict:
    """Serving workload: `nreq` requests of the mixed trace (2-D sides
    log-uniform on [64, 2048], 10 % 3-D 128^3, labels in {2,3,4,8}), each run
    to relative gap `tol` or `max_iter` iterations.  `drawn` (from
    draw_requests) supplies the trace and its capacities instead.

    Throughput is measured at saturation (every request queued at t = 0) for
    the one-at-a-time FP32 path (single-solve API) and for the pool; latency
    (p50/p99) is measured with Poisson arrivals at `latency_load` x the
    one-at-a-time throughput, on the same arrival trace for both paths.
    `working_set` (default: no bound beyond the arena) caps the summed
    footprint of resident solves; a 192 MiB cap cost a quarter of the pool's
    throughput on this mix.
    """
    import torch

    from . import maxflow, synth

    def say(*a):
        if log:
            log(" ".join(str(x) for x in a))

    if drawn is None:
        drawn = {"requests": synth.serving_trace(nreq, seed=seed), "caps": None, "seed": seed}
    base = drawn["requests"]
    seed = drawn["seed"]
    caps = {}
    for i, r in enumerate(base):
        host = drawn["caps"][i] if drawn["caps"] is not None else synth.request_caps(r).astype(np.float32)
        caps[r.rid] = torch.from_numpy(host).cuda()
        if drawn["caps"] is not None:
            drawn["caps"][i] = None   # the device copy is the one kept
    torch.cuda.synchronize()
    npx = {r.rid: int(np.prod(r.shape)) for r in base}

    def kw_seq(r):
        return dict(model=r.model, nlabels=r.nlabels, method="eb", alpha=r.alpha, storage="f32", tol=tol,
                    max_iter=max_iter, check_every=10)

    def kw_pool(r):
        d = kw_seq(r)
        d["storage"] = pool_storage
        if pool_storage == "bf16":   # finish in FP32 once BF16 rounding floors the gap
            d["promote_gap"] = promote_gap
            d["promote_iter"] = promote_iter
        return d

    stream = torch.cuda.Stream()

    def with_arrivals(reqs, times):
        out = []
        for r, t in zip(reqs, times):
            rr = synth.Request(**{**r.__dict__, "arrival": float(t)})
            out.append(rr)
        return out

    sat = with_arrivals(base, [0.0] * len(base))
    # warm-up: compile caches, first graph capture
    warm = sat[:2]
    run_sequential(warm, lambda r: caps[r.rid], kw_seq, stream=stream)
    pool = maxflow.Pool(arena_bytes, max_slots=max_slots, max_tiles=1 << 18,
                        steps_per_advance=steps_per_advance, stream=stream)
    serve(warm, PoolBackend(pool, lambda r: caps[r.rid], kw_pool))
    torch.cuda.synchronize()

    seq = run_sequential(sat, lambda r: caps[r.rid], kw_seq, stream=stream)
    say("sequential fp32 saturation:", seq.as_dict())
    bp = serve(sat, PoolBackend(pool, lambda r: caps[r.rid], kw_pool), working_set=working_set)
    say("pool", pool_storage, "saturation:", bp.as_dict())

    rate = latency_load * seq.solves_per_s
    seq_l = pool_l = None
    if latency:
        rng = np.random.Generator(np.random.PCG64(seed + 1))
        times = np.cumsum(rng.exponential(1.0 / rate, size=len(base)))
        arr = with_arrivals(base, times)
        say("sequential fp32 under Poisson arrivals")
        seq_l = run_sequential(arr, lambda r: caps[r.rid], kw_seq, stream=stream)
        say("pool under Poisson arrivals")
        pool_l = serve(arr, PoolBackend(pool, lambda r: caps[r.rid], kw_pool), working_set=working_set)
    promotions = pool.stats()["promotions"]
    pool.close()

    def iters(rep):
        it = np.array([r.iters for r in rep.records])
        st = np.array([r.status for r in rep.records])
        return dict(mean_iters=float(it.mean()), converged=int((st == 0).sum()), capped=int((st == 1).sum()),
                    diverged=int((st == -4).sum()))

    return {
        "promotions_total": promotions,
        "requests": len(base), "tol": tol, "max_iter": max_iter, "pool_storage": pool_storage,
        "working_set_bytes": working_set,
        "promote_gap": promote_gap if pool_storage == "bf16" else None,
        "promote_iter": promote_iter if pool_storage == "bf16" else None,
        "total_pixels": int(sum(npx.values())),
        "sequential_iters": {r.rid: int(r.iters) for r in seq.records},
        "sequential_fp32": {**seq.as_dict(), **iters(seq)},
        "pool": {**bp.as_dict(), **iters(bp)},
        "speedup_solves_per_s": bp.solves_per_s / seq.solves_per_s,
        "latency_rate_per_s": rate if latency else None,
        "sequential_fp32_latency": {k: v for k, v in seq_l.as_dict().items() if k != "results"} if latency else None,
        "pool_latency": pool_l.as_dict() if latency else None,
    }
