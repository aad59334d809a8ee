"""Scheduling logic of the serving loop, on the CPU with a fake backend:
footprint admission, FIFO order, head-of-line blocking, retirement as soon
as a solve converges, latency accounting, and the too-big request error."""
from dataclasses import dataclass

import numpy as np
import pytest

from paper_2004_11227_amd.serving import serve


@dataclass
class Req:
    rid: int
    arrival: float
    nbytes: int
    steps: int          # super-steps until the fake solve converges


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeBackend:
    """Each advance() costs `dt` seconds of simulated time and moves every
    resident solve one super-step; a solve converges after req.steps."""

    def __init__(self, clock, budget, slots, dt=1.0):
        self.clock, self.budget, self.slots, self.dt = clock, budget, slots, dt
        self.active = {}
        self.used = 0
        self.next = 0
        self.admit_order = []
        self.max_used = 0

    def admit(self, req):
        if self.used + req.nbytes > self.budget or len(self.active) >= self.slots:
            return None
        sid = self.next
        self.next += 1
        self.active[sid] = [req, 0, False]
        self.used += req.nbytes
        self.max_used = max(self.max_used, self.used)
        self.admit_order.append(req.rid)
        return sid

    def advance(self):
        self.clock.t += self.dt
        for st in self.active.values():
            st[1] += 1

    def poll(self):
        out = []
        for sid, st in self.active.items():
            if not st[2] and st[1] >= st[0].steps:
                st[2] = True
                out.append((sid, dict(iter=st[1] * 10, status=0, rel_gap=1e-5)))
        return out

    def retire(self, sid):
        req, _, done = self.active.pop(sid)
        assert done
        self.used -= req.nbytes


def test_all_complete_fifo_and_budget():
    rng = np.random.default_rng(0)
    reqs = [Req(i, float(i) * 0.5, int(rng.integers(1, 5)), int(rng.integers(1, 8))) for i in range(60)]
    clk = FakeClock()
    be = FakeBackend(clk, budget=8, slots=4)
    rep = serve(reqs, be, clock=clk)
    assert len(rep.records) == 60
    assert all(np.isfinite(r.finished) for r in rep.records)
    assert be.admit_order == list(range(60))          # FIFO
    assert be.max_used <= 8 and be.used == 0
    for r in rep.records:
        req = reqs[r.rid]
        assert r.admitted >= req.arrival - 1e-12
        assert r.finished - r.admitted >= req.steps * be.dt - 1e-9   # served at least its steps
    lat = np.array([r.latency for r in rep.records])
    assert rep.p50 == pytest.approx(np.percentile(lat, 50))
    assert rep.p99 == pytest.approx(np.percentile(lat, 99))


def test_head_of_line_blocks_until_memory_frees():
    # request 1 needs the whole budget: it waits until request 0 retires,
    # and request 2 (small) must not overtake it.
    reqs = [Req(0, 0.0, 6, 3), Req(1, 0.0, 10, 1), Req(2, 0.0, 1, 1)]
    clk = FakeClock()
    be = FakeBackend(clk, budget=10, slots=8)
    rep = serve(reqs, be, clock=clk)
    rec = {r.rid: r for r in rep.records}
    assert be.admit_order == [0, 1, 2]
    assert rec[1].admitted >= rec[0].finished
    assert rec[2].admitted >= rec[1].admitted


def test_retire_as_soon_as_converged():
    reqs = [Req(0, 0.0, 1, 2), Req(1, 0.0, 1, 9)]
    clk = FakeClock()
    be = FakeBackend(clk, budget=10, slots=8)
    rep = serve(reqs, be, clock=clk)
    rec = {r.rid: r for r in rep.records}
    assert rec[0].finished == pytest.approx(2.0)
    assert rec[1].finished == pytest.approx(9.0)


def test_request_larger_than_pool_is_an_error():
    clk = FakeClock()
    be = FakeBackend(clk, budget=4, slots=2)
    with pytest.raises(RuntimeError):
        serve([Req(0, 0.0, 5, 1)], be, clock=clk)


def test_idle_until_arrival():
    reqs = [Req(0, 0.0, 1, 1), Req(1, 100.0, 1, 1)]
    clk = FakeClock()

    class Ticking(FakeBackend):
        pass

    be = Ticking(clk, budget=4, slots=2)
    # the loop busy-waits on the clock; make the clock move when idle
    orig = clk.__call__

    class AutoClock(FakeClock):
        def __call__(self):
            self.t += 0.25
            return self.t

    ac = AutoClock()
    be.clock = ac
    rep = serve(reqs, be, clock=ac)
    rec = {r.rid: r for r in rep.records}
    assert rec[1].admitted >= 100.0
