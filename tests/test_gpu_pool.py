"""The batched pool (persistent work-list kernels, hipGraph super-steps,
device-side convergence decisions) through the C ABI.

* every solve's result is bit-identical alone and in a mix of grids of
  different sizes and models, with the same stop iterate;
* a pool solve equals the single-solve API with the same storage, bit for
  bit (same tile bodies);
* FP32 pool iterates match the FP64 oracle;
* admission is decided by footprint and memory is reused after retirement.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2004_11227_amd import maxflow as mfx
from paper_2004_11227_amd import serving, synth

from _gpu import banner, gpu_solver, need_gpu, oracle_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _mix():
    out = []
    rng = np.random.default_rng(11)
    for i, (shape, model, n) in enumerate([((64, 64), "two", 2), ((131, 77), "two", 2), ((200, 256), "two", 2),
                                           ((90, 97), "potts", 3), ((64, 130), "potts", 4),
                                           ((75, 75), "potts", 8), ((70, 128), "potts", 2),
                                           ((20, 24, 37), "two", 2), ((33, 40, 64), "two", 2)]):
        if len(shape) == 3:
            caps = synth.two_label_caps(synth.ellipsoid_volume(*shape, 4, 0.1, 500 + i))
        elif model == "two":
            caps = synth.two_label_caps(synth.ellipse_image(*shape, 5, 0.12, 500 + i))
        else:
            img, _ = synth.voronoi_image(*shape, n, 0.12, 500 + i, ncells=12)
            caps = synth.potts_caps(img, n)
        kw = dict(model=model, nlabels=n, method="eb" if i % 2 else "fg", alpha=float(rng.uniform(0.2, 0.5)),
                  storage="bf16", tol=1e-4, max_iter=600, check_every=10, promote_gap=2e-3, promote_iter=200)
        out.append((torch.from_numpy(caps.astype(np.float32)).cuda(), kw))
    return out


def _run_pool(items, steps=10, depth=0):
    pool = mfx.Pool(1 << 30, max_slots=64, max_tiles=1 << 15, steps_per_advance=steps, depth=depth)
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


def test_alone_equals_mix_bitwise():
    banner("pool alone vs mix")
    items = _mix()
    mixed = _run_pool(items)
    for k, it in enumerate(items):
        alone = _run_pool([it])[0]
        gm, um, lm = mixed[k]
        ga, ua, la = alone
        assert gm["iter"] == ga["iter"] and gm["status"] == ga["status"], (k, gm, ga)
        assert np.array_equal(um, ua) and np.array_equal(lm, la), k
        assert gm["status"] in (0, 1)
        if gm["status"] == 0:
            assert gm["rel_gap"] <= 1e-4


def test_pool_depth2_equals_depth1_bitwise():
    """Two iterations per super-step (the two-iteration pass for the
    two-label 2-D solves, two sweeps for the others) give the iterates,
    stop iterations and gaps of one-iteration super-steps, promotions
    included."""
    banner("pool depth 2 vs depth 1")
    items = _mix()
    d1 = _run_pool(items, depth=1)
    d2 = _run_pool(items, depth=2)
    for k, (a, b) in enumerate(zip(d1, d2)):
        assert a[0]["iter"] == b[0]["iter"] and a[0]["status"] == b[0]["status"], (k, a[0], b[0])
        assert a[0]["rel_gap"] == b[0]["rel_gap"], k
        assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2]), k


def test_pool_depth_rules():
    with pytest.raises(mfx.MaxflowError):
        mfx.Pool(1 << 24, max_slots=2, max_tiles=64, steps_per_advance=10, depth=3)
    for depth in (0, 1, 2):
        p = mfx.Pool(1 << 24, max_slots=2, max_tiles=64, steps_per_advance=10, depth=depth)
        p.close()


@pytest.mark.parametrize("steps", [5, 20, 1])
def test_pool_rejects_other_step_counts(steps):
    """Advances of other than 10 steps are rejected at creation."""
    with pytest.raises(mfx.MaxflowError) as ei:
        mfx.Pool(1 << 24, max_slots=2, max_tiles=64, steps_per_advance=steps)
    assert ei.value.status == mfx.MF_EINVAL


@pytest.mark.skip(reason="20-step pools are rejected: a serving run with a 20-step pool after a 10-step one "
                         "ended in a host segmentation fault whose cause has not been found")
def test_pool_twenty_steps_after_ten_equals_single_solves():
    """The configuration of the unexplained fault: a 10-step serving run,
    then a 20-step pool in the same process; every result must equal the
    single-solve API with the same storage and cadence."""
    banner("pool 20 steps after 10")
    items = _mix()
    _run_pool(items, steps=10)
    for c, kw in items:
        kw20 = {**kw, "check_every": 20, "promote_iter": 0, "promote_gap": 0.0, "storage": "f32"}
        g, u, _ = _run_pool([(c, kw20)], steps=20)[0]
        s = mfx.Solver(c, **kw20)
        gs = s.solve()
        assert gs["iter"] == g["iter"] and np.array_equal(s.u().cpu().numpy(), u)
        s.close()


@pytest.mark.parametrize("model,n,storage", [("two", 2, "bf16"), ("potts", 4, "bf16"), ("two", 2, "f32"),
                                             ("potts", 3, "f32")])
def test_pool_equals_single_solve_api(model, n, storage):
    banner(f"pool vs single {model} {n} {storage}")
    shape = (150, 203)
    if model == "two":
        caps = synth.two_label_caps(synth.ellipse_image(*shape, 6, 0.12, 77))
    else:
        img, _ = synth.voronoi_image(*shape, n, 0.12, 77, ncells=16)
        caps = synth.potts_caps(img, n)
    kw = dict(model=model, nlabels=n, method="eb", alpha=0.35, storage=storage, tol=1e-3, max_iter=500,
              check_every=10)
    t = torch.from_numpy(caps.astype(np.float32)).cuda()
    g, u, lab = _run_pool([(t, kw)])[0]
    s = mfx.Solver(t, **kw)
    gs = s.solve()
    us = s.u().cpu().numpy()
    s.close()
    assert gs["iter"] == g["iter"] and gs["status"] == g["status"]
    assert np.array_equal(us, u)
    assert abs(gs["rel_gap"] - g["rel_gap"]) <= 1e-9 * max(1.0, abs(gs["rel_gap"]))


def test_pool_fp32_matches_oracle():
    banner("pool fp32 vs oracle")
    shape = (97, 130)
    caps = synth.two_label_caps(synth.ellipse_image(*shape, 5, 0.1, 91)).astype(np.float32).astype(np.float64)
    kw = dict(model="two", method="eb", relax=1.5, alpha=0.5, storage="f32", tol=0.0, max_iter=120,
              check_every=10)
    g, u, _ = _run_pool([(torch.from_numpy(caps.astype(np.float32)).cuda(), kw)])[0]
    assert g["iter"] == 120 and g["status"] == 1
    pr = oracle_problem(shape, kw)
    st = oracle.init_state(pr, caps)
    oracle.step(pr, caps, st, 120)
    assert np.max(np.abs(u - st.u)) <= 1e-4
    e = oracle.energy(pr, caps, st)
    assert abs(g["rel_gap"] - e["rel_gap"]) < 1e-5


def test_bf16_promotion_reaches_tolerance():
    """BF16 flow storage floors the Potts gap near 1e-3; with promotion the
    solve finishes in FP32 storage and reaches 1e-4."""
    banner("pool promotion")
    img, _ = synth.voronoi_image(256, 256, 4, 0.15, 2004, ncells=32)
    caps = torch.from_numpy(synth.potts_caps(img, 4).astype(np.float32)).cuda()
    base = dict(model="potts", nlabels=4, method="eb", alpha=0.3, storage="bf16", tol=1e-4, max_iter=1000)
    pool = mfx.Pool(1 << 30, max_slots=8, max_tiles=1 << 14, steps_per_advance=10)
    a = pool.admit(caps, **base)
    b = pool.admit(caps, promote_gap=2e-3, promote_iter=300, **base)
    res = {}
    while len(res) < 2:
        pool.advance()
        for sid, g in pool.poll():
            pool.retire(sid)
            res[sid] = g
    assert pool.stats()["promotions"] == 1
    pool.close()
    assert res[a]["status"] == 1 and res[a]["rel_gap"] > 1e-4     # floored in BF16
    assert res[b]["status"] == 0 and res[b]["rel_gap"] <= 1e-4     # finished in FP32


def test_admission_by_footprint_and_reuse():
    banner("pool footprint admission")
    shape = (256, 256)
    kw = dict(model="two", method="eb", alpha=0.5, storage="bf16", tol=1e-3, max_iter=200)
    fp = mfx.pool_footprint(shape, **kw)
    table = mfx._pool_lib().mf_pool_table_bytes(8, 4096)
    pool = mfx.Pool(table + 2 * fp + 4096, max_slots=8, max_tiles=4096, steps_per_advance=10)
    caps = torch.from_numpy(synth.two_label_caps(synth.ellipse_image(*shape, 5, 0.1, 3)).astype(np.float32)).cuda()
    a = pool.admit(caps, **kw)
    b = pool.admit(caps, **kw)
    c = pool.admit(caps, **kw)
    assert a is not None and b is not None and c is None     # third does not fit
    done = []
    while not done:
        pool.advance()
        done = pool.poll()
    for sid, _ in done:
        pool.retire(sid)
    c = pool.admit(caps, **kw)
    assert c is not None                                        # memory reused
    pool.close()


def test_serving_loop_end_to_end():
    banner("serving loop")
    reqs = synth.serving_trace(24, seed=7, rate=None, lo=48, hi=320, frac3d=0.1, side3d=32)
    caps = {r.rid: torch.from_numpy(synth.request_caps(r).astype(np.float32)).cuda() for r in reqs}

    def kw_of(r):
        return dict(model=r.model, nlabels=r.nlabels, method="eb", alpha=r.alpha, storage="bf16", tol=1e-4,
                    max_iter=1000, check_every=10)

    pool = mfx.Pool(2 << 30, max_slots=32, max_tiles=1 << 15, steps_per_advance=10)
    be = serving.PoolBackend(pool, lambda r: caps[r.rid], kw_of)
    rep = serving.serve(reqs, be)
    pool.close()
    assert len(rep.records) == 24
    assert all(r.status in (0, 1) for r in rep.records)
    assert all(r.iters % 10 == 0 or r.iters == 1000 for r in rep.records)


def test_pool_rejects_unaligned_check_cadence():
    pool = mfx.Pool(1 << 28, max_slots=4, max_tiles=1024, steps_per_advance=10)
    caps = torch.ones((2, 32, 32), device="cuda")
    with pytest.raises(mfx.MaxflowError):
        pool.admit(caps, model="two", check_every=5, max_iter=100)
    with pytest.raises(mfx.MaxflowError):
        pool.admit(caps, model="two", check_every=10, max_iter=105)
    with pytest.raises(mfx.MaxflowError):
        pool.admit(caps, model="two", method="dr")
    assert pool.admit(caps, model="two", check_every=10, max_iter=100) is not None
    pool.close()


def test_reused_slot_not_judged_by_older_snapshot():
    """A poll after an advance reads the status as of the advance before it.
    A solve admitted into the slot of a just-retired one must not be
    reported from a snapshot that still shows its predecessor finished."""
    banner("pool snapshot lag and slot reuse")
    shape = (96, 96)
    caps = torch.from_numpy(synth.two_label_caps(synth.ellipse_image(*shape, 3, 0.1, 11)).astype(np.float32)).cuda()
    pool = mfx.Pool(1 << 28, max_slots=1, max_tiles=1 << 12, steps_per_advance=10)
    first = pool.admit(caps, model="two", method="eb", alpha=0.5, tol=1e-2, max_iter=50)
    done = []
    while not done:
        pool.advance()
        done = pool.poll()
    assert [sid for sid, _ in done] == [first]
    pool.retire(first, want_u=False, want_labels=False)
    second = pool.admit(caps, model="two", method="eb", alpha=0.5, tol=0.0, max_iter=200)
    assert second is not None and second != first
    pool.advance()
    assert pool.poll() == []        # the snapshot read predates the admission
    reported = []
    for _ in range(30):
        pool.advance()
        reported += pool.poll()
        if reported:
            break
    pool.close()
    assert [sid for sid, _ in reported] == [second]
    assert reported[0][1]["iter"] == 200 and reported[0][1]["status"] == 1


def test_graphs_follow_growing_lists_and_changing_class_sets():
    """Admissions in the middle of running solves: a class whose item count
    passes its graph's grid (a 64^2 solve joined by a 1024x768 one: 4 -> 772
    tiles), a new class joining and leaving (Potts n = 3), retirements in
    between.  Every solve still equals the single-solve API bit for bit."""
    banner("pool graphs: growing lists, changing class sets")
    specs = [((64, 64), "two", 2, 0), ((1024, 768), "two", 2, 3), ((90, 97), "potts", 3, 5),
             ((200, 130), "two", 2, 9), ((40, 300), "potts", 3, 14)]
    items = []
    for i, (shape, model, n, at) in enumerate(specs):
        if model == "two":
            caps = synth.two_label_caps(synth.ellipse_image(*shape, 5, 0.12, 700 + i))
        else:
            img, _ = synth.voronoi_image(*shape, n, 0.12, 700 + i, ncells=12)
            caps = synth.potts_caps(img, n)
        kw = dict(model=model, nlabels=n, method="eb", alpha=0.35, storage="f32", tol=1e-4, max_iter=300,
                  check_every=10)
        items.append((torch.from_numpy(caps.astype(np.float32)).cuda(), kw, at))
    pool = mfx.Pool(1 << 30, max_slots=16, max_tiles=1 << 14, steps_per_advance=10)
    sids, res, adv = {}, {}, 0
    while len(res) < len(items):
        for k, (t, kw, at) in enumerate(items):
            if at == adv and k not in sids:
                sids[k] = pool.admit(t, **kw)
                assert sids[k] is not None
        pool.advance()
        adv += 1
        for sid, g in pool.poll():
            u, lab = pool.retire(sid)
            res[sid] = (g, u.cpu().numpy(), lab.cpu().numpy())
    pool.close()
    for k, (t, kw, _) in enumerate(items):
        g, u, lab = res[sids[k]]
        s = mfx.Solver(t, **kw)
        gs = s.solve()
        us = s.u().cpu().numpy()
        ls = s.labels().cpu().numpy()
        s.close()
        assert gs["iter"] == g["iter"] and gs["status"] == g["status"], (k, gs, g)
        assert np.array_equal(us, u), k
        assert np.array_equal(ls, lab), k
