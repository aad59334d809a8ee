"""GPU parity of the rpADMM sweeps (rpADMMI = fg, rpADMMII = eb) against the
FP64 oracle, through the C ABI.

Bar (FP32 storage): after the same number of iterations from the same initial
point, max |u - u_oracle| <= 1e-4 and thresholded-label disagreement <= 0.1 %.
Fused and unfused passes, and every tile height, must agree bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2004_11227_amd import synth

from _gpu import banner, compare_run, gpu_fields, gpu_solver, need_gpu, oracle_problem

pytestmark = pytest.mark.gpu

TOL_U = 1e-4
TOL_LAB = 1e-3


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


@pytest.mark.parametrize("method", ["fg", "eb"])
@pytest.mark.parametrize("variant", ["fused", "unfused"])
def test_config0_two_label(method, variant):
    """128x128 ellipses, alpha 0.5, relaxation 1.5, 300 iterations."""
    banner(f"c0 two-label {method} {variant}")
    inp = synth.config_inputs("c0")
    du, dis, _, _ = compare_run(inp["caps"], 300, model="two", method=method, relax=1.5,
                                alpha=0.5, variant=variant)
    print(f"max|du|={du:.3e} label disagreement={dis:.2e}")
    assert du <= TOL_U and dis <= TOL_LAB


@pytest.mark.parametrize("shape", [(77, 131), (1, 200), (150, 1), (65, 64), (64, 65), (3, 3), (1, 1)])
@pytest.mark.parametrize("tv", ["iso", "aniso"])
def test_ragged_shapes(shape, tv):
    banner(f"ragged {shape} {tv}")
    rng = np.random.default_rng(sum(shape))
    caps = synth.two_label_caps(rng.uniform(0, 1, size=shape))
    du, dis, _, _ = compare_run(caps, 120, model="two", method="eb", relax=1.5, alpha=0.3, tv=tv)
    assert du <= TOL_U and dis <= TOL_LAB


@pytest.mark.parametrize("n", [2, 3, 4, 8])
@pytest.mark.parametrize("method", ["fg", "eb"])
def test_potts_2d(n, method):
    banner(f"potts n={n} {method}")
    img, _ = synth.voronoi_image(96, 130, n, 0.15, 2000 + n, ncells=16)
    caps = synth.potts_caps(img, n)
    du, dis, _, _ = compare_run(caps, 200, model="potts", nlabels=n, method=method, alpha=0.3)
    print(f"max|du|={du:.3e} label disagreement={dis:.2e}")
    assert du <= TOL_U and dis <= TOL_LAB


@pytest.mark.parametrize("model,n", [("two", 2), ("potts", 3)])
def test_3d_unfused(model, n):
    banner(f"3d unfused {model} n={n}")
    vol = synth.ellipsoid_volume(20, 22, 37, 4, 0.1, 3001)
    caps = synth.two_label_caps(vol) if model == "two" else synth.potts_caps(vol, n)
    du, dis, _, _ = compare_run(caps, 100, model=model, nlabels=n, method="eb", relax=1.5,
                                alpha=0.4, variant="unfused")
    assert du <= TOL_U and dis <= TOL_LAB


@pytest.mark.parametrize("shape", [(20, 22, 37), (9, 8, 64), (1, 13, 70), (33, 5, 3)])
@pytest.mark.parametrize("method", ["fg", "eb"])
def test_3d_fused_two_label(shape, method):
    banner(f"3d fused {shape} {method}")
    vol = synth.ellipsoid_volume(*shape, 4, 0.1, 3003)
    caps = synth.two_label_caps(vol)
    du, dis, _, _ = compare_run(caps, 100, model="two", method=method, relax=1.5, alpha=0.4)
    assert du <= TOL_U and dis <= TOL_LAB


@pytest.mark.parametrize("storage", ["f32", "bf16"])
@pytest.mark.parametrize("shape", [(19, 21, 70), (40, 16, 64)])
def test_3d_fused_equals_unfused_bitwise(storage, shape):
    banner(f"3d bitwise {shape} {storage}")
    caps = synth.two_label_caps(synth.ellipsoid_volume(*shape, 5, 0.1, 3004))
    ref = None
    for variant in ("unfused", "fused"):
        s = gpu_solver(caps, model="two", method="eb", relax=1.5, alpha=0.4, storage=storage, variant=variant)
        s.step(23)
        torch.cuda.synchronize()
        g = gpu_fields(s)
        s.close()
        if ref is None:
            ref = g
        else:
            for f in ref:
                assert np.array_equal(ref[f], g[f]), f


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_3d_tile_height_and_slab_depth_bitwise(storage):
    """The 3-D sweep's launch shape (64 x 8 or 64 x 16 xy tiles, slab depths
    4 .. more than D) never changes the iterates: every combination gives the
    unfused passes' bits, on a volume ragged in every axis, across a gap
    check."""
    shape = (37, 45, 70)
    caps = synth.two_label_caps(synth.ellipsoid_volume(*shape, 5, 0.1, 3007))
    kw = dict(model="two", method="eb", relax=1.5, alpha=0.4, storage=storage, tol=0.0, max_iter=13,
              check_every=5)
    s = gpu_solver(caps, variant="unfused", **kw)
    s.solve()
    ref = gpu_fields(s)
    s.close()
    for rows in (8, 16):
        for sd in (0, 4, 5, 16, 64):
            banner(f"3d {storage} tile_rows={rows} slab_depth={sd}")
            s = gpu_solver(caps, tile_rows=rows, slab_depth=sd, **kw)
            s.solve()
            g = gpu_fields(s)
            s.close()
            for f in ref:
                assert np.array_equal(ref[f], g[f]), (rows, sd, f)


def test_3d_fused_gap_and_solve():
    banner("3d fused solve")
    caps = synth.two_label_caps(synth.ellipsoid_volume(24, 26, 30, 4, 0.1, 3005)).astype(np.float32).astype(np.float64)
    kw = dict(model="two", method="eb", relax=1.5, alpha=0.4, tol=1e-3, max_iter=3000, check_every=10)
    s = gpu_solver(caps, **kw)
    res = s.solve()
    assert res["status"] == 0 and res["iter"] % 10 == 0
    g = gpu_fields(s)
    s.close()
    pr = oracle_problem(caps.shape[1:], kw)
    st = oracle.init_state(pr, caps)
    oracle.step(pr, caps, st, res["iter"])
    e = oracle.energy(pr, caps, st)
    assert abs(res["rel_gap"] - e["rel_gap"]) < 1e-5
    assert np.max(np.abs(g["u"] - st.u)) <= TOL_U


def test_3d_full_size_one_step_random_state():
    """256^3 (the 3-D workload size, launched with the slab depth the solver
    picks for it), one iteration from a seeded random admissible state, every
    field compared with the oracle."""
    banner("3d one step 256^3 random state")
    inp = synth.config_inputs("c3")
    caps = inp["caps"].astype(np.float32).astype(np.float64)
    shape = caps.shape[1:]
    rs = synth.random_state(shape, 2, "two", 0.4, caps, seed=98)
    f32 = {k: v.astype(np.float32).astype(np.float64) for k, v in rs.items()}
    del rs
    s = gpu_solver(caps, model="two", method="eb", relax=1.5, alpha=0.4)
    for f in ("u", "q", "ps", "p"):
        s.write(f, torch.from_numpy(f32[f].astype(np.float32)))
    s.step(1)
    g = gpu_fields(s)
    s.close()
    pr = oracle_problem(shape, dict(model="two", method="eb", relax=1.5, alpha=0.4))
    st = oracle.state_from_arrays(pr, f32["u"], f32["q"], f32["ps"], f32["p"])
    oracle.step(pr, caps, st, 1)
    for f in ("u", "q", "ps", "p"):
        err = np.max(np.abs(g[f] - getattr(st, f)))
        assert err < 2e-5, (f, err)


def test_3d_full_size_fused_equals_unfused_bitwise():
    """256^3, 12 iterations (one gap check inside): the fused z-marching
    sweep at its production slab depth gives the unfused passes' bits."""
    banner("3d bitwise 256^3")
    caps = synth.config_inputs("c3")["caps"]
    ref = None
    for variant in ("unfused", "fused"):
        s = gpu_solver(caps, model="two", method="eb", relax=1.5, alpha=0.4, variant=variant,
                       tol=0.0, max_iter=12, check_every=10)
        s.solve()
        torch.cuda.synchronize()
        g = {f: s.read(f).cpu().numpy() for f in ("u", "q")}
        s.close()
        if ref is None:
            ref = g
        else:
            for f in ref:
                assert np.array_equal(ref[f], g[f]), f


def test_potts_3d_fused_request_runs_unfused():
    banner("potts 3d")
    vol = synth.ellipsoid_volume(12, 14, 18, 3, 0.1, 3006)
    caps = synth.potts_caps(vol, 4)
    du, dis, _, _ = compare_run(caps, 60, model="potts", nlabels=4, method="eb", alpha=0.4)
    assert du <= TOL_U and dis <= TOL_LAB


def _bits(g):
    return {k: v.copy() for k, v in g.items()}


@pytest.mark.parametrize("model,n,storage", [("two", 2, "f32"), ("two", 2, "bf16"),
                                             ("potts", 4, "f32"), ("potts", 8, "bf16")])
def test_fused_unfused_tiles_bitwise(model, n, storage):
    banner(f"bitwise fused/unfused/tiles {model} n={n} {storage}")
    if model == "two":
        caps = synth.config_inputs("c0", size=(70, 150))["caps"]
    else:
        img, _ = synth.voronoi_image(70, 150, n, 0.15, 7, ncells=12)
        caps = synth.potts_caps(img, n)
    ref = None
    for variant, tr in [("unfused", 0), ("fused", 8), ("fused", 16), ("fused", 32)]:
        s = gpu_solver(caps, model=model, nlabels=n, method="eb", relax=1.5, alpha=0.4,
                       storage=storage, variant=variant, tile_rows=tr)
        s.step(37)
        torch.cuda.synchronize()
        g = gpu_fields(s)
        s.close()
        if ref is None:
            ref = g
            continue
        for f in ref:
            assert np.array_equal(ref[f], g[f]), f"{variant} tile {tr} differs in {f}"


def test_one_step_full_size_random_state():
    """2048x2048 (the two-label benchmark size), one iteration from a seeded
    random admissible state written through the ABI, all fields compared."""
    banner("one step 2048^2 random state")
    inp = synth.config_inputs("c1")
    caps = inp["caps"].astype(np.float32).astype(np.float64)
    shape = caps.shape[1:]
    rs = synth.random_state(shape, 2, "two", 0.5, caps, seed=99)
    f32 = {k: v.astype(np.float32).astype(np.float64) for k, v in rs.items()}
    for method in ("fg", "eb"):
        s = gpu_solver(caps, model="two", method=method, relax=1.5, alpha=0.5)
        for f in ("u", "q", "ps", "p"):
            s.write(f, torch.from_numpy(f32[f].astype(np.float32)))
        s.step(1)
        g = gpu_fields(s)
        s.close()
        pr = oracle_problem(shape, dict(model="two", method=method, relax=1.5, alpha=0.5))
        st = oracle.state_from_arrays(pr, f32["u"], f32["q"], f32["ps"], f32["p"])
        oracle.step(pr, caps, st, 1)
        for f in ("u", "q", "ps", "p"):
            err = np.max(np.abs(g[f] - getattr(st, f)))
            assert err < 2e-5, (method, f, err)


def test_full_size_100_iterations():
    """2048x2048 config, 100 iterations of rpADMMII with relaxation 1.5."""
    banner("c1 2048^2 100 its")
    inp = synth.config_inputs("c1")
    du, dis, _, _ = compare_run(inp["caps"], 100, model="two", method="eb", relax=1.5, alpha=0.5)
    print(f"max|du|={du:.3e} label disagreement={dis:.2e}")
    assert du <= TOL_U and dis <= TOL_LAB


def test_config1_generator_512_full_500_iterations():
    banner("c1 generator 512^2 500 its")
    inp = synth.config_inputs("c1", size=(512, 512))
    du, dis, _, _ = compare_run(inp["caps"], 500, model="two", method="eb", relax=1.5, alpha=0.5)
    print(f"max|du|={du:.3e} label disagreement={dis:.2e}")
    assert du <= TOL_U and dis <= TOL_LAB


@pytest.mark.parametrize("model,n", [("two", 2), ("potts", 3), ("potts", 8)])
def test_gap_matches_oracle_on_random_state(model, n):
    banner(f"gap on random state {model} n={n}")
    shape = (57, 91)
    rng = np.random.default_rng(5)
    img = rng.uniform(0, 1, size=shape)
    caps = synth.two_label_caps(img) if model == "two" else synth.potts_caps(img, n)
    caps = caps.astype(np.float32).astype(np.float64)
    rs = synth.random_state(shape, n, model, 0.4, caps, seed=17)
    f32 = {k: v.astype(np.float32).astype(np.float64) for k, v in rs.items()}
    for tv in ("iso", "aniso"):
        s = gpu_solver(caps, model=model, nlabels=n, alpha=0.4, tv=tv)
        for f in ("u", "q", "ps", "p"):
            s.write(f, torch.from_numpy(f32[f].astype(np.float32)))
        g = s.gap()
        s.close()
        pr = oracle_problem(shape, dict(model=model, nlabels=n, alpha=0.4, tv=tv))
        e = oracle.energy(pr, caps, oracle.state_from_arrays(pr, f32["u"], f32["q"], f32["ps"], f32["p"]))
        for key in ("primal", "dual", "flow"):
            assert abs(g[key] - e[key]) <= 1e-9 * max(1.0, abs(e[key])), (tv, key, g[key], e[key])
        assert abs(g["resid_rms"] - e["resid_rms"]) <= 1e-9 * max(1.0, e["resid_rms"])


@pytest.mark.parametrize("variant", ["fused", "unfused"])
def test_solve_stops_at_checked_iterate(variant):
    """solve() stops at the first multiple of check_every whose gap <= tol and
    leaves the state at that iterate."""
    banner(f"solve stop {variant}")
    inp = synth.config_inputs("c0", size=(64, 96))
    caps = inp["caps"].astype(np.float32).astype(np.float64)
    kw = dict(model="two", method="eb", relax=1.5, alpha=0.5, tol=1e-3, max_iter=2000,
              check_every=10, variant=variant)
    s = gpu_solver(caps, **kw)
    res = s.solve()
    assert res["status"] == 0 and res["iter"] % 10 == 0 and res["rel_gap"] <= 1e-3
    k = res["iter"]
    g = gpu_fields(s)
    assert s.iter == k
    s.close()
    pr = oracle_problem(caps.shape[1:], kw)
    st, hist = oracle.solve(pr, caps, 2000, check_every=10, tol=1e-3)
    ks = [kk for kk, _ in hist]
    assert abs(ks[-1] - k) <= 10          # same stop up to one check of FP32 drift
    st_k = oracle.init_state(pr, caps)
    oracle.step(pr, caps, st_k, k)
    assert np.max(np.abs(g["u"] - st_k.u)) <= TOL_U
    e = oracle.energy(pr, caps, st_k)
    assert abs(res["rel_gap"] - e["rel_gap"]) < 1e-5


def test_solve_cap_and_zero_iterations():
    banner("solve cap")
    caps = synth.config_inputs("c0", size=(40, 40))["caps"]
    s = gpu_solver(caps, model="two", method="fg", alpha=0.5, tol=0.0, max_iter=25, check_every=10)
    res = s.solve()
    assert res["status"] == 1 and res["iter"] == 25 and s.iter == 25
    s.close()
    s = gpu_solver(caps, model="two", method="fg", alpha=0.5, tol=0.0, max_iter=0)
    res = s.solve()
    assert res["status"] == 1 and res["iter"] == 0
    s.close()


def test_invalid_parameters_rejected():
    caps = torch.ones((2, 8, 8), device="cuda")
    from paper_2004_11227_amd import maxflow as mfx
    for kw in [dict(alpha=-1.0), dict(relax=2.5), dict(a=3.0), dict(method="fg", relax=1.7),
               dict(model="potts", nlabels=5), dict(tile_rows=12), dict(depth=3),
               dict(depth=2, variant="unfused"), dict(depth=2, method="dr")]:
        with pytest.raises(mfx.MaxflowError):
            mfx.Solver(caps if kw.get("model") != "potts" else torch.ones((5, 8, 8), device="cuda"), **kw)


def test_export_import_resume_bitwise():
    banner("checkpoint resume")
    caps = synth.config_inputs("c0", size=(50, 70))["caps"]
    kw = dict(model="two", method="eb", relax=1.5, alpha=0.5)
    a = gpu_solver(caps, **kw)
    a.step(40)
    ga = gpu_fields(a)
    b = gpu_solver(caps, **kw)
    b.step(17)
    blob = b.export_state()
    c = gpu_solver(caps, **kw)
    c.import_state(blob, 17)
    c.step(23)
    gc = gpu_fields(c)
    for f in ga:
        assert np.array_equal(ga[f], gc[f])
    for s in (a, b, c):
        s.close()


def test_autotune_keeps_state_and_caches(tmp_path, monkeypatch):
    """maxflow_tune times the candidate launch shapes (tile height, fusion
    depth, 3-D slab depth) without moving the iterate; the tuned solver
    continues bit-identically; the choice is cached and reused."""
    banner("autotune")
    from paper_2004_11227_amd import maxflow as mfx
    from paper_2004_11227_amd import tuning
    monkeypatch.setenv("MF_TUNING_CACHE", str(tmp_path / "tune.json"))
    tuning.clear()
    caps = synth.config_inputs("c1", size=(300, 333))["caps"]
    kw = dict(model="two", method="eb", relax=1.5, alpha=0.5)
    ref = gpu_solver(caps, depth=1, **kw)
    ref.step(7)
    s = gpu_solver(caps, **kw)
    s.step(5)
    before = gpu_fields(s)
    best, cands = s.tune(sweeps=5)
    shapes = {(c["tile_rows"], c["depth"]) for c in cands}
    assert shapes == {(8, 1), (16, 1), (32, 1), (16, 2), (32, 2)} and all(c["us_per_iter"] > 0 for c in cands)
    assert (best["tile_rows"], best["depth"]) in shapes and s.iter == 5
    assert best["tile_rows"] == s.params.tile_rows and best["depth"] == s.params.depth
    after = gpu_fields(s)
    for f in before:
        assert np.array_equal(before[f], after[f]), f
    s.step(2)
    a, b = gpu_fields(ref), gpu_fields(s)
    for f in a:
        assert np.array_equal(a[f], b[f]), f
    s.close()
    ref.close()
    # only the tile height when the depth is fixed
    d = gpu_solver(caps, depth=2, **kw)
    best, cands = d.tune(sweeps=3, what=mfx.MF_TUNE_TILE)
    assert {(c["tile_rows"], c["depth"]) for c in cands} == {(16, 2), (32, 2)} and best["depth"] == 2
    d.close()
    # the cache: tuned on a miss, read back on a hit
    t = gpu_solver(caps, tile_rows="auto", **kw)
    got = tuning.lookup(caps.shape[1:], t.device, **kw)
    assert got == dict(tile_rows=t.params.tile_rows, depth=t.params.depth, slab_depth=t.params.slab_depth)
    t.close()
    tuning.clear()
    u = gpu_solver(caps, tile_rows="auto", **kw)   # from the file, no tuning
    assert (u.params.tile_rows, u.params.depth) == (got["tile_rows"], got["depth"])
    u.close()
    tuning.clear()
    # 3-D: tile height x slab depth
    caps3 = synth.two_label_caps(synth.ellipsoid_volume(40, 48, 70, 4, 0.1, 3008))
    v = gpu_solver(caps3, model="two", method="eb", relax=1.5, alpha=0.4)
    v.step(3)
    before = gpu_fields(v)
    best, cands = v.tune(sweeps=3)
    assert {(c["tile_rows"], c["slab_depth"]) for c in cands} == {(r, z) for r in (8, 16) for z in (4, 8, 16, 32)}
    assert v.iter == 3 and best["slab_depth"] == v.params.slab_depth
    # with the slab depth given, only the tile height is free
    _, c2 = v.tune(sweeps=2, what=mfx.MF_TUNE_TILE)
    assert {(c["tile_rows"], c["slab_depth"]) for c in c2} == {(8, best["slab_depth"]), (16, best["slab_depth"])}
    after = gpu_fields(v)
    for f in before:
        assert np.array_equal(before[f], after[f]), f
    v.step(2)
    w = gpu_solver(caps3, model="two", method="eb", relax=1.5, alpha=0.4, variant="unfused")
    w.step(5)
    a, b = gpu_fields(v), gpu_fields(w)
    for f in a:
        assert np.array_equal(a[f], b[f]), f
    v.close()
    w.close()
    # fused rPDRQ: 16 or 32 rows; in-place rPDRQ times nothing
    r = gpu_solver(caps, model="two", method="dr", alpha=0.5)
    r.step(2)
    before = gpu_fields(r)
    best, cands = r.tune(sweeps=3)
    assert {c["tile_rows"] for c in cands} == {16, 32} and r.iter == 2
    after = gpu_fields(r)
    for f in before:
        assert np.array_equal(before[f], after[f]), f
    r.close()
    r = gpu_solver(caps, model="two", method="dr", alpha=0.5, variant="unfused")
    best, cands = r.tune(sweeps=3)
    assert cands == []
    r.close()


@pytest.mark.parametrize("storage", ["f32", "bf16"])
@pytest.mark.parametrize("shape", [(1, 1), (1, 70), (70, 1), (17, 130), (65, 64), (200, 333)])
def test_depth2_equals_depth1_bitwise(storage, shape):
    """Two iterations per pass (iterate k+1 kept in LDS) give the depth-1
    iterates bit for bit, for odd and even step counts and both tile
    heights."""
    banner(f"depth2 {shape} {storage}")
    caps = synth.two_label_caps(synth.ellipse_image(*shape, 3, 0.15, 3100))
    kw = dict(model="two", method="eb", relax=1.5, alpha=0.5, storage=storage)
    ref = gpu_solver(caps, depth=1, **kw)
    runs = [gpu_solver(caps, depth=2, tile_rows=tr, **kw) for tr in (16, 32)]
    for n in (2, 1, 4, 3):
        ref.step(n)
        a = gpu_fields(ref)
        for s in runs:
            s.step(n)
            b = gpu_fields(s)
            for f in a:
                assert np.array_equal(a[f], b[f]), (n, s.params.tile_rows, f)
    for s in runs + [ref]:
        s.close()


@pytest.mark.parametrize("method", ["fg", "eb"])
def test_depth2_solve_stops_like_depth1(method):
    """solve(): the gap is fused into the two-iteration pass at the checked
    iterate; the stop iterate, the gap and the accepted state (rolled back
    past passes already queued) equal the depth-1 solve."""
    banner(f"depth2 solve {method}")
    caps = synth.config_inputs("c1", size=(257, 300))["caps"]
    kw = dict(model="two", method=method, relax=1.5, alpha=0.5, tol=2e-3, max_iter=997, check_every=10)
    out = []
    for depth in (1, 2):
        s = gpu_solver(caps, depth=depth, **kw)
        res = s.solve()
        out.append((res, gpu_fields(s)))
        s.step(3)   # continue from the accepted iterate
        out.append((None, gpu_fields(s)))
        s.close()
    (r1, f1), (_, g1), (r2, f2), (_, g2) = out
    assert r1["iter"] == r2["iter"] and r1["status"] == r2["status"] and r1["iter"] < 997
    assert r1["rel_gap"] == r2["rel_gap"]
    for f in f1:
        assert np.array_equal(f1[f], f2[f]), f
        assert np.array_equal(g1[f], g2[f]), f


def test_depth2_cap_reached_odd_max_iter():
    banner("depth2 odd cap")
    caps = synth.config_inputs("c1", size=(130, 190))["caps"]
    kw = dict(model="two", method="eb", relax=1.5, alpha=0.5, tol=0.0, max_iter=33, check_every=10)
    res = []
    for depth in (1, 2):
        s = gpu_solver(caps, depth=depth, **kw)
        r = s.solve()
        res.append((r, gpu_fields(s)))
        s.close()
    assert res[0][0]["iter"] == res[1][0]["iter"] == 33
    for f in res[0][1]:
        assert np.array_equal(res[0][1][f], res[1][1][f]), f
