"""The solve's first iteration from the initial point runs as a pointwise
pass (with q^0 = 0 and p_t^0 = p_s^0 the stencil terms are exactly zero);
its iterates must equal plain sweeps bit for bit, and a solve after a reset
must repeat itself exactly.  The check at iterate 0 then leads to the same
stop iteration and gap as before."""
import numpy as np
import pytest

from paper_2004_11227_amd import synth

from _gpu import banner, gpu_fields, gpu_solver, need_gpu

pytestmark = pytest.mark.gpu

CASES = [((70, 131), dict(method="eb", relax=1.5), "f32", 1),
         ((70, 131), dict(method="fg", relax=1.3), "bf16", 2),
         ((64, 256), dict(method="eb", relax=1.5, tv="aniso"), "f32", 2),
         ((20, 37, 50), dict(method="eb", relax=1.5), "f32", 1),
         ((20, 37, 50), dict(method="fg", relax=1.0), "bf16", 1)]


@pytest.mark.parametrize("shape,kw,storage,depth", CASES)
def test_pointwise_first_iteration_is_bitwise(shape, kw, storage, depth):
    need_gpu()
    banner(f"first iteration {shape} {kw} {storage} depth {depth}")
    if len(shape) == 2:
        caps = synth.two_label_caps(synth.ellipse_image(*shape, 6, 0.1, 91))
    else:
        caps = synth.two_label_caps(synth.ellipsoid_volume(*shape, 5, 0.1, 92))
    common = dict(model="two", alpha=0.45, storage=storage, check_every=10, **kw)
    if len(shape) == 2:
        common["depth"] = depth
    # a solve that runs exactly 20 iterations (tol 0: no early stop)
    a = gpu_solver(caps, tol=0.0, max_iter=20, **common)
    ga = a.solve()
    assert ga["iter"] == 20
    fa = gpu_fields(a)
    # plain sweeps from the same initial point
    b = gpu_solver(caps, tol=0.0, max_iter=20, **common)
    b.step(20)
    fb = gpu_fields(b)
    for f in fa:
        assert np.array_equal(fa[f], fb[f]), f
    # after a reset the solve repeats itself, decision and gap included
    a.reset()
    ga2 = a.solve()
    fa2 = gpu_fields(a)
    for f in fa:
        assert np.array_equal(fa[f], fa2[f]), f
    assert ga2["iter"] == ga["iter"] and ga2["status"] == ga["status"]
    assert abs(ga2["rel_gap"] - ga["rel_gap"]) <= 1e-12 * max(1.0, abs(ga["rel_gap"]))
    # a step after the reset takes the sweep path; the solve that follows
    # starts from iterate 1 and ends where the other did
    a.reset()
    a.step(1)
    ga3 = a.solve()
    assert ga3["iter"] == 20
    fa3 = gpu_fields(a)
    for f in fa:
        assert np.array_equal(fa[f], fa3[f]), f
    a.close()
    b.close()


def test_first_check_gives_the_same_stop():
    """A converging 2-D solve: stop iteration, final gap and fields with the
    pointwise first iteration equal those of a solve whose first check runs
    the gap-carrying sweep (forced by writing back the initial u)."""
    need_gpu()
    banner("first iteration: stop iteration unchanged")
    caps = synth.two_label_caps(synth.ellipse_image(128, 160, 6, 0.1, 93))
    kw = dict(model="two", method="eb", relax=1.5, alpha=0.5, tol=1e-4, check_every=10, max_iter=1000)
    a = gpu_solver(caps, **kw)
    ga = a.solve()
    b = gpu_solver(caps, **kw)
    b.write("u", b.read("u"))   # a field write marks the state as no longer the untouched initial point
    gb = b.solve()
    assert ga["iter"] == gb["iter"] and ga["status"] == gb["status"] == 0
    assert abs(ga["rel_gap"] - gb["rel_gap"]) <= 1e-9 * abs(gb["rel_gap"])
    fa, fb = gpu_fields(a), gpu_fields(b)
    for f in fa:
        assert np.array_equal(fa[f], fb[f]), f
    a.close()
    b.close()


@pytest.mark.parametrize("shape,storage", [((70, 131), "f32"), ((20, 37, 50), "bf16")])
def test_initial_point_appears_where_needed(shape, storage):
    """The initial point is stored only when something needs it: fields read
    right after creation, and a solve that stops at its first check (a
    tolerance every iterate meets), give u = 0, q = 0, p_t = p_s =
    min(C_s, C_t) in the storage type."""
    need_gpu()
    banner(f"initial point on demand {shape} {storage}")
    if len(shape) == 2:
        caps = synth.two_label_caps(synth.ellipse_image(*shape, 6, 0.1, 94))
    else:
        caps = synth.two_label_caps(synth.ellipsoid_volume(*shape, 5, 0.1, 95))
    kw = dict(model="two", method="eb", relax=1.5, alpha=0.45, storage=storage, check_every=10, max_iter=100)
    ref = gpu_solver(caps, depth=1, **kw) if len(shape) == 2 else gpu_solver(caps, **kw)
    f0 = gpu_fields(ref)
    m = np.minimum(caps[0], caps[1]).astype(np.float32)
    if storage == "bf16":   # round to nearest even, as the store does
        b = m.view(np.uint32).astype(np.uint64)
        b = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
        m = b.astype(np.uint32).view(np.float32)
    assert np.all(f0["u"] == 0) and np.all(f0["q"] == 0)
    assert np.array_equal(f0["ps"], m.astype(np.float64)) and np.array_equal(f0["p"][0], m.astype(np.float64))
    s = gpu_solver(caps, tol=1e3, **kw) if len(shape) == 3 else gpu_solver(caps, tol=1e3, depth=1, **kw)
    g = s.solve()
    assert g["iter"] == 0 and g["status"] == 0
    f1 = gpu_fields(s)
    for f in f0:
        assert np.array_equal(f0[f], f1[f]), f
    s.close()
    ref.close()
