"""The allocation-free entry point maxflow_solve_static, through the C ABI,
against the entry points it stands for (maxflow_create + maxflow_solve +
maxflow_read_u + maxflow_labels with a caller workspace): the same kernels,
so u, labels, the accepted iterate and its gap must agree bit for bit.  Two
calls in a row share the static device array, the second on a smaller input
(and a third on a different model), so nothing may depend on the contents a
previous call left there."""
import numpy as np
import pytest
import torch

from paper_2004_11227_amd import maxflow as mfx
from paper_2004_11227_amd import synth

from _gpu import banner, need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _reference(caps_t, **kw):
    s = mfx.Solver(caps_t, **kw)
    g = s.solve()
    u = s.u().cpu().numpy()
    lab = s.labels().cpu().numpy()
    s.close()
    return g, u, lab


def _static(caps_t, **kw):
    g, u, lab = mfx.solve_static(caps_t, **kw)
    torch.cuda.synchronize()
    return g, u.cpu().numpy(), lab.cpu().numpy()


def _same(a, b):
    ga, ua, la = a
    gb, ub, lb = b
    assert ga["iter"] == gb["iter"] and ga["status"] == gb["status"], (ga, gb)
    for key in ("primal", "dual", "rel_gap", "resid_rms", "flow"):
        assert ga[key] == gb[key], (key, ga[key], gb[key])
    assert np.array_equal(ua, ub)
    assert np.array_equal(la, lb)


def _cases():
    # first call: Potts n = 3 at 512 x 600 (35 MiB of workspace), FP32
    img, _ = synth.voronoi_image(512, 600, 3, 0.15, 7001, ncells=24)
    c1 = torch.from_numpy(synth.potts_caps(img, 3).astype(np.float32)).cuda()
    k1 = dict(model="potts", nlabels=3, method="eb", relax=1.5, alpha=0.3, tol=1e-4, max_iter=400, check_every=10)
    # second call, smaller: two-label 200 x 333 (depth-2 passes), converges
    c2 = torch.from_numpy(synth.two_label_caps(synth.ellipse_image(200, 333, 6, 0.1, 7002))
                          .astype(np.float32)).cuda()
    k2 = dict(model="two", method="eb", relax=1.5, alpha=0.5, tol=1e-4, max_iter=1000, check_every=10)
    # third: 3-D BF16 two-label, stopped by the cap
    c3 = torch.from_numpy(synth.two_label_caps(synth.ellipsoid_volume(24, 40, 70, 5, 0.1, 7003))
                          .astype(np.float32)).cuda()
    k3 = dict(model="two", method="fg", alpha=0.4, storage="bf16", tol=0.0, max_iter=150, check_every=10)
    return [(c1, k1), (c2, k2), (c3, k3)]


def test_static_equals_create_solve_bitwise_on_consecutive_calls():
    banner("solve_static vs create/solve, consecutive calls")
    cases = _cases()
    outs = [_static(c, **k) for c, k in cases]           # back to back on the shared array
    for (c, k), o in zip(cases, outs):
        _same(o, _reference(c, **k))
    assert outs[1][0]["status"] == 0 and outs[2][0]["status"] == 1 and outs[2][0]["iter"] == 150
    # the same calls again after other work, largest last: still the same bits
    for (c, k), o in zip(cases[::-1], outs[::-1]):
        _same(_static(c, **k), o)


def test_static_rejects_problems_above_the_scratch():
    banner("solve_static size limit")
    shape = (2048, 2048)   # 192 MiB of workspace
    assert mfx.workspace_bytes(mfx.make_params(shape, model="two")) > mfx.STATIC_SCRATCH_BYTES
    caps = torch.zeros((2,) + shape, dtype=torch.float32, device="cuda")
    with pytest.raises(mfx.MaxflowError) as ei:
        mfx.solve_static(caps, model="two", alpha=0.5)
    assert ei.value.status == mfx.MF_ENOMEM
    assert "static scratch" in str(ei.value)
    with pytest.raises(mfx.MaxflowError) as ei:
        mfx.solve_static(caps[:, :8, :8].contiguous(), model="two", alpha=-1.0)
    assert ei.value.status == mfx.MF_EINVAL
