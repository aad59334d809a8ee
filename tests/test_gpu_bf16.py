"""BF16 flow/capacity storage with FP32 arithmetic: objective error and label
disagreement against the FP64 oracle (run on the unrounded capacities)."""
import numpy as np
import pytest

import oracle
from paper_2004_11227_amd import synth

from _gpu import banner, gpu_fields, gpu_solver, label_disagreement, need_gpu, oracle_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


@pytest.mark.parametrize("model,n,method", [("two", 2, "eb"), ("potts", 4, "eb"), ("potts", 8, "fg"),
                                            ("two", 2, "dr")])
def test_bf16_error_vs_fp64(model, n, method):
    banner(f"bf16 {model} n={n} {method}")
    shape = (160, 192)
    if model == "two":
        caps = synth.config_inputs("c1", size=shape)["caps"]
        alpha = 0.5
    else:
        img, _ = synth.voronoi_image(*shape, n, 0.15, 2000 + n, ncells=24)
        caps = synth.potts_caps(img, n)
        alpha = 0.3
    iters = 300
    kw = dict(model=model, nlabels=n, method=method, alpha=alpha)
    s = gpu_solver(caps, storage="bf16", **kw)
    s.step(iters)
    g = gpu_fields(s)
    gap = s.gap()
    s.close()
    pr = oracle_problem(shape, kw)
    st = oracle.init_state(pr, caps)
    oracle.step(pr, caps, st, iters)
    e = oracle.energy(pr, caps, st)
    # primal energy of the BF16 run's u, evaluated exactly on the FP64 capacities
    st_b = oracle.state_from_arrays(pr, g["u"], st.q, st.ps, st.p)
    if method == "dr":
        st_b.zq, st_b.zs, st_b.zp = st.zq, st.zs, st.zp
    eb = oracle.energy(pr, caps, st_b)
    obj_err = abs(eb["primal"] - e["primal"]) / abs(e["primal"])
    dis = label_disagreement(g["u"], st.u, model)
    print(f"bf16 objective rel err={obj_err:.3e} label disagreement={dis:.3e} "
          f"gpu gap={gap['rel_gap']:.3e} fp64 gap={e['rel_gap']:.3e}")
    assert obj_err < 5e-3
    assert dis < 0.02


def _bf16_nearest_even(x: np.ndarray) -> np.ndarray:
    """BF16 rounding from its definition: of the two BF16 neighbours of x
    (the truncation and the next value away from zero), take the nearer in
    exact arithmetic, the one with an even last mantissa bit on a tie."""
    u = x.astype(np.float32).view(np.uint32)
    lo = (u & np.uint32(0xFFFF0000))
    hi = lo + np.uint32(0x10000)
    flo = lo.view(np.float32).astype(np.float64)
    fhi = hi.view(np.float32).astype(np.float64)
    xv = x.astype(np.float64)
    dlo, dhi = np.abs(xv - flo), np.abs(fhi - xv)
    even_lo = ((lo >> np.uint32(16)) & np.uint32(1)) == 0
    pick_hi = (dhi < dlo) | ((dhi == dlo) & ~even_lo)
    return np.where(pick_hi, fhi, flo).astype(np.float32)


def test_bf16_storage_rounds_to_nearest_even():
    """Values written into BF16 flow storage read back rounded to nearest,
    ties to even: random values, exact ties (odd and even), values just off
    a tie, small normals, large magnitudes and zeros of both signs."""
    import torch
    shape = (64, 96)
    rng = np.random.default_rng(7)
    n = 2 * shape[0] * shape[1]
    base = rng.normal(scale=3.0, size=n).astype(np.float32)
    u = base.view(np.uint32) & np.uint32(0xFFFF0000)
    ties = (u | np.uint32(0x8000)).view(np.float32)                 # exactly halfway
    near = (u | np.uint32(0x8001)).view(np.float32)                 # just above halfway
    below = (u | np.uint32(0x7FFF)).view(np.float32)                # just below halfway
    vals = np.concatenate([base, ties, near, below,
                           np.array([0.0, -0.0, 1e-30, -3e-35, 3e38, -3.3e38, 1.0, 65504.0], np.float32)])
    vals = np.resize(vals, n).astype(np.float32)
    caps = np.ones((2,) + shape)
    s = gpu_solver(caps, model="two", method="eb", storage="bf16", variant="unfused")
    s.write("q", torch.from_numpy(vals.reshape((2,) + shape)))
    got = s.read("q").cpu().numpy().reshape(-1)
    s.close()
    expect = _bf16_nearest_even(vals)
    assert np.array_equal(got.view(np.uint32), expect.view(np.uint32))
