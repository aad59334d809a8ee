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
