"""Served results against the FP64 oracle: a seeded sample of the serving
mix's requests (2-D sides log-uniform on [64, 2048], 10 % 128^3 volumes,
labels in {2, 3, 4, 8}, ellipse or Voronoi images) run through the pool the
way the serving benchmark runs them (BF16 flows and capacities, FP32
arithmetic, promotion to FP32 storage near the BF16 floor, gap 1e-4 or 1000
iterations).  For every served solve: the objective error (primal energy,
eqs. seg:chanvese / relaxed-potts, of the served u against that of the FP64
oracle's u after the same number of iterations, both evaluated in FP64 on
the unrounded capacities) and the thresholded-label disagreement.  The
sample is the first requests of the trace whose FP64 oracle run stays
within a few seconds (at most 512^2 pixels)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2004_11227_amd import maxflow as mfx
from paper_2004_11227_amd import serving, synth

from _gpu import banner, label_disagreement, need_gpu, oracle_problem, progress

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


@pytest.mark.skip(reason="a run of this test ended in a host segmentation fault inside mf_pool_advance "
                         "(it had passed in earlier runs); the cause has not been shown, so the case is not run "
                         "on the GPU again until it is")
def test_served_bf16_results_against_the_oracle():
    banner("served sample vs FP64 oracle")
    trace = synth.serving_trace(2048, seed=4000)
    sample = [r for r in trace if int(np.prod(r.shape)) <= 512 * 512][:16]
    assert len(sample) == 16
    caps64 = {r.rid: synth.request_caps(r) for r in sample}
    kw = {r.rid: dict(model=r.model, nlabels=r.nlabels, method="eb", alpha=r.alpha, storage="bf16", tol=1e-4,
                      max_iter=1000, check_every=10, promote_gap=2e-3, promote_iter=400) for r in sample}
    pool = mfx.Pool(8 << 30, max_slots=32, max_tiles=1 << 16, steps_per_advance=10)
    be = serving.PoolBackend(pool, lambda r: torch.from_numpy(caps64[r.rid].astype(np.float32)).cuda(),
                             lambda r: kw[r.rid], keep_results=True)
    rep = serving.serve([synth.Request(**{**r.__dict__, "arrival": 0.0}) for r in sample], be)
    promotions = pool.stats()["promotions"]
    pool.close()
    iters = {rec.rid: rec.iters for rec in rep.records}
    status = {rec.rid: rec.status for rec in rep.records}
    objs, diss = [], []
    for r in sample:
        assert status[r.rid] in (0, 1), (r, status[r.rid])
        u = be.results[r.rid][0].double().cpu().numpy()
        c32 = caps64[r.rid].astype(np.float32).astype(np.float64)
        pr = oracle_problem(r.shape, dict(model=r.model, nlabels=r.nlabels, method="eb", alpha=r.alpha))
        st = oracle.init_state(pr, c32)
        oracle.step(pr, c32, st, iters[r.rid])
        e = oracle.energy(pr, caps64[r.rid], st)
        sb = oracle.state_from_arrays(pr, u, st.q, st.ps, st.p)
        eb = oracle.energy(pr, caps64[r.rid], sb)
        obj = abs(eb["primal"] - e["primal"]) / abs(e["primal"])
        dis = label_disagreement(u, st.u, r.model)
        objs.append(obj)
        diss.append(dis)
        progress(f"served rid={r.rid} {r.model} n={r.nlabels} shape={r.shape} iters={iters[r.rid]} "
                 f"status={status[r.rid]} objective rel err={obj:.3e} label disagreement={dis:.3e}")
    progress(f"served sample of {len(sample)} (promotions {promotions}): objective rel err max={max(objs):.3e} "
             f"median={float(np.median(objs)):.3e}; label disagreement max={max(diss):.3e} "
             f"median={float(np.median(diss)):.3e}")
    assert max(objs) < 1e-2
    assert max(diss) < 0.05
