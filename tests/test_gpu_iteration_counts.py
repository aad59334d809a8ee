"""Iteration counts of the paper's methods on the synthetic stand-ins, in
the manner of Tables 1-2: iterate until the relative error of the primal
energy, (P(u^k) - E*) / E*, is below epsilon, with E* the primal energy at
the end of a long FP64 oracle run of rpADMMII: to a relative primal-dual gap
of 1e-10 for two labels; for four labels the relaxed gap closes sublinearly,
so 20000 iterations bound E* to within a relative 1e-6, ten times below the
smallest epsilon.  The solver runs on
the GPU through the C ABI (FP32 state, FP64 energy).  Parameters are the
paper's: alpha = 0.5, c = 0.3, a = 8; rpADMMI r = 1.618, pADMMI r = 1,
rpADMMII rho = 1.9, rPDRQ rho = 1.9 with (sigma, tau) = (0.2, 1) for two
labels and (5, 0.4) for four, ALG1 sigma = 0.4, tau = 1 / (L^2 sigma).

The images of the tables are not available, so the counts are not the
tables' counts; the test prints them and checks the orderings of the tables
that the stand-ins reproduce.  MF_ITERATION_TABLE=<file.json> saves them.

The iteration counts are decided on the FP64 energy of the FP32 iterates;
the gap reduction's atomic summation order can change its last bits between
runs, far below the margins of the asserted orderings."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2004_11227_amd import synth

from _gpu import banner, gpu_solver, need_gpu

pytestmark = pytest.mark.gpu

EPS = (1e-4, 1e-5)
RELAX = {"ty": 1.0, "cp": 1.0, "fg1": 1.0, "fg": 1.618, "eb": 1.9, "dr": 1.9}
NAMES = {"ty": "pADMM-TY", "cp": "ALG1", "fg1": "pADMMI", "fg": "rpADMMI", "eb": "rpADMMII", "dr": "rPDRQ"}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def _e_star(caps, model, n, alpha):
    pr = oracle.Problem(caps.shape[1:], model=model, nlabels=n, method="eb", alpha=alpha)
    if model == "two":
        st, hist = oracle.solve(pr, caps, 100000, check_every=50, tol=1e-10)
        bound = 1e-10
    else:
        st, hist = oracle.solve(pr, caps, 20000, check_every=1000, tol=0.0)
        bound = 1e-6
    e = hist[-1][1]
    assert e["rel_gap"] <= bound
    return e["primal"]


def _count(caps, model, n, alpha, key, e_star, cap_iters):
    method = "fg" if key == "fg1" else key
    s = gpu_solver(caps, model=model, nlabels=n, method=method, relax=RELAX[key], alpha=alpha, tol=0.0,
                   max_iter=cap_iters)
    out = {}
    for k in range(1, cap_iters + 1):
        s.step(1)
        err = (s.gap()["primal"] - e_star) / e_star
        for eps in EPS:
            if eps not in out and err <= eps:
                out[eps] = k
        if len(out) == len(EPS):
            break
    s.close()
    return {eps: out.get(eps) for eps in EPS}


def _table(caps, model, n, alpha, keys, cap_iters):
    caps = caps.astype(np.float32).astype(np.float64)
    e_star = _e_star(caps, model, n, alpha)
    rows = {k: _count(caps, model, n, alpha, k, e_star, cap_iters) for k in keys}
    for k in keys:
        print(f"  {NAMES[k]:9s} " + "  ".join(f"eps={eps:.0e}: {rows[k][eps]}" for eps in EPS), flush=True)
    return rows


def _save(name, rows):
    out = os.environ.get("MF_ITERATION_TABLE")
    if out:
        d = json.load(open(out)) if os.path.exists(out) else {}
        d[name] = {NAMES[k]: {f"{e:.0e}": v[e] for e in EPS} for k, v in rows.items()}
        json.dump(d, open(out, "w"), indent=1)


def test_two_label_iteration_counts():
    banner("iteration counts, two labels (40-ellipse stand-in, 256^2)")
    caps = synth.config_inputs("c1", size=(256, 256))["caps"]
    rows = _table(caps, "two", 2, 0.5, ["ty", "cp", "fg1", "fg", "eb", "dr"], 6000)
    _save("two_label_256", rows)
    for k, v in rows.items():
        assert v[1e-4] is not None, NAMES[k]
    # Table 1's order of these four at epsilon = 1e-4: rpADMMII, rpADMMI,
    # pADMM-TY, ALG1 (rPDRQ, first in the table, is slower on this stand-in)
    n = {k: v[1e-4] for k, v in rows.items()}
    assert n["eb"] <= n["fg"] <= n["ty"] < n["cp"]


def test_four_label_iteration_counts():
    banner("iteration counts, four labels (Voronoi stand-in, 96^2)")
    img, _ = synth.voronoi_image(96, 96, 4, 0.15, 2004, ncells=24)
    caps = synth.potts_caps(img, 4)
    rows = _table(caps, "potts", 4, 0.5, ["ty", "cp", "fg1", "fg", "eb", "dr"], 6000)
    _save("four_label_96", rows)
    for k, v in rows.items():
        assert v[1e-4] is not None, NAMES[k]
    # Table 2's order at epsilon = 1e-4: rpADMMII before rpADMMI before
    # pADMMI before ALG1, rPDRQ with the rpADMM methods
    n = {k: v[1e-4] for k, v in rows.items()}
    assert n["eb"] < n["fg"] < n["fg1"] < n["cp"]
    assert n["dr"] < n["fg1"]
