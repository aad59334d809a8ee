"""Hand-worked minimum cuts (tests/golden/hand_worked_cuts.json) against the
oracle's converged relaxed solutions and against the brute-force search."""
import json
import os

import numpy as np
import pytest

import oracle

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hand_worked_cuts.json")))


@pytest.mark.parametrize("case", GOLD["cases"], ids=[c["name"] for c in GOLD["cases"]])
@pytest.mark.parametrize("method", ["fg", "eb", "dr"])
def test_hand_worked(case, method):
    shape = tuple(case["shape"])
    if case["model"] == "two":
        caps = np.array([case["C_s"], case["C_t"]], dtype=np.float64)
        pr = oracle.Problem(shape, model="two", method=method, tv="aniso", alpha=case["alpha"])
        best, lab, _ = oracle.brute_force_binary(caps, case["alpha"])
    else:
        caps = np.array(case["C"], dtype=np.float64)
        pr = oracle.Problem(shape, model="potts", nlabels=caps.shape[0], method=method,
                            tv="aniso", alpha=case["alpha"])
        best, lab, _ = oracle.brute_force_potts(caps, case["alpha"])
    assert abs(best - case["min_energy"]) < 1e-12
    assert np.array_equal(lab, np.array(case["labels"]))
    st, hist = oracle.solve(pr, caps, 50000, check_every=20, tol=1e-12)
    e = hist[-1][1]
    assert abs(e["primal"] - case["min_energy"]) < 1e-9
    got = oracle.labels(pr, st.u if case["model"] == "potts" else st.u[0])
    assert np.array_equal(got, np.array(case["labels"]))
