"""Shared helpers for the GPU parity tests: run the HIP solver and the FP64
oracle on the same seeded inputs and compare."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle

try:  # the binding must load the real library; there is no fallback
    from paper_2004_11227_amd import maxflow as mfx
except Exception:  # pragma: no cover
    mfx = None


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    mfx.lib()


def banner(msg: str):
    print(f"\n[case] {msg}", flush=True)


def gpu_solver(caps: np.ndarray, **kw):
    t = torch.from_numpy(np.ascontiguousarray(caps, dtype=np.float32)).cuda()
    return mfx.Solver(t, **kw)


def oracle_problem(shape, kw) -> oracle.Problem:
    return oracle.Problem(shape, model=kw.get("model", "two"), method=kw.get("method", "eb"),
                          tv=kw.get("tv", "iso"), nlabels=kw.get("nlabels", 2),
                          alpha=kw.get("alpha", 0.5), c=kw.get("c", 0.0), relax=kw.get("relax", 0.0),
                          sigma=kw.get("sigma", 0.0), tau=kw.get("tau", 0.0), a=kw.get("a", 0.0),
                          a_tilde=kw.get("a_tilde", 0.0), a1=kw.get("a1", 0.0), a2=kw.get("a2", 0.0),
                          gs_sweeps=kw.get("gs_sweeps", 0), relax0=kw.get("relax0", 0.0),
                          relax_ramp=kw.get("relax_ramp", 0))


def gpu_fields(s) -> dict:
    out = {f: s.read(f).double().cpu().numpy() for f in ("u", "q", "ps", "p")}
    out["q"] = out["q"].reshape((s.L, s.ndim) + s.shape)
    out["ps"] = out["ps"].reshape(s.shape)
    if s.params.method == 2:
        for f in ("zq", "zs", "zp"):
            out[f] = s.read(f).double().cpu().numpy()
        out["zq"] = out["zq"].reshape((s.L, s.ndim) + s.shape)
        out["zs"] = out["zs"].reshape(s.shape)
    return out


def label_disagreement(u_gpu, u_or, model) -> float:
    if model == "two":
        a, b = u_gpu[0] > 0.5, u_or[0] > 0.5
    else:
        a, b = np.argmax(u_gpu, 0), np.argmax(u_or, 0)
    return float(np.mean(a != b))


def compare_run(caps, iters, **kw):
    """Run `iters` iterations on both sides from the initial point; return
    (max |u - u_oracle|, label disagreement, gpu fields, oracle state)."""
    shape = caps.shape[1:]
    s = gpu_solver(caps, **kw)
    s.step(iters)
    torch.cuda.synchronize()
    g = gpu_fields(s)
    pr = oracle_problem(shape, kw)
    st = oracle.init_state(pr, caps.astype(np.float32).astype(np.float64))
    oracle.step(pr, caps.astype(np.float32).astype(np.float64), st, iters)
    du = float(np.max(np.abs(g["u"] - st.u)))
    dis = label_disagreement(g["u"], st.u, kw.get("model", "two"))
    s.close()
    return du, dis, g, st


def progress(msg: str):
    """A progress line for long cases: printed, and appended to the file named
    by MF_TEST_PROGRESS when that variable is set (visible while the test
    still runs, whatever pytest captures)."""
    import os
    print(f"[progress] {msg}", flush=True)
    path = os.environ.get("MF_TEST_PROGRESS")
    if path:
        with open(path, "a") as f:
            f.write(msg + "\n")


def oracle_run(pr, caps64, iters, chunk=100, tag=""):
    """The FP64 oracle from the initial point for `iters` iterations, in
    chunks with a progress line after each."""
    st = oracle.init_state(pr, caps64)
    done = 0
    while done < iters:
        n = min(chunk, iters - done)
        oracle.step(pr, caps64, st, n)
        done += n
        progress(f"{tag} oracle {done}/{iters}")
    return st


def bf16_statement(pr, caps64, u_bf16, st_or, model):
    """Objective error of a BF16-storage run's u against the FP64 oracle at the
    same iteration count (both primal energies evaluated in FP64 on the
    unrounded capacities) and the thresholded-label disagreement."""
    e = oracle.energy(pr, caps64, st_or)
    st_b = oracle.state_from_arrays(pr, u_bf16, st_or.q, st_or.ps, st_or.p)
    if pr.method == "dr":
        st_b.zq, st_b.zs, st_b.zp = st_or.zq, st_or.zs, st_or.zp
    eb = oracle.energy(pr, caps64, st_b)
    obj = abs(eb["primal"] - e["primal"]) / abs(e["primal"])
    return obj, label_disagreement(u_bf16, st_or.u, model)
