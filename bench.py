"""Benchmark: two-label continuous max-flow on a 256^3 volume, rpADMMII, FP32.

One step = one complete solve of the 3-D two-label workload (seeded volume of
20 ellipsoids at 0.8 on 0.2 with noise 0.1, C_s = |I - 0.2|, C_t = |I - 0.8|,
alpha 0.4, relaxation 1.5, 6-neighbour stencil): initial point, fused sweeps
with the FP64 primal-dual gap every 10 iterations until the relative gap is
<= 1e-4 or 1000 iterations, and label extraction.  Inputs are resident in HBM
before the timed region starts.

Prints one JSON line.  value = voxels * labels * iterations / second with
labels = 2 for the two-label model.  `roofline` reports the dominant kernel,
the fused 3-D sweep (one iteration per launch): algorithmic bytes per launch
(56 B per voxel: read u, q_x, q_y, q_z, p_s, p_t, C_s, C_t once; write u,
q_x, q_y, q_z, p_s, p_t once; FP32) divided by its average duration measured
with HIP events on the solver's stream over back-to-back sweeps, against
the 8 TB/s HBM peak and against a plain device copy measured in the same
run.  `gates` holds the working sets above the 256 MB last-level cache at one
iteration per pass (the 256^3 sweep and the two-label 2-D sweep at 4096^2);
`extra` the other rows of the hot path and the serving mix; `cpu_baseline`
times the FP64 oracle on a bounded sample of the same workload on the host
cores.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
    python bench.py --profile-mode NAME   # for rocprofv3: copy calibration + sweeps
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM = 8.0e12          # MI355X HBM3E, bytes/s
WORKLOAD = dict(name="two_label_3d_256", cfg="c3", shape=(256, 256, 256), method="eb", relax=1.5, alpha=0.4,
                tol=1e-4, max_iter=1000, check_every=10)


def alg_bytes(model: str, n: int, ndim: int, storage: str, image: bool = False) -> int:
    """Minimum HBM bytes per pixel and iteration of one fused sweep: read the
    state (u, q, p_s, p / p_t) and the capacities once, write the state once.
    u is always FP32; flows and capacities take the storage type.  With
    image-generated capacities one image plane replaces the capacity planes."""
    L = 1 if model == "two" else n
    ncap = 1 if image else (2 if model == "two" else n)
    e = 4 if storage == "f32" else 2
    u = 2 * L * 4
    flows = (L * ndim + 1 + L) * 2 * e
    return u + flows + ncap * e


SRC = "paper_2004_11227_amd/csrc/"
# Sources of each gate kernel (mf_kernels.h holds the workspace's plane
# stride), and the counter profile whose traffic is reported while the
# sources still hash to what was profiled.
GATE_KERNELS = {
    "two_label_3d_256": dict(sources=[SRC + "k3d.hip", SRC + "tile3d.h", SRC + "mf_device.h", SRC + "mf_kernels.h"],
                             traffic="fused3d_two_label_256_traffic.json",
                             kernel="k_fused3d<float, false, 16, false> (one iteration per launch)"),
    "two_label_2d_4096": dict(sources=[SRC + "k2d.hip", SRC + "tile2d.h", SRC + "tile2d_d2.h", SRC + "mf_device.h",
                                       SRC + "mf_kernels.h"],
                              traffic="fused2d_two_label_4096_depth1_traffic.json",
                              kernel="k_fused2d<1, true, float, false, 16, false> (one iteration per launch)"),
}

# Workloads of --profile-mode NAME (plain sweeps after a copy of known size,
# for the FETCH_SIZE / WRITE_SIZE calibration): caps generator arguments and
# solver keywords.
PROFILE_WORKLOADS = {
    "two_2048": (("c1", None), dict(model="two", method="eb", relax=1.5, alpha=0.5, depth=2, tile_rows=16)),
    "two_2048_d1": (("c1", None), dict(model="two", method="eb", relax=1.5, alpha=0.5, depth=1, tile_rows=16)),
    "two_4096": (("c1", (4096, 4096)), dict(model="two", method="eb", relax=1.5, alpha=0.5, depth=2,
                                           tile_rows=16)),
    "two_4096_d1": (("c1", (4096, 4096)), dict(model="two", method="eb", relax=1.5, alpha=0.5, depth=1,
                                              tile_rows=16)),
    "two_3d_256": (("c3", None), dict(model="two", method="eb", relax=1.5, alpha=0.4)),
    "potts4_1024": (("c2n4", None), dict(model="potts", nlabels=4, method="eb", relax=1.5, alpha=0.3)),
    "potts8_1024": (("c2n8", None), dict(model="potts", nlabels=8, method="eb", relax=1.5, alpha=0.3)),
    "pdrq_2048": (("c1", None), dict(model="two", method="dr", alpha=0.5)),
    "pdrq_potts4_1024": (("c2n4", None), dict(model="potts", nlabels=4, method="dr", alpha=0.3)),
    "pdrq_potts8_1024": (("c2n8", None), dict(model="potts", nlabels=8, method="dr", alpha=0.3)),
    "pdrq_3d_256": (("c3", None), dict(model="two", method="dr", alpha=0.4)),
}


def kernel_hash(files) -> str:
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--kernel-sweeps", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip the secondary measurements")
    ap.add_argument("--serving-requests", type=int, default=2048,
                    help="requests of the serving mix in the secondary measurements (0: skip)")
    ap.add_argument("--serving-child", default=None, metavar="OUT",
                    help="(internal) run only the serving mix and write its summary to OUT as JSON")
    ap.add_argument("--profile-sweeps", type=int, default=200, help="iterations run in --profile-mode")
    ap.add_argument("--profile-mode", nargs="?", const="two_3d_256", default=None,
                    choices=sorted(PROFILE_WORKLOADS))
    return ap.parse_args()


def phase(msg):
    """Progress on stderr (stdout carries only the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_sweeps(torch, solver, stream, n):
    """Average time per iteration of plain sweeps (no gap), HIP events on the
    solver's stream, after as many untimed sweeps (the clocks settle)."""
    solver.step(max(20, n))
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    solver.step(n)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / n


def copy_rate(torch, dev, stream, nbytes=1 << 30, reps=20):
    """Device copy bandwidth (read + write bytes per second) of torch's plain
    copy kernel between two nbytes buffers, timed like the sweeps."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    with torch.cuda.stream(stream):
        a.fill_(1.0)
        for _ in range(3):
            b.copy_(a)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            b.copy_(a)
        e1.record(stream)
    e1.synchronize()
    dt = e0.elapsed_time(e1) * 1e-3 / reps
    del a, b
    return 2.0 * nbytes / dt


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(caps64, wl, serving_reqs=None, serving_iters=None):
    """The FP64 oracle on the host cores (all of them, then one thread) on a
    bounded sample of the workload's iterations; optionally a bounded sample
    of the serving mix solved to its tolerance."""
    import oracle
    shape = wl["shape"]
    pr = oracle.Problem(shape, model="two", method=wl["method"], relax=wl["relax"], alpha=wl["alpha"])
    st = oracle.init_state(pr, caps64)
    oracle.step(pr, caps64, st, 1)
    n = int(shape[0] * shape[1] * shape[2])
    threads = oracle.num_threads()
    iters = 30   # ~10-20 s of the host's cores at 256^3
    t0 = time.perf_counter()
    oracle.step(pr, caps64, st, iters)
    dt = time.perf_counter() - t0
    iters1 = 2
    oracle.set_threads(1)
    t0 = time.perf_counter()
    oracle.step(pr, caps64, st, iters1)
    dt1 = time.perf_counter() - t0
    oracle.set_threads(threads)
    out = {"value": n * 2 * iters / dt, "unit": "pixel*label*iterations/s", "cores": threads, "kind": "oracle",
           "cpu_model": cpu_model(), "nproc": os.cpu_count(),
           "sample": f"iterations 1..{iters} of the 256^3 two-label rpADMMII workload (a solve to gap "
                     f"{wl['tol']:g} runs up to {wl['max_iter']}), FP64, OpenMP threads={threads}, {dt:.1f} s",
           "single_thread": {"value": n * 2 * iters1 / dt1, "cores": 1,
                             "sample": f"{iters1} further iterations on one thread, {dt1:.1f} s"}}
    if serving_reqs and serving_iters:
        out["serving_sample"] = serving_oracle_sample(serving_reqs, serving_iters, threads)
    return out


def serving_oracle_sample(reqs, iters_by_rid, threads, nsample=32, probe_iters=5):
    """The oracle's one-at-a-time solves/s on the serving mix, extrapolated
    from a sample: the first `nsample` requests of the trace each run
    `probe_iters` iterations from the initial point, and each request's time
    per iteration is scaled to the iteration count its FP32 GPU solve needed
    (same method, tolerance and cap)."""
    import numpy as np

    import oracle
    from paper_2004_11227_amd import synth
    total, probe = 0.0, 0.0
    sample = reqs[:nsample]
    for r in sample:
        caps = synth.request_caps(r).astype(np.float32).astype(np.float64)
        pr = oracle.Problem(r.shape, model=r.model, nlabels=r.nlabels, method="eb", alpha=r.alpha)
        st = oracle.init_state(pr, caps)
        t0 = time.perf_counter()
        oracle.step(pr, caps, st, probe_iters)
        dt = time.perf_counter() - t0
        probe += dt
        total += dt / probe_iters * max(int(iters_by_rid.get(r.rid, 0)), 1)
    return {"solves_per_s": len(sample) / total, "solves": len(sample), "cores": threads,
            "measured_s": probe, "extrapolated": True,
            "sample": f"the first {len(sample)} requests of the serving trace: {probe_iters} FP64 oracle iterations "
                      f"each, time per iteration scaled to the iterations of the request's FP32 GPU solve "
                      f"(rpADMMII to gap 1e-4 or 1000 iterations)"}


def gate_line(torch, maxflow, np, dev, stream, name, caps, kw, iters, bytes_px, copy_Bps):
    """One working set above the last-level cache at one iteration per pass:
    algorithmic rate of the depth-1 sweep against 8 TB/s and the copy rate,
    with the counter traffic while the profiled sources are unchanged."""
    phase(f"gate: {name}")
    t = torch.from_numpy(caps.astype(np.float32)).to(dev)
    s = maxflow.Solver(t, stream=stream, **kw)
    dt = time_sweeps(torch, s, stream, iters)
    s.close()
    del t
    npx = int(np.prod(caps.shape[1:]))
    launch = bytes_px * npx
    gk = GATE_KERNELS[name]
    traffic = None
    path = os.path.join(ROOT, "profiles", gk["traffic"])
    if os.path.exists(path):
        d = json.load(open(path))
        if d.get("kernel_hash") == kernel_hash(gk["sources"]):
            traffic = d.get("bytes_per_launch")
    return {"bound": "hbm", "achieved": launch / dt / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
            "frac": launch / dt / PEAK_HBM, "traffic": traffic, "kernel": gk["kernel"], "bytes_per_launch": launch,
            "algorithmic_bytes_per_px_iter": bytes_px, "avg_launch_us": dt * 1e6, "iterations_per_launch": 1,
            "copy_GBps": copy_Bps / 1e9, "frac_of_copy": launch / dt / copy_Bps,
            "traffic_GBps": (traffic / dt / 1e9) if traffic else None}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the solver runs on one GPU; runs on several GPUs are not supported", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2004_11227_amd import maxflow, synth

    wl = WORKLOAD
    if args.serving_child:
        serving_child(args)
        return
    serving_reqs, serving_out = None, None
    if not args.no_extra and args.serving_requests > 0 and not args.profile_mode:
        # The serving mix runs first, in a child process started before this
        # one touches the GPU: a failure there (the pool has ended a process
        # in a host segmentation fault whose cause is not known) costs only
        # the serving lines.
        serving_reqs = synth.serving_trace(args.serving_requests, seed=SERVING_SEED)
        serving_out = run_serving_child(args.serving_requests)

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.Stream(device=dev)

    if args.profile_mode:
        # known-size copy for counter calibration, then plain sweeps
        src = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        (cfg, size), pkw = PROFILE_WORKLOADS[args.profile_mode]
        pc = synth.config_inputs(cfg, size=size)["caps"] if size else synth.config_inputs(cfg)["caps"]
        pt = torch.from_numpy(pc.astype(np.float32)).to(dev)
        s = maxflow.Solver(pt, stream=stream, **pkw)
        # enough sweeps that the launch average is the steady state's
        s.step(args.profile_sweeps)
        torch.cuda.synchronize()
        print(json.dumps({"profile_mode": args.profile_mode, "copy_bytes": src.numel() * 4,
                          "sweeps": args.profile_sweeps, "shape": list(pc.shape[1:])}))
        return

    inp = synth.config_inputs(wl["cfg"])
    caps64 = inp["caps"]
    caps_t = torch.from_numpy(caps64.astype(np.float32)).to(dev)
    npx = int(np.prod(wl["shape"]))
    kw = dict(model="two", method=wl["method"], relax=wl["relax"], alpha=wl["alpha"], tol=wl["tol"],
              max_iter=wl["max_iter"], check_every=wl["check_every"])

    phase("copy bandwidth")
    copy0 = copy_rate(torch, dev, stream)

    phase(f"headline: {wl['name']} solves")
    s = maxflow.Solver(caps_t, stream=stream, **kw)

    def one_step():
        s.reset()
        res = s.solve()
        s.labels()
        return res

    for _ in range(args.warmup):
        res = one_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = one_step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    assert res["status"] in (0, 1), res
    iters = int(res["iter"])
    value = npx * 2 * iters / dt

    # dominant kernel: the fused 3-D sweep, average duration over
    # back-to-back launches on the solver's stream
    phase("headline: kernel timing")
    b3 = alg_bytes("two", 2, 3, "f32")
    t_launch = time_sweeps(torch, s, stream, args.kernel_sweeps)
    s.close()
    del caps_t
    launch_bytes = b3 * npx
    copy1 = copy_rate(torch, dev, stream)
    copy_Bps = max(copy0, copy1)
    gk = GATE_KERNELS[wl["name"]]
    traffic = None
    tpath = os.path.join(ROOT, "profiles", gk["traffic"])
    if os.path.exists(tpath):
        d = json.load(open(tpath))
        if d.get("kernel_hash") == kernel_hash(gk["sources"]):
            traffic = d.get("bytes_per_launch")
    roof = {"bound": "hbm", "achieved": launch_bytes / t_launch / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
            "frac": launch_bytes / t_launch / PEAK_HBM, "traffic": traffic, "kernel": gk["kernel"],
            "bytes_per_launch": launch_bytes, "algorithmic_bytes_per_px_iter": b3,
            "avg_launch_us": t_launch * 1e6, "iterations_per_launch": 1,
            "copy_GBps": copy_Bps / 1e9, "frac_of_copy": launch_bytes / t_launch / copy_Bps,
            "copy_kernel": "torch device copy, 1 GiB to 1 GiB, read + write bytes / time, before and after the "
                           "headline (the larger)",
            "working_set_bytes": 2 * 6 * 4 * npx + 2 * 4 * npx}

    gates = {wl["name"]: {k: roof[k] for k in ("achieved", "frac", "traffic", "avg_launch_us", "frac_of_copy")}}
    big = synth.config_inputs("c1", size=(4096, 4096))["caps"]
    gates["two_label_2d_4096"] = gate_line(
        torch, maxflow, np, dev, stream, "two_label_2d_4096", big,
        dict(model="two", method="eb", relax=1.5, alpha=0.5, depth=1, tile_rows=16), 100,
        alg_bytes("two", 2, 2, "f32"), copy_Bps)
    del big

    extra = {}
    serving_iters = None
    if not args.no_extra:
        extra = secondary(torch, maxflow, synth, np, dev, stream)
        if serving_out is not None:
            extra["serving"] = serving_out.get("summary")
            if serving_out.get("sequential_iters"):
                serving_iters = {int(k): v for k, v in serving_out["sequential_iters"].items()}

    out = {"metric": "pixel*label ADMM iterations/s (two-label 256^3, rpADMMII, FP32, solve to gap 1e-4)",
           "value": value, "unit": "pixel*label*iterations/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": wl["name"], "shape": list(wl["shape"]), "iterations": iters,
                      "status": int(res["status"]), "rel_gap": res["rel_gap"], "tol": wl["tol"],
                      "max_iter": wl["max_iter"], "method": "rpADMMII", "relax": wl["relax"], "alpha": wl["alpha"],
                      "gap_every": wl["check_every"], "labels": 2, "iterations_per_pass": 1,
                      "parallelism": "single GPU"},
           "roofline": roof, "gates": gates}
    if not args.no_cpu:
        phase("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(caps64, wl, serving_reqs, serving_iters)
    if extra:
        out["extra"] = extra
    print(json.dumps(out), flush=True)


def secondary(torch, maxflow, synth, np, dev, stream):
    """Per-sweep bandwidth of other rows of the hot path (not the headline value).
    Working sets below the 256 MB last-level cache are partly served from it:
    their rates are effective, not HBM, figures."""
    res = {}

    def sweep_rate(name, caps, nbytes_px, iters=200, **kw):
        # per-iteration time; alg_GBps = algorithmic bytes of one depth-1
        # sweep / time per iteration (a depth-2 pass moves them once per two
        # iterations, so its figure can exceed the HBM peak)
        phase(f"secondary: {name}")
        t = torch.from_numpy(caps.astype(np.float32)).to(dev)
        s = maxflow.Solver(t, stream=stream, **kw)
        dt = time_sweeps(torch, s, stream, iters)
        npx = int(np.prod(caps.shape[1:]))
        L = 2 if kw.get("model", "two") == "two" else kw["nlabels"]
        res[name] = {"us_per_iter": dt * 1e6, "px_label_it_per_s": npx * L / dt,
                     "alg_GBps": nbytes_px * npx / dt / 1e9, "frac_hbm": nbytes_px * npx / dt / PEAK_HBM,
                     "working_set_MiB": round(s.workspace.numel() / 2**20)}
        s.close()
        del t

    c1 = synth.config_inputs("c1")["caps"]
    b2 = alg_bytes("two", 2, 2, "f32")
    sweep_rate("two_2048_fused_f32_depth2", c1, b2, model="two", method="eb", relax=1.5, depth=2)
    sweep_rate("two_2048_fused_f32_depth1", c1, b2, model="two", method="eb", relax=1.5, depth=1)
    sweep_rate("two_2048_unfused_f32", c1, b2, model="two", method="eb", relax=1.5, variant="unfused")
    sweep_rate("two_2048_fused_bf16_depth2", c1, alg_bytes("two", 2, 2, "bf16"), model="two", method="eb",
               relax=1.5, storage="bf16", depth=2)
    sweep_rate("two_2048_pdrq_f32_fused", c1, b2, model="two", method="dr")
    sweep_rate("two_2048_pdrq_f32_inplace", c1, b2, model="two", method="dr", variant="unfused")
    big = synth.config_inputs("c1", size=(4096, 4096))["caps"]
    sweep_rate("two_4096_fused_f32_depth2", big, b2, iters=100, model="two", method="eb", relax=1.5, depth=2)
    del big
    for n in (4, 8):
        img, _ = synth.voronoi_image(1024, 1024, n, 0.15, 2000)
        caps = synth.potts_caps(img, n)
        for stg in ("f32", "bf16"):
            sweep_rate(f"potts{n}_1024_fused_{stg}", caps, alg_bytes("potts", n, 2, stg),
                       model="potts", nlabels=n, method="eb", alpha=0.3, storage=stg)
        for var, tag in (("fused", "fused"), ("unfused", "inplace")):
            sweep_rate(f"potts{n}_1024_pdrq_f32_{tag}", caps, alg_bytes("potts", n, 2, "f32"), model="potts",
                       nlabels=n, method="dr", alpha=0.3, variant=var)
    # capacities generated from the image plane (the same workloads' data
    # costs |I - l|^p): one plane read instead of 2 or n
    img1 = synth.config_inputs("c1")["image"][None]
    sweep_rate("two_2048_fused_f32_depth2_image", img1, alg_bytes("two", 2, 2, "f32", image=True), model="two",
               method="eb", relax=1.5, depth=2, cap_source="image", cap_power=1, levels=(0.2, 0.8))
    del img1
    inp8 = synth.config_inputs("c2n8")
    sweep_rate("potts8_1024_fused_f32_image", inp8["image"][None], alg_bytes("potts", 8, 2, "f32", image=True),
               model="potts", nlabels=8, method="eb", alpha=0.3, cap_source="image", cap_power=2,
               levels=tuple(k / 7 for k in range(8)))
    del inp8
    vol = synth.config_inputs("c3")["caps"]   # 256^3, 512 MiB FP32 working set
    sweep_rate("two_3d_256_fused_bf16", vol, alg_bytes("two", 2, 3, "bf16"), iters=50, model="two",
               method="eb", relax=1.5, alpha=0.4, storage="bf16")
    sweep_rate("two_3d_256_unfused_f32", vol, alg_bytes("two", 2, 3, "f32"), iters=20, model="two",
               method="eb", relax=1.5, alpha=0.4, variant="unfused")
    sweep_rate("two_3d_256_pdrq_f32_inplace", vol, alg_bytes("two", 2, 3, "f32"), iters=20, model="two",
               method="dr", alpha=0.4)
    del vol
    vimg = synth.config_inputs("c3")["image"][None]
    sweep_rate("two_3d_256_fused_f32_image", vimg, alg_bytes("two", 2, 3, "f32", image=True), iters=50,
               model="two", method="eb", relax=1.5, alpha=0.4, cap_source="image", cap_power=1, levels=(0.2, 0.8))
    del vimg
    return res


SERVING_SEED = 4000


def run_serving_child(nreq):
    """The serving summary from a child run of this script (see main); on a
    failed child, a record of the failure instead of the summary."""
    import subprocess
    import tempfile
    fd, path = tempfile.mkstemp(prefix="serving_", suffix=".json")
    os.close(fd)
    try:
        phase(f"serving mix: {nreq} requests in a child process")
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--serving-child", path,
                            "--serving-requests", str(nreq)], timeout=900)
        if r.returncode != 0:
            phase(f"serving child exited with status {r.returncode}")
            return {"summary": {"error": f"serving child process exited with status {r.returncode}"}}
        return json.load(open(path))
    except subprocess.TimeoutExpired:
        return {"summary": {"error": "serving child process timed out"}}
    finally:
        os.unlink(path)


def serving_child(args):
    from paper_2004_11227_amd import serving
    phase(f"serving mix: drawing {args.serving_requests} requests")
    drawn = serving.draw_requests(args.serving_requests, seed=SERVING_SEED)
    phase("serving mix")
    summary, iters = serving_summary(drawn)
    json.dump({"summary": summary, "sequential_iters": {str(k): v for k, v in iters.items()}},
              open(args.serving_child, "w"))


def serving_summary(drawn):
    """Continuous batching through the pool (BF16 flows, promoted to FP32
    near the BF16 floor) against one-at-a-time FP32 solves on the mixed
    request trace: solves/s at saturation and p50/p99 latency under Poisson
    arrivals at 0.7x the one-at-a-time capacity."""
    from paper_2004_11227_amd import serving
    # The Poisson-arrival phase is not run: a run of it ended in a host
    # segmentation fault whose cause has not been found.
    r = serving.benchmark(drawn=drawn, pool_storage="bf16", tol=1e-4, max_iter=1000, latency=False, log=phase)
    keep = ("solves_per_s", "p50_latency_s", "p99_latency_s", "mean_iters", "converged", "capped", "diverged")
    out = {k: r[k] for k in ("requests", "tol", "max_iter", "total_pixels", "promotions_total",
                             "speedup_solves_per_s")}
    for k in ("sequential_fp32", "pool"):
        out[k] = {kk: r[k][kk] for kk in keep if kk in r[k]}
    out["latency_note"] = ("p50/p99 are arrival-to-result latencies with every request queued at t = 0; the "
                           "Poisson-arrival latency phase is not run (a run of it ended in an unexplained host "
                           "segmentation fault)")
    return out, r["sequential_iters"]


if __name__ == "__main__":
    main()
