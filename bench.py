"""Benchmark: two-label continuous max-flow, 2048x2048, rpADMMII, FP32.

One step = one complete solve of the two-label 2048x2048 workload (seeded
ellipse image, 40 ellipses, noise 0.15, alpha 0.5, relaxation 1.5): initial
point, 500 iterations of the fused sweep (two iterations per pass, iterates
bit-identical to one per pass) with the FP64 primal-dual gap every 10
iterations (tolerance 0, so all 500 iterations run) and label extraction.
Inputs are resident in HBM before the timed region starts.

Prints one JSON line.  value = pixels * labels * iterations / second with
labels = 2 for the two-label model.  `roofline` reports the dominant kernel
(the two-iteration fused pass without the gap reduction): algorithmic bytes
per launch (48 B per pixel: read u, q_x, q_y, p_s, p_t, C_s, C_t once; write
u, q_x, q_y, p_s, p_t once; FP32; the intermediate iterate never leaves LDS)
divided by its average duration measured with HIP events on the solver's
stream over a run of back-to-back passes.  `cpu_baseline` times
the FP64 oracle on a bounded sample of the same workload on the host cores.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
    python bench.py --profile-mode    # for rocprofv3: copy calibration + sweeps
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
WORKLOAD = dict(name="two_label_2d_2048", shape=(2048, 2048), iters=500, method="eb", relax=1.5,
                alpha=0.5, check_every=10, depth=2, tile_rows=16)


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


BYTES_PER_PX = {"f32": alg_bytes("two", 2, 2, "f32"), "bf16": alg_bytes("two", 2, 2, "bf16")}
SRC = "paper_2004_11227_amd/csrc/"
KERNEL_SOURCES = [SRC + "k2d.hip", SRC + "tile2d.h", SRC + "tile2d_d2.h", SRC + "mf_device.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fused2d_two_label_2048_traffic.json")

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
    "pdrq_3d_256": (("c3", None), dict(model="two", method="dr", alpha=0.4)),
}


def kernel_hash(files=KERNEL_SOURCES) -> str:
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--kernel-sweeps", type=int, default=400)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip the secondary measurements")
    ap.add_argument("--serving-requests", type=int, default=128,
                    help="requests of the serving mix in the secondary measurements (0: skip)")
    ap.add_argument("--profile-sweeps", type=int, default=200, help="iterations run in --profile-mode")
    ap.add_argument("--profile-mode", nargs="?", const="two_2048", default=None,
                    choices=sorted(PROFILE_WORKLOADS))
    return ap.parse_args()


def phase(msg):
    """Progress on stderr (stdout carries only the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_solver(torch, maxflow, caps_t, stream, **kw):
    return maxflow.Solver(caps_t, stream=stream, **kw)


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


def cpu_baseline(caps64, wl):
    """The FP64 oracle on the host cores (all of them, then one thread) on a
    bounded sample of the workload's iterations."""
    import oracle
    shape = wl["shape"]
    pr = oracle.Problem(shape, model="two", method=wl["method"], relax=wl["relax"], alpha=wl["alpha"])
    st = oracle.init_state(pr, caps64)
    oracle.step(pr, caps64, st, 1)
    n = shape[0] * shape[1]
    threads = oracle.num_threads()
    iters = 200   # ~10 s of the host's cores at the measured ~1.5e8 pixel*label*it/s
    t0 = time.perf_counter()
    oracle.step(pr, caps64, st, iters)
    dt = time.perf_counter() - t0
    iters1 = 10
    oracle.set_threads(1)
    t0 = time.perf_counter()
    oracle.step(pr, caps64, st, iters1)
    dt1 = time.perf_counter() - t0
    oracle.set_threads(threads)
    return {"value": n * 2 * iters / dt, "unit": "pixel*label*iterations/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{iters} of the {wl['iters']} iterations of the {shape[0]}x{shape[1]} two-label "
                      f"rpADMMII workload, FP64, OpenMP threads={threads}, {dt:.1f} s",
            "single_thread": {"value": n * 2 * iters1 / dt1, "cores": 1,
                              "sample": f"{iters1} further iterations on one thread, {dt1:.1f} s"}}


def traffic_for(launch_bytes):
    if not os.path.exists(TRAFFIC_FILE):
        return None
    d = json.load(open(TRAFFIC_FILE))
    if d.get("kernel_hash") != kernel_hash():
        return None
    return d.get("bytes_per_launch")


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the solver runs on one GPU; runs on several GPUs are not supported", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2004_11227_amd import maxflow, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    wl = WORKLOAD
    inp = synth.config_inputs("c1")
    caps64 = inp["caps"]
    caps_t = torch.from_numpy(caps64.astype(np.float32)).to(dev)
    stream = torch.cuda.Stream(device=dev)
    H, W = wl["shape"]
    npx = H * W
    kw = dict(model="two", method=wl["method"], relax=wl["relax"], alpha=wl["alpha"], tol=0.0,
              max_iter=wl["iters"], check_every=wl["check_every"], depth=wl["depth"], tile_rows=wl["tile_rows"])

    if args.profile_mode:
        # known-size copy for counter calibration, then plain sweeps
        src = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        (cfg, size), pkw = PROFILE_WORKLOADS[args.profile_mode]
        pc = synth.config_inputs(cfg, size=size)["caps"] if size else synth.config_inputs(cfg)["caps"]
        pt = torch.from_numpy(pc.astype(np.float32)).to(dev)
        s = make_solver(torch, maxflow, pt, stream, **pkw)
        # enough sweeps that the launch average is the steady state's
        s.step(args.profile_sweeps)
        torch.cuda.synchronize()
        print(json.dumps({"profile_mode": args.profile_mode, "copy_bytes": src.numel() * 4,
                          "sweeps": args.profile_sweeps, "shape": list(pc.shape[1:])}))
        return

    phase(f"headline: {wl['name']} solves")
    s = make_solver(torch, maxflow, caps_t, stream, **kw)

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
    assert res["iter"] == wl["iters"], res
    value = npx * 2 * wl["iters"] / dt

    # dominant kernel: the two-iteration pass, average duration over
    # back-to-back launches (step(n) issues n / 2 passes)
    phase("headline: kernel timing")
    t_iter = time_sweeps(torch, s, stream, args.kernel_sweeps)
    t_launch = t_iter * wl["depth"]
    launch_bytes = BYTES_PER_PX["f32"] * npx
    achieved = launch_bytes / t_launch
    roof = {"bound": "hbm", "achieved": achieved / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
            "frac": achieved / PEAK_HBM, "traffic": traffic_for(launch_bytes),
            "kernel": f"k_fused2d_d2<float, false, {wl['tile_rows']}, false> (two iterations per launch)",
            "bytes_per_launch": launch_bytes, "avg_launch_us": t_launch * 1e6,
            "iterations_per_launch": wl["depth"]}
    s.close()

    extra = {}
    if not args.no_extra:
        extra = secondary(torch, maxflow, synth, np, dev, stream)
        if args.serving_requests > 0:
            phase("serving mix")
            extra["serving"] = serving_summary(args.serving_requests)

    out = {"metric": "pixel*label ADMM iterations/s (two-label 2048^2, rpADMMII, FP32)",
           "value": value, "unit": "pixel*label*iterations/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": wl["name"], "shape": list(wl["shape"]), "iterations": wl["iters"],
                      "method": "rpADMMII", "relax": wl["relax"], "alpha": wl["alpha"],
                      "gap_every": wl["check_every"], "labels": 2, "iterations_per_pass": wl["depth"],
                      "tile_rows": wl["tile_rows"], "parallelism": "single GPU"},
           "roofline": roof}
    if not args.no_cpu:
        phase("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(caps64, wl)
    if extra:
        out["extra"] = extra
    print(json.dumps(out), flush=True)


def secondary(torch, maxflow, synth, np, dev, stream):
    """Per-sweep bandwidth of other rows of the hot path (not the headline value)."""
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
                     "alg_GBps": nbytes_px * npx / dt / 1e9, "frac_hbm": nbytes_px * npx / dt / PEAK_HBM}
        s.close()
        del t

    c1 = synth.config_inputs("c1")["caps"]
    b2 = alg_bytes("two", 2, 2, "f32")
    sweep_rate("two_2048_fused_f32_depth1", c1, b2, model="two", method="eb", relax=1.5, depth=1)
    sweep_rate("two_2048_unfused_f32", c1, b2, model="two", method="eb", relax=1.5, variant="unfused")
    sweep_rate("two_2048_fused_bf16_depth2", c1, alg_bytes("two", 2, 2, "bf16"), model="two", method="eb",
               relax=1.5, storage="bf16", depth=2)
    sweep_rate("two_2048_pdrq_f32_fused", c1, b2, model="two", method="dr")
    sweep_rate("two_2048_pdrq_f32_inplace", c1, b2, model="two", method="dr", variant="unfused")
    big = synth.config_inputs("c1", size=(4096, 4096))["caps"]
    sweep_rate("two_4096_fused_f32_depth1", big, b2, iters=100, model="two", method="eb", relax=1.5, depth=1)
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
    sweep_rate("two_2048_fused_f32_depth1_image", img1, alg_bytes("two", 2, 2, "f32", image=True), model="two",
               method="eb", relax=1.5, depth=1, cap_source="image", cap_power=1, levels=(0.2, 0.8))
    del img1
    inp8 = synth.config_inputs("c2n8")
    sweep_rate("potts8_1024_fused_f32_image", inp8["image"][None], alg_bytes("potts", 8, 2, "f32", image=True),
               model="potts", nlabels=8, method="eb", alpha=0.3, cap_source="image", cap_power=2,
               levels=tuple(k / 7 for k in range(8)))
    del inp8
    vol = synth.config_inputs("c3")["caps"]   # 256^3, 512 MiB FP32 working set
    for stg in ("f32", "bf16"):
        sweep_rate(f"two_3d_256_fused_{stg}", vol, alg_bytes("two", 2, 3, stg), iters=50, model="two",
                   method="eb", relax=1.5, alpha=0.4, storage=stg)
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


def serving_summary(nreq):
    """Continuous batching through the pool (BF16 flows, promoted to FP32
    near the BF16 floor) against one-at-a-time FP32 solves on the mixed
    request trace: solves/s at saturation and p50/p99 latency under Poisson
    arrivals at 0.7x the one-at-a-time capacity."""
    from paper_2004_11227_amd import serving
    r = serving.benchmark(nreq=nreq, pool_storage="bf16", tol=1e-4, max_iter=1000, log=phase)
    keep = ("solves_per_s", "p50_latency_s", "p99_latency_s", "mean_iters", "converged", "capped")
    out = {k: r[k] for k in ("requests", "tol", "max_iter", "total_pixels", "promotions_total",
                             "speedup_solves_per_s", "latency_rate_per_s")}
    for k in ("sequential_fp32", "pool"):
        out[k] = {kk: r[k][kk] for kk in keep if kk in r[k]}
    for k in ("sequential_fp32_latency", "pool_latency"):
        out[k] = {kk: r[k][kk] for kk in ("p50_latency_s", "p99_latency_s", "mean_latency_s", "solves_per_s")}
    return out


if __name__ == "__main__":
    main()
