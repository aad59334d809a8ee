"""Cache of autotuned launch shapes.

The autotuner itself is native (``maxflow_tune``: it times the candidate
launch shapes, tile height x fusion depth x 3-D slab depth, with HIP events on
the solver's stream).  This module keeps its choices in a JSON file so that a
shape class is timed once per device: the key is (device name, model,
labels, dimensions, storage, method, variant, requested depth and slab depth
(0: tuned), capacity source, log2 of the pixel count), the value the chosen
shape and the measured microseconds per iteration of every candidate.
``Solver(..., tile_rows="auto")`` looks the class up and tunes on a miss.

The file is ``$MF_TUNING_CACHE`` if set, else
``~/.cache/paper_2004_11227_amd/tuning.json``.  Entries never change
results: every tile height gives the same iterates bit for bit.
"""
from __future__ import annotations

import json
import math
import os
import threading

_lock = threading.Lock()
_mem: dict | None = None


def cache_path() -> str:
    p = os.environ.get("MF_TUNING_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_2004_11227_amd", "tuning.json")


def key(shape, device, model="two", nlabels=2, storage="f32", method="eb", variant="fused", depth=0,
        cap_source="planes", slab_depth=0, **_) -> str:
    import torch
    name = torch.cuda.get_device_name(device) if device is not None else "cpu"
    npx = 1
    for s in shape:
        npx *= int(s)
    L = 2 if model == "two" else int(nlabels)
    return "|".join([name, model, str(L), f"{len(shape)}d", storage, method, variant, f"depth{int(depth)}",
                     f"slab{int(slab_depth)}", f"caps-{cap_source}",
                     f"px2^{int(round(math.log2(max(npx, 1))))}"])


def _load() -> dict:
    global _mem
    if _mem is None:
        try:
            with open(cache_path()) as f:
                _mem = json.load(f)
        except (OSError, ValueError):
            _mem = {}
    return _mem


def lookup(shape, device, **kw):
    """Cached launch shape dict(tile_rows, depth, slab_depth) for this shape
    class, or None."""
    with _lock:
        e = _load().get(key(shape, device, **kw))
    if not e or "choice" not in e:
        return None
    return {k: int(v) for k, v in e["choice"].items()}


def store(shape, device, best: dict, cands: list, **kw):
    """Record a tuning result (the chosen dict(tile_rows, depth, slab_depth)
    and every candidate with its microseconds per iteration) and write the
    cache file (best effort)."""
    k = key(shape, device, **kw)
    with _lock:
        d = _load()
        d[k] = {"choice": {kk: int(v) for kk, v in best.items()}, "candidates": list(cands)}
        path = cache_path()
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            tmp = path + f".{os.getpid()}.tmp"
            with open(tmp, "w") as f:
                json.dump(d, f, indent=1, sort_keys=True)
            os.replace(tmp, path)
        except OSError:
            pass


def clear():
    """Forget the in-memory cache (the file stays)."""
    global _mem
    with _lock:
        _mem = None
