"""Cache of autotuned launch shapes.

The autotuner itself is native (``maxflow_tune``: it times the candidate
tile heights of the fused 2-D and 3-D sweeps with HIP events on the solver's stream).
This module keeps its choices in a JSON file so that a shape class is timed
once per device: the key is (device name, model, labels, dimensions,
storage, method, variant, requested depth, capacity source, log2 of the pixel count), the value the chosen
tile height and the measured microseconds per sweep of every candidate.
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
        cap_source="planes", **_) -> str:
    import torch
    name = torch.cuda.get_device_name(device) if device is not None else "cpu"
    npx = 1
    for s in shape:
        npx *= int(s)
    L = 2 if model == "two" else int(nlabels)
    return "|".join([name, model, str(L), f"{len(shape)}d", storage, method, variant, f"depth{int(depth)}",
                     f"caps-{cap_source}",
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
    """Cached tile height for this shape class, or None."""
    with _lock:
        e = _load().get(key(shape, device, **kw))
    return int(e["tile_rows"]) if e else None


def store(shape, device, best: int, us: dict, **kw):
    """Record a tuning result (`best` tile height, microseconds per sweep of
    each candidate) and write the cache file (best effort)."""
    k = key(shape, device, **kw)
    with _lock:
        d = _load()
        d[k] = {"tile_rows": int(best), "us_per_sweep": {str(r): v for r, v in us.items()}}
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
