"""Autotuner for the trial-pass launch shape and the batched schedule.

Candidates are the ara_tuning knobs: the single-layer pass variant (the
XCD-affine pass, or the rank-based pass with 16 or 32 lanes per trial group),
lanes per trial group in the batched pass (8/16/32/64), and the order of the
batched (layer, tile) work list.  Each candidate runs the
caller's layers a few times with ARA_PROFILE; the kernel time the library
measures with HIP events decides.  Results are cached per (device, shape
class) in a JSON file, so a shape is tuned once.
"""

from __future__ import annotations

import json
import math
import os
import threading
from typing import Dict, Iterable, List, Optional, Sequence

from . import ara

DEFAULT_CACHE = os.environ.get("ARA_AUTOTUNE_CACHE",
                               os.path.join(os.path.expanduser("~"), ".cache", "ara_autotune.json"))
_LOCK = threading.Lock()


def shape_class(tables: "ara.Tables", layers: Sequence["ara.LayerSpec"]) -> str:
    """Coarse key: catalogue parts, log2 of mean events per trial, log2 of
    trials per layer, layer count class, log2 of mean ELTs per layer."""
    n_layers = len(layers)
    trials = sum(l.trial_count for l in layers) / max(n_layers, 1)
    mean_events = tables.n_events / max(tables.n_trials, 1)
    mean_j = sum(l.n_elts for l in layers) / max(n_layers, 1)
    parts = (tables.catalogue_size + (1 << 18) - 1) >> 18
    b = lambda v: int(round(math.log2(max(v, 1.0))))  # noqa: E731
    layer_class = "one" if n_layers == 1 else ("few" if n_layers <= 8 else "many")
    return f"P{parts}-ev{b(mean_events)}-n{b(trials)}-{layer_class}-J{b(mean_j)}"


def candidates(n_layers: int) -> List[Dict[str, int]]:
    if n_layers > 1:
        out = [dict(part_lanes_per_trial=lpt) for lpt in (8, 16, 32, 64)]
        out += [dict(part_lanes_per_trial=lpt, schedule=1) for lpt in (16, 32)]
        return out
    out = [dict(pass_variant=0)]
    out += [dict(part_lanes_per_trial=lpt, pass_variant=1) for lpt in (16, 32)]
    return out


def load_cache(path: str = DEFAULT_CACHE) -> Dict[str, Dict[str, int]]:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache: Dict[str, Dict[str, int]], path: str = DEFAULT_CACHE) -> None:
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def device_name() -> str:
    import torch
    return torch.cuda.get_device_name(torch.cuda.current_device()).strip() or "gfx950"


def measure(tables: "ara.Tables", layers: Sequence["ara.LayerSpec"], knobs: Dict[str, int], out,
            flags: int = 0, repeats: int = 5, warmup: int = 1) -> float:
    """Average device time (ms) of the pass kernel(s) for one candidate."""
    import torch
    ara.set_tuning(tables, **knobs)
    batched = len(layers) > 1 and not flags & ara.ARA_PER_LAYER
    # the partitioned pass times its merge separately: count both
    kernels = [ara.KERNEL_BATCHED] if batched else [ara.KERNEL_TRIAL_PASS, ara.KERNEL_COMBINE]
    for _ in range(warmup):
        ara.run_layers(tables, layers, out=out, flags=flags)
    torch.cuda.synchronize()
    for k in kernels:
        ara.kernel_stats(tables, k, reset=True)
    for _ in range(repeats):
        ara.run_layers(tables, layers, out=out, flags=flags | ara.ARA_PROFILE)
    total = 0.0
    for k in kernels:
        n, ms = ara.kernel_stats(tables, k, reset=True)
        total += ms / max(n, 1) if n else 0.0
    return total


def tune(tables: "ara.Tables", layers: Sequence["ara.LayerSpec"], out, flags: int = 0, repeats: int = 5,
         cands: Optional[Iterable[Dict[str, int]]] = None) -> Dict[str, object]:
    """Time every candidate; set and return the best (with all timings)."""
    timings = []
    for knobs in (cands if cands is not None else candidates(len(layers))):
        timings.append((measure(tables, layers, knobs, out, flags, repeats), knobs))
    best_ms, best = min(timings, key=lambda x: x[0])
    ara.set_tuning(tables, **best)
    return {"best": best, "best_ms": best_ms, "timings": [(ms, k) for ms, k in timings]}


def tuned(tables: "ara.Tables", layers: Sequence["ara.LayerSpec"], out, flags: int = 0,
          path: str = DEFAULT_CACHE, repeats: int = 5) -> Dict[str, int]:
    """The cached choice for this (device, shape class), tuning it on a miss."""
    key = f"{device_name()}|{shape_class(tables, layers)}"
    with _LOCK:
        cache = load_cache(path)
        if key in cache:
            ara.set_tuning(tables, **cache[key])
            return cache[key]
    res = tune(tables, layers, out, flags, repeats)
    with _LOCK:
        cache = load_cache(path)
        cache[key] = res["best"]
        save_cache(cache, path)
    return res["best"]
