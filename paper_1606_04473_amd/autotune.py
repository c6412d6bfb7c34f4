"""Autotuner for the pass over the YET, its launch shape and the batched schedule.

Candidates are the ara_tuning knobs: the pass variant (0: the 16-bit stream
copy; 2: the XCD-affine pass over the 32-bit partitioned copy; 1: the
rank-based pass, which for several layers is one persistent launch over a
(layer, tile) work list), lanes per trial group of the rank-based passes
(8/16/32/64) and the order of the batched work list.  Each candidate runs the
caller's layers a few times; the device time of the whole call, from HIP
events on its stream, decides, and the per-kernel times the library records
with ARA_PROFILE are kept beside it.  Results are cached per (device, shape
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
    parts = (tables.catalogue_size + (1 << 16) - 1) >> 16
    b = lambda v: int(round(math.log2(max(v, 1.0))))  # noqa: E731
    layer_class = "one" if n_layers == 1 else ("few" if n_layers <= 8 else "many")
    return f"P{parts}-ev{b(mean_events)}-n{b(trials)}-{layer_class}-J{b(mean_j)}"


def candidates(n_layers: int) -> List[Dict[str, int]]:
    out = [dict(pass_variant=0), dict(pass_variant=2)]
    if n_layers > 1:
        # one persistent launch for all the layers
        out += [dict(pass_variant=1, part_lanes_per_trial=lpt) for lpt in (8, 16, 32, 64)]
        out += [dict(pass_variant=1, part_lanes_per_trial=lpt, schedule=1) for lpt in (16, 32)]
        return out
    out += [dict(pass_variant=1, part_lanes_per_trial=lpt) for lpt in (16, 32)]
    return out


KERNEL_CLASSES = {"fold": ara.KERNEL_FOLD, "trial_pass": ara.KERNEL_TRIAL_PASS, "combine": ara.KERNEL_COMBINE,
                  "batched": ara.KERNEL_BATCHED}


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


def measure_detail(tables: "ara.Tables", layers: Sequence["ara.LayerSpec"], knobs: Dict[str, int], out,
                   flags: int = 0, repeats: int = 5, warmup: int = 1, stream=None) -> Dict[str, float]:
    """One candidate: the average device time (ms) of a whole ara_run_layers
    call (HIP events around `repeats` calls on the stream), then, from
    `repeats` more calls with ARA_PROFILE, the average time per call of each
    kernel class that ran.  Raises if no kernel time was recorded."""
    import torch
    ara.set_tuning(tables, **knobs)
    s = stream if stream is not None else torch.cuda.current_stream()
    for _ in range(warmup):
        ara.run_layers(tables, layers, out=out, flags=flags, stream=s)
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    s.synchronize()
    a.record(s)
    for _ in range(repeats):
        ara.run_layers(tables, layers, out=out, flags=flags, stream=s)
    b.record(s)
    s.synchronize()
    res = {"call_ms": a.elapsed_time(b) / repeats}
    for k in KERNEL_CLASSES.values():
        ara.kernel_stats(tables, k, reset=True)
    for _ in range(repeats):
        ara.run_layers(tables, layers, out=out, flags=flags | ara.ARA_PROFILE, stream=s)
    s.synchronize()
    recorded = 0.0
    for name, k in KERNEL_CLASSES.items():
        n, ms = ara.kernel_stats(tables, k, reset=True)
        if n:
            res[name + "_ms"] = ms / repeats
            recorded += ms
    if not recorded > 0.0 or not res["call_ms"] > 0.0:
        raise RuntimeError(f"candidate {knobs}: no device time recorded")
    return res


def measure(tables: "ara.Tables", layers: Sequence["ara.LayerSpec"], knobs: Dict[str, int], out,
            flags: int = 0, repeats: int = 5, warmup: int = 1) -> float:
    """Average device time (ms) of one ara_run_layers call with these knobs."""
    return measure_detail(tables, layers, knobs, out, flags, repeats, warmup)["call_ms"]


def tune(tables: "ara.Tables", layers: Sequence["ara.LayerSpec"], out, flags: int = 0, repeats: int = 5,
         cands: Optional[Iterable[Dict[str, int]]] = None) -> Dict[str, object]:
    """Time every candidate; set and return the best (with all timings)."""
    timings, detail = [], []
    for knobs in (cands if cands is not None else candidates(len(layers))):
        d = measure_detail(tables, layers, knobs, out, flags, repeats)
        timings.append((d["call_ms"], knobs))
        detail.append({"knobs": knobs, **{k: round(v, 4) for k, v in d.items()}})
    best_ms, best = min(timings, key=lambda x: x[0])
    ara.set_tuning(tables, **best)
    return {"best": best, "best_ms": best_ms, "timings": [(ms, k) for ms, k in timings], "detail": detail}


def tuned(tables: "ara.Tables", layers: Sequence["ara.LayerSpec"], out, flags: int = 0,
          path: str = DEFAULT_CACHE, repeats: int = 5, report: Optional[dict] = None) -> Dict[str, int]:
    """The cached choice for this (device, shape class, flags), tuning it on a
    miss; `report` (a dict) receives the timings when a tuning ran."""
    key = f"{device_name()}|{shape_class(tables, layers)}|f{flags}"
    with _LOCK:
        cache = load_cache(path)
        if key in cache:
            ara.set_tuning(tables, **cache[key])
            if report is not None:
                report.update({"cached": True, "best": cache[key]})
            return cache[key]
    res = tune(tables, layers, out, flags, repeats)
    if report is not None:
        report.update({"cached": False, "best": res["best"], "best_ms": res["best_ms"], "detail": res["detail"]})
    with _LOCK:
        cache = load_cache(path)
        cache[key] = res["best"]
        save_cache(cache, path)
    return res["best"]
