"""Calibrate the layer terms of the synthetic workloads from quantiles.

TEST INFRASTRUCTURE: runs the CPU oracle once and writes the constants to
workloads/layer_terms.json, which the generators read (they never compute a
loss themselves).  Recipe, per layer:

* OccR = midpoint of the order statistics around the 10th percentile of the
  nonzero ELT-combined losses y(E) over the catalogue; OccR + OccL = the
  midpoint of the widest relative gap between distinct y values between the
  98.5th and 99.5th percentiles (the cap sits among the atoms of
  ELT-capped losses and must keep clear of them);
* AggR = midpoint around the median of the annual totals S over a sample of
  the layer's first trials (with the occurrence terms above and no aggregate
  terms); AggL = midpoint at the 99.9th percentile minus AggR.

Midpoints between distinct neighbouring values keep the terms off data
points, so no occurrence or trial sits exactly on a kink.  Usage:  python -m oracle.calibrate_layer_terms [--only config0]
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import reference as ref  # noqa: E402
from workloads import generators as gen  # noqa: E402

SAMPLE_SINGLE = 20_000
SAMPLE_LIBRARY = 4_000


def quantile_midpoint(values: np.ndarray, q_permille: int) -> float:
    """Midpoint between the order statistic k = ceil(q n) and the next larger
    distinct value.  Losses capped by one ELT's limit all share the same value,
    so plain neighbours can be equal; skipping ties keeps the term strictly
    between data values (no occurrence sits exactly on its kink)."""
    v = np.sort(np.asarray(values, dtype=np.float64))
    n = v.shape[0]
    if n < 2:
        raise ValueError("need at least two values")
    k = (q_permille * n + 999) // 1000
    k = min(max(k, 1), n - 1)
    lo = v[k - 1]
    above = v[k - 1:][v[k - 1:] > lo]
    if above.shape[0] == 0:
        below = v[v < lo]
        return float((below[-1] + lo) * 0.5) if below.shape[0] else float(lo)
    return float((lo + above[0]) * 0.5)


def widest_gap_midpoint(values: np.ndarray, lo_permille: int, hi_permille: int) -> float:
    """Midpoint of the widest relative gap between consecutive distinct values
    whose order statistics lie between the two quantiles.  Used for the
    occurrence cap, which sits among the atoms of ELT-capped losses: a
    central difference with step 1e-4 relative must not straddle an atom."""
    v = np.sort(np.asarray(values, dtype=np.float64))
    n = v.shape[0]
    a = min(max((lo_permille * n + 999) // 1000, 1), n) - 1
    b = min(max((hi_permille * n + 999) // 1000, 1), n)
    d = np.unique(v[a:b + 1])
    if d.shape[0] < 2:
        return quantile_midpoint(v, (lo_permille + hi_permille) // 2)
    rel = (d[1:] - d[:-1]) / d[1:]
    i = int(np.argmax(rel))
    return float((d[i] + d[i + 1]) * 0.5)


def calibrate(yet, pool, layer: gen.Layer, n_sample: int) -> dict:
    free = gen.Layer(layer.elt_index, 0.0, math.inf, 0.0, math.inf, layer.trial_begin,
                     layer.trial_count)
    y, _ = ref.occurrence_catalogue(pool, free)
    nz = y[y > 0.0]
    occ_r = quantile_midpoint(nz, 100)
    occ_l = widest_gap_midpoint(nz, 985, 995) - occ_r
    count = layer.resolved_count(yet.n_trials)
    sample = gen.Layer(layer.elt_index, occ_r, occ_l, 0.0, math.inf, layer.trial_begin,
                       min(n_sample, count))
    _, S = ref.run_layer(yet, pool, sample)
    agg_r = quantile_midpoint(S, 500)
    agg_l = quantile_midpoint(S, 999) - agg_r
    return dict(occ_retention=occ_r, occ_limit=occ_l, agg_retention=agg_r, agg_limit=agg_l,
                sample_trials=int(sample.trial_count))


def main(argv=None) -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default=None)
    args = ap.parse_args(argv)
    path = gen._TERMS_FILE
    out = gen.load_layer_terms()
    out["recipe"] = (
        "OccR = q10 midpoint of nonzero y(E); OccR + OccL = midpoint of the widest gap "
        "between distinct y values in [q98.5, q99.5]; "
        "AggR = q50 midpoint of S over the first sample_trials trials; "
        "AggL = q99.9 midpoint - AggR; written by oracle/calibrate_layer_terms.py")
    for name in ("config0", "config1"):
        if args.only and args.only != name:
            continue
        t0 = time.time()
        w = gen.make_config(name, n_prefix=SAMPLE_SINGLE, calibrated=False)
        out[name] = calibrate(w.yet, w.pool, w.layers[0], SAMPLE_SINGLE)
        print(name, out[name], f"{time.time() - t0:.1f}s", flush=True)
    if args.only in (None, "library"):
        t0 = time.time()
        w = gen.make_config("config2", calibrated=False)
        lib = []
        for i, layer in enumerate(w.layers):
            entry = calibrate(w.yet, w.pool, layer, SAMPLE_LIBRARY)
            entry.update(elt_index=layer.elt_index.tolist(), trial_begin=layer.trial_begin,
                         trial_count=layer.trial_count)
            lib.append(entry)
            print("library", i, f"J={layer.n_elts}", f"{time.time() - t0:.1f}s", flush=True)
        out["library"] = lib
    with open(path + ".tmp", "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")
    os.replace(path + ".tmp", path)
    print("wrote", path)


if __name__ == "__main__":
    main()
