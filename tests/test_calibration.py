"""The stored layer terms are reproducible from their recipe and keep every
kink off the data (no occurrence or trial sits exactly on a clamp boundary),
so finite differences and strict subgradients agree."""

import json
import math

import numpy as np
import pytest

import oracle
from oracle import calibrate_layer_terms as cal
from workloads import generators as gen
from workloads import make_config


def test_widest_gap_midpoint():
    v = np.array([1.0, 2.0, 2.0, 2.1, 3.0, 3.05, 9.0, 10.0])
    # between the order statistics k=2..8 the widest relative gap is 3.05 -> 9.0
    assert cal.widest_gap_midpoint(v, 200, 1000) == 6.025


def test_quantile_midpoint_skips_ties():
    v = np.array([1.0, 2.0, 2.0, 2.0, 2.0, 5.0])
    # k = ceil(0.5 * 6) = 3 -> v_3 = 2.0; next distinct value 5.0
    assert cal.quantile_midpoint(v, 500) == 3.5
    assert cal.quantile_midpoint(np.array([1.0, 3.0]), 500) == 2.0


def test_config0_terms_reproducible():
    w = make_config("config0", calibrated=False)
    got = cal.calibrate(w.yet, w.pool, w.layers[0], cal.SAMPLE_SINGLE)
    stored = gen.load_layer_terms()["config0"]
    for k in ("occ_retention", "occ_limit", "agg_retention", "agg_limit"):
        assert got[k] == stored[k], k


@pytest.mark.parametrize("name,n_prefix", [("config0", None), ("config1", 20_000)])
def test_terms_off_data_atoms(name, n_prefix):
    w = make_config(name, n_prefix=n_prefix)
    layer = w.layers[0]
    y, _ = oracle.occurrence_catalogue(w.pool, layer)
    nz = y[y > 0.0]
    for edge in (layer.occ_retention, layer.occ_retention + layer.occ_limit):
        assert np.min(np.abs(nz - edge)) > 1e-9 * edge
    # the cap keeps a central difference at step 1e-4 clear of every atom
    cap = layer.occ_retention + layer.occ_limit
    assert np.min(np.abs(nz - cap)) > 2e-4 * cap
    _, S = oracle.run_layer(w.yet, w.pool, layer)
    for edge in (layer.agg_retention, layer.agg_retention + layer.agg_limit):
        assert np.min(np.abs(S - edge)) > 1e-9 * edge
    for j in layer.elt_index:
        row = w.pool.losses[j]
        row = row[row > 0.0]
        R, L = w.pool.retention[j], w.pool.limit[j]
        assert np.min(np.abs(row - R)) > 1e-9 * R
        assert np.min(np.abs(row - (R + L))) > 1e-9 * (R + L)
