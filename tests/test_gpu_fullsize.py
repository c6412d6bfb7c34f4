"""Oracle parity at the workloads' full sizes, through the C ABI, in the launch
configurations the benchmark times.

* The 1M-trial, 16-ELT workload: every one of its 1 000 000 year losses
  against the C oracle (Algorithm 3, exact sums), then mean, PML and TVaR at
  99% and 99.6% against the oracle's sort-based metrics.
* The 64-layer library over a 256-ELT pool: every layer run in one call
  (per-layer sequences, the default), 200 sampled trials of each layer (plus
  its first and last) against the oracle; the persistent batched launch on
  the same samples.
* A portfolio of 10 programs over those 64 layers at full size (every layer
  over all trials, YET unsplit and split 8 ways): 200 sampled trials of every
  layer, program and the portfolio against the oracle.

Year losses are compared within 1e-12 of max(YLT, S) (S the annual total
before the aggregate terms: just above AggR a correctly rounded S can move the
small YLT by more than 1e-12 of itself), metrics within 1e-12 relative.
"""

import math

import numpy as np
import pytest

import oracle
from workloads import Layer, make_config, make_tiny_yet, portfolio_programs

pytestmark = pytest.mark.gpu

REL = 1e-12


@pytest.fixture(scope="module")
def ara():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_1606_04473_amd import ara as mod
    mod.lib()
    return mod


def _within(got, ref, scale):
    err = np.abs(np.asarray(got) - np.asarray(ref))
    bound = REL * np.maximum(np.abs(ref), np.abs(scale))
    return bool(np.all(err <= bound)), float(np.max(err / np.maximum(bound / REL, 1e-300), initial=0.0))


def test_config1_every_year_loss_and_metrics(ara):
    import torch
    w = make_config("config1")
    yet, pool, layer = w.yet, w.pool, w.layers[0]
    tables = ara.create_tables(yet.offsets, yet.ids, pool.losses)
    spec = ara.LayerSpec.from_layer(layer, pool, yet.n_trials)
    out = torch.empty(yet.n_trials, dtype=torch.float64, device="cuda")
    ara.run_layers(tables, [spec], out=out)
    probs = list(w.probs)
    res = ara.risk_metrics(out, probs, outputs=torch.empty(1 + 2 * len(probs), dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    ylt = out.cpu().numpy()
    h = res.cpu().numpy()
    tables.close()
    ref, S = oracle.run_layer(yet, pool, layer)
    ok, worst = _within(ylt, ref, S)
    exact = float(np.mean(ylt == ref))
    print(f"config1: {ylt.shape[0]} year losses, worst error {worst:.3e} of max(YLT, S), "
          f"{exact:.6f} bit-identical")
    assert ok, worst
    assert exact > 0.999
    mean, pml, tvar = oracle.risk_metrics(ref, probs)
    assert abs(h[0] - mean) <= REL * mean
    for q in range(len(probs)):
        assert abs(h[1 + q] - pml[q]) <= REL * pml[q], (probs[q], h[1 + q], pml[q])
        assert abs(h[1 + len(probs) + q] - tvar[q]) <= REL * tvar[q], (probs[q], h[1 + len(probs) + q], tvar[q])


@pytest.fixture(scope="module")
def cfg2(ara):
    w = make_config("config2")
    tables = ara.create_tables(w.yet.offsets, w.yet.ids, w.pool.losses)
    yield w, tables
    tables.close()


def _sample(rng, begin, count, k=200):
    s = rng.integers(begin, begin + count, size=k)
    return np.unique(np.concatenate([s, [begin, begin + count - 1]]))


def _sub_yet(yet, trials):
    return make_tiny_yet([yet.trial(int(t)).tolist() for t in trials], yet.catalogue_size)


def test_config2_every_layer_sampled(ara, cfg2):
    import torch
    w, tables = cfg2
    yet, pool = w.yet, w.pool
    specs = [ara.LayerSpec.from_layer(l, pool, yet.n_trials) for l in w.layers]
    total = sum(l.trial_count for l in w.layers)
    out = torch.empty(total, dtype=torch.float64, device="cuda")
    ara.run_layers(tables, specs, out=out)
    torch.cuda.synchronize()
    per_layer = out.cpu().numpy()
    ara.set_tuning(tables, pass_variant=1)
    ara.run_layers(tables, specs, out=out)                 # one persistent launch for all layers
    torch.cuda.synchronize()
    batched = out.cpu().numpy()
    ara.set_tuning(tables)
    rng = np.random.default_rng(201)
    off = 0
    n_checked = 0
    for i, l in enumerate(w.layers):
        trials = _sample(rng, l.trial_begin, l.trial_count)
        sub = _sub_yet(yet, trials)
        ref, S = oracle.run_layer(sub, pool, Layer(l.elt_index, l.occ_retention, l.occ_limit, l.agg_retention,
                                                  l.agg_limit, 0, sub.n_trials))
        at = off + (trials - l.trial_begin)
        for name, y in (("per-layer", per_layer), ("batched", batched)):
            ok, worst = _within(y[at], ref, S)
            assert ok, (i, name, worst)
        n_checked += trials.shape[0]
        off += l.trial_count
    assert len(w.layers) == 64 and n_checked > 64 * 200


def test_portfolio_full_size_sampled(ara, cfg2):
    import torch
    w, tables = cfg2
    yet, pool = w.yet, w.pool
    N = yet.n_trials
    progs = portfolio_programs(w.layers, 10, 0, N, seed=w.meta["seed"] + 100)
    specs = [[ara.LayerSpec.from_layer(l, pool, N) for l in p] for p in progs]
    n_layers = sum(len(p) for p in progs)
    outs = {"layer": torch.empty((n_layers, N), dtype=torch.float64, device="cuda"),
            "program": torch.empty((len(progs), N), dtype=torch.float64, device="cuda"),
            "portfolio": torch.empty(N, dtype=torch.float64, device="cuda")}
    got = {}
    for n_splits in (1, 8):
        ara.run_portfolio(tables, specs, n_splits, outs=outs)
        torch.cuda.synchronize()
        got[n_splits] = {k: v.cpu().numpy() for k, v in outs.items()}
    for k in outs:
        assert np.array_equal(got[1][k], got[8][k]), k
    trials = _sample(np.random.default_rng(202), 0, N)
    sub = _sub_yet(yet, trials)
    sub_progs = [[Layer(l.elt_index, l.occ_retention, l.occ_limit, l.agg_retention, l.agg_limit, 0, sub.n_trials)
                  for l in p] for p in progs]
    rows, prog_rows, pf_row = oracle.portfolio(sub, pool, sub_progs)
    S_rows = np.stack([oracle.run_layer(sub, pool, l)[1] for p in sub_progs for l in p])
    ok, worst = _within(got[1]["layer"][:, trials], rows, S_rows)
    assert ok, worst
    first = 0
    for p, prog in enumerate(sub_progs):
        scale = S_rows[first:first + len(prog)].sum(axis=0)
        ok, worst = _within(got[1]["program"][p, trials], prog_rows[p], scale)
        assert ok, (p, worst)
        first += len(prog)
    ok, worst = _within(got[1]["portfolio"][trials], pf_row, S_rows.sum(axis=0))
    assert ok, worst
    assert math.isfinite(float(pf_row.sum())) and np.count_nonzero(pf_row) > 100
