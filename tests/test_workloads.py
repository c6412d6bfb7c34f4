"""Generator determinism, prefix consistency and input-shape checks."""

import hashlib

import numpy as np

from workloads import (ELTPool, elt_terms_from_losses, make_config, make_elt_pool,
                       make_tiny_yet, make_yet)


def _h(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def test_yet_deterministic_and_prefix_consistent():
    a = make_yet(200_000, 20.0, 50_000, seed=7)
    b = make_yet(200_000, 20.0, 50_000, seed=7)
    assert _h(a.ids) == _h(b.ids) and _h(a.offsets) == _h(b.offsets)
    p = make_yet(200_000, 20.0, 50_000, seed=7, n_prefix=70_000)
    assert p.n_trials == 70_000
    assert np.array_equal(p.offsets, a.offsets[:70_001])
    assert np.array_equal(p.ids, a.ids[:p.n_events])
    c = make_yet(200_000, 20.0, 50_000, seed=8)
    assert _h(c.ids) != _h(a.ids)


def test_yet_shape_and_distribution():
    y = make_yet(20_000, 100.0, 100_000, seed=3, with_timestamps=True)
    K = np.diff(y.offsets)
    assert y.offsets[0] == 0 and np.all(K >= 0)
    assert abs(K.mean() - 100.0) < 0.5
    assert y.ids.dtype == np.uint32 and int(y.ids.max()) < 100_000
    ts = y.timestamps
    assert ts.dtype == np.float32 and ts.shape == y.ids.shape
    assert float(ts.min()) >= 0.0 and float(ts.max()) < 365.0
    for t in range(0, 20_000, 997):
        seg = ts[y.offsets[t]:y.offsets[t + 1]]
        assert np.all(np.diff(seg) >= 0)


def test_elt_pool_layout_and_terms():
    pool = make_elt_pool(3, 10_000, 500, seed=9)
    assert pool.losses.shape == (3, 10_000)
    for j in range(3):
        row = pool.losses[j]
        nz = row[row != 0.0]
        assert nz.shape[0] == 500 and np.all(nz > 0.0)
        R, L = elt_terms_from_losses(nz)
        assert R == pool.retention[j] and L == pool.limit[j]
        v = np.sort(nz)
        assert v[99] < R < v[100]           # k = ceil(0.2 * 500) = 100
        assert v[474] < L < v[475]          # k = ceil(0.95 * 500) = 475
    again = make_elt_pool(3, 10_000, 500, seed=9)
    assert np.array_equal(again.losses, pool.losses)


def test_tiny_yet():
    y = make_tiny_yet([[1, 2], [], [5]], 8)
    assert y.offsets.tolist() == [0, 2, 2, 3] and y.ids.tolist() == [1, 2, 5]
    assert isinstance(ELTPool(np.zeros((1, 8)), np.zeros(1), np.zeros(1)).n_elts, int)


def test_config0_matches_recipe():
    w = make_config("config0")
    assert w.yet.n_trials == 10_000 and w.yet.catalogue_size == 100_000
    assert w.pool.losses.shape == (4, 100_000)
    layer = w.layers[0]
    assert layer.elt_index.tolist() == [0, 1, 2, 3]
    assert 0 < layer.occ_retention < layer.occ_limit
    assert 0 < layer.agg_retention and 0 < layer.agg_limit
    assert tuple(w.probs) == (0.99,)


def test_portfolio_programs_partition_the_layers():
    from workloads import Layer, portfolio_programs
    layers = [Layer(np.array([i % 7], dtype=np.int32), 0.0, 1.0, 0.0, 2.0, 5 * i, 10 + i)
              for i in range(64)]
    a = portfolio_programs(layers, 10, 0, 1000, seed=7)
    b = portfolio_programs(layers, 10, 0, 1000, seed=7)
    assert len(a) == 10 and all(len(p) >= 1 for p in a)
    flat = [l for p in a for l in p]
    assert [int(l.elt_index[0]) for l in flat] == [i % 7 for i in range(64)]   # order kept
    assert all(l.trial_begin == 0 and l.trial_count == 1000 for l in flat)
    assert [len(p) for p in a] == [len(p) for p in b]
    assert [len(p) for p in portfolio_programs(layers, 1, 0, 9, seed=1)] == [64]
