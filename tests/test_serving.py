"""Serving loop: admission (CPU) and alone-vs-mix equality on the GPU."""

import math
import threading
import time

import numpy as np
import pytest

from paper_1606_04473_amd.serving import (AdmissionController, make_requests, percentile, summarize,
                                          Result)


def test_admission_fifo_and_budget():
    ac = AdmissionController(100)
    assert ac.acquire(60)
    order = []

    def want(n, tag):
        assert ac.acquire(n)
        order.append(tag)

    t1 = threading.Thread(target=want, args=(50, "big"))
    t1.start()
    time.sleep(0.05)
    t2 = threading.Thread(target=want, args=(10, "small"))   # fits, but must wait behind "big"
    t2.start()
    time.sleep(0.05)
    assert order == []
    ac.release(60)
    t1.join(2)
    t2.join(2)
    assert order == ["big", "small"]
    assert ac.used == 60 and ac.peak <= 100
    ac.release(50)
    ac.release(10)
    assert ac.used == 0


def test_admission_refuses_oversized_and_times_out():
    ac = AdmissionController(10)
    assert not ac.acquire(11)
    assert ac.acquire(10)
    assert not ac.acquire(1, timeout=0.05)
    ac.release(10)
    assert ac.acquire(1)


def test_requests_are_seeded_and_shaped():
    a = make_requests(4, 5, 10.0, 50_000, 64, seed=7)
    b = make_requests(4, 5, 10.0, 50_000, 64, seed=7)
    assert [(r.rid, r.arrival, r.trial_begin, r.n_trials, r.layer_ids) for r in a] == \
           [(r.rid, r.arrival, r.trial_begin, r.n_trials, r.layer_ids) for r in b]
    assert all(a[i].arrival <= a[i + 1].arrival for i in range(len(a) - 1))
    for r in a:
        assert 10_000 <= r.n_trials <= 50_000 and 0 <= r.trial_begin <= 50_000 - r.n_trials
        assert 1 <= len(r.layer_ids) <= 16 and len(set(r.layer_ids)) == len(r.layer_ids)


def test_percentile_and_summary():
    assert percentile([1, 2, 3, 4], 50) == 2
    assert percentile([1, 2, 3, 4], 99) == 4
    rs = [Result(0, 0, 0.0, finished=0.5), Result(1, 0, 0.0, finished=1.0), Result(2, 0, 0.0, error="x")]
    s = summarize(rs, 2.0)
    assert s["completed"] == 2 and s["rejected"] == 1 and s["p99_ms"] == 1000.0


def test_power_sampler_summary_on_synthetic_samples():
    """Energy is the trapezoid integral of the power samples over time; mean
    power is that energy over the sampled span; activity is the mean of the
    samples that report one."""
    from paper_1606_04473_amd.serving import PowerSampler
    s = PowerSampler.__new__(PowerSampler)
    s.samples = [(10.0, 100.0, 50.0), (11.0, 200.0, 60.0), (13.0, 200.0, None)]
    r = s.summary()
    assert r["energy_j"] == 0.5 * (100.0 + 200.0) * 1.0 + 0.5 * (200.0 + 200.0) * 2.0
    assert r["mean_power_w"] == r["energy_j"] / 3.0
    assert r["mean_gfx_activity_pct"] == 55.0 and r["samples"] == 3
    s.samples = [(0.0, 300.0, None), (0.5, 300.0, None), (2.0, 300.0, None)]
    r = s.summary()
    assert r["energy_j"] == 600.0 and r["mean_power_w"] == 300.0 and r["mean_gfx_activity_pct"] is None
    s.samples = [(0.0, 5.0, 1.0)]
    assert s.summary() is None


def test_split_ranges_cover_the_trials():
    from paper_1606_04473_amd.serving import split_ranges
    for n, v in ((10, 3), (7, 8), (1_000_000, 8)):
        r = split_ranges(n, v)
        assert len(r) == v and sum(c for _, c in r) == n
        assert all(r[i][0] + r[i][1] == r[i + 1][0] for i in range(v - 1))
        assert max(c for _, c in r) - min(c for _, c in r) <= 1


@pytest.mark.gpu
def test_alone_equals_mix_all_modes():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1606_04473_amd import ara
    from paper_1606_04473_amd.serving import Server
    from workloads import make_elt_pool, make_yet
    C = 600_000
    yet = make_yet(20_000, 60.0, C, seed=71)
    pool = make_elt_pool(24, C, 8_000, seed=72)
    rng = np.random.default_rng(73)
    library = []
    for _ in range(10):
        J = int(rng.integers(1, 9))
        idx = rng.choice(24, size=J, replace=False).astype(np.int32)
        library.append(ara.LayerSpec(idx, pool.retention[idx], pool.limit[idx], 2000.0, 4.0e5, 5.0e4,
                                     3.0e5, 0, 0))
    bad = library[3]
    library.append(ara.LayerSpec(bad.elt_index, bad.elt_retention, bad.elt_limit, math.nan,
                                 bad.occ_limit, bad.agg_retention, bad.agg_limit, 0, 0))
    base = ara.create_tables(yet.offsets, yet.ids, pool.losses)
    reqs = make_requests(4, 4, 200.0, yet.n_trials, len(library) - 1, seed=74, n_min=500, n_max=8000,
                         layers_max=4)
    reqs[5].layer_ids = reqs[5].layer_ids + [len(library) - 1]       # poisoned request
    from paper_1606_04473_amd.serving import pin_ids
    pinned = pin_ids(yet.ids)
    ref = None
    for mode in ("resident", "concurrent", "sequential"):
        alone = Server(base, yet.offsets, yet.ids, library, 1, mode, budget_bytes=8 << 30,
                       pinned_ids=pinned).run(reqs, 0.0)
        mix = Server(base, yet.offsets, yet.ids, library, 4, mode, budget_bytes=8 << 30,
                     pinned_ids=pinned).run(reqs, 1.0)
        for a, m in zip(alone, mix):
            assert (a.error is None) == (m.error is None), (mode, a.rid, a.error, m.error)
            if a.rid == reqs[5].rid:
                assert a.error is not None and "INVALID_ARG" in a.error
                continue
            assert a.error is None, a.error
            assert a.metrics == m.metrics, (mode, a.rid)
        if ref is None:
            ref = {r.rid: r.metrics for r in alone}
        else:
            for r in alone:
                if r.error is None:
                    assert r.metrics == ref[r.rid], (mode, r.rid)
    base.close()


def test_autotune_cache_and_shape_class(tmp_path):
    from paper_1606_04473_amd import autotune

    class T:
        n_events, n_trials, catalogue_size = 1_000_000_000, 1_000_000, 2_000_000

    class L:
        def __init__(self, J, n):
            self.n_elts, self.trial_count = J, n

    one = autotune.shape_class(T, [L(16, 1_000_000)])
    many = autotune.shape_class(T, [L(16, 500_000)] * 64)
    assert one.startswith("P31-ev10-") and one.endswith("-one-J4") and "-many-" in many
    assert len(autotune.candidates(1)) == 4 and len(autotune.candidates(64)) == 8
    assert {c["pass_variant"] for c in autotune.candidates(64)} == {0, 1, 2}
    path = str(tmp_path / "cache.json")
    assert autotune.load_cache(path) == {}
    autotune.save_cache({"k": {"part_lanes_per_trial": 32}}, path)
    assert autotune.load_cache(path) == {"k": {"part_lanes_per_trial": 32}}
