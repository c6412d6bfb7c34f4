"""Pins that tie the CPU oracle to the paper's definitions and to mathematics.

Each test checks the oracle against something other than itself: hand-worked
closed forms (tests/golden), invariants that follow from the term
definitions, a textbook reduction (sparse matrix-vector product), brute force
over tiny inputs with an independent pure-Python rendering, Python's
math.fsum, and finite differences for the gradients.
"""

import itertools
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from workloads import ELTPool, Layer, make_tiny_yet, make_yet, make_elt_pool

INF = math.inf


def _inf(v):
    return INF if v == "inf" else float(v)


@pytest.fixture(scope="module")
def golden(golden_dir):
    with open(os.path.join(golden_dir, "closed_form_cases.json")) as f:
        return json.load(f)


def _golden_pool(g):
    losses = np.array(g["elts"], dtype=np.float64)
    return ELTPool(losses=losses, retention=np.array(g["elt_retention"]),
                   limit=np.array(g["elt_limit"]))


def _golden_layer(case, n_trials):
    t = case["terms"]
    return Layer(np.array(case["elt_index"], dtype=np.int32), _inf(t["occ_retention"]),
                 _inf(t["occ_limit"]), _inf(t["agg_retention"]), _inf(t["agg_limit"]), 0,
                 n_trials)


# ---------------------------------------------------------------------------
# exact summation
# ---------------------------------------------------------------------------

def test_exact_sum_matches_fsum_random():
    rng = np.random.default_rng(1)
    for _ in range(200):
        n = int(rng.integers(0, 400))
        x = rng.lognormal(10, 4, size=n) * rng.choice([1.0, 1e-20, 1e20], size=n)
        assert oracle.exact_sum(x) == math.fsum(x.tolist())


def test_exact_sum_matches_fsum_adversarial():
    cases = [
        [1e16, 1.0, -1e16],
        [1.0, 1e100, 1.0, -1e100],
        [0.1] * 10,
        [2.0 ** 53, 1.0, 1.0],                  # half-way cases
        [2.0 ** 53, 1.0, 2.0 ** -60],
        [2.0 ** 53, 1.0, -(2.0 ** -60)],
        [1.0, 2.0 ** -53, 2.0 ** -106],
        [5e-324, 5e-324, 1.0],
        [],
    ]
    for c in cases:
        assert oracle.exact_sum(np.array(c, dtype=np.float64)) == math.fsum(c), c


# ---------------------------------------------------------------------------
# P1: closed forms
# ---------------------------------------------------------------------------

def test_closed_form_year_losses(golden):
    pool = _golden_pool(golden)
    for case in golden["cases"]:
        yet = make_tiny_yet(case["trials"], golden["catalogue_size"])
        layer = _golden_layer(case, yet.n_trials)
        for mode in ("exact", "sequential"):
            ylt, S = oracle.run_layer(yet, pool, layer, sum_mode=mode)
            assert ylt.tolist() == case["year_loss"], (case["name"], mode)
            if "annual_total" in case:
                assert S.tolist() == case["annual_total"]
        ylt_py, _ = oracle.run_layer_python(case["trials"], pool.losses, layer.elt_index,
                                            pool.retention[layer.elt_index],
                                            pool.limit[layer.elt_index], layer.occ_retention,
                                            layer.occ_limit, layer.agg_retention,
                                            layer.agg_limit)
        assert ylt_py == case["year_loss"]
        ylt_np, _, _, _ = oracle.run_layer_numpy(yet, pool, layer)
        assert ylt_np.tolist() == case["year_loss"]


def test_closed_form_per_event_values(golden):
    pool = _golden_pool(golden)
    both = Layer(np.array([0, 1], dtype=np.int32), 0.0, INF, 0.0, INF)
    y, o = oracle.occurrence_catalogue(pool, both)
    assert y.tolist() == golden["combined_y"]
    assert o.tolist() == golden["combined_y"]
    caseB = golden["cases"][1]
    layerB = _golden_layer(caseB, 1)
    _, oB = oracle.occurrence_catalogue(pool, layerB)
    assert oB.tolist() == caseB["occurrence_net"]
    for j in range(2):
        single = Layer(np.array([j], dtype=np.int32), 0.0, INF, 0.0, INF)
        yj, _ = oracle.occurrence_catalogue(pool, single)
        assert yj.tolist() == golden["net_x"][j]


def test_closed_form_metrics(golden):
    g = golden["metrics_case_C_first4"]
    ylt = np.array(g["year_loss"])
    for row in g["by_p"]:
        mean, pml, tvar = oracle.risk_metrics(ylt, [row["p"]])
        assert mean == g["mean"]
        assert oracle.tail_count(4, row["p"]) == row["m"]
        assert pml[0] == row["pml"]
        expected = row["tvar"] if "tvar" in row else row["tvar_num"] / row["tvar_den"]
        assert tvar[0] == expected


def test_closed_form_gradients(golden):
    pool = _golden_pool(golden)
    caseC = golden["cases"][2]
    g = golden["gradients_case_C_first4"]
    trials = caseC["trials"][:4]
    yet = make_tiny_yet(trials, golden["catalogue_size"])
    layer = _golden_layer(caseC, yet.n_trials)
    res = oracle.gradients(yet, pool, layer, g["tvar_p"])
    assert res["grad_mean"].tolist() == g["grad_mean"]
    assert res["grad_tvar"].tolist() == g["grad_tvar"]
    yet6 = make_tiny_yet([[6]], golden["catalogue_size"])
    layer6 = _golden_layer(caseC, 1)
    _, S6 = oracle.run_layer(yet6, pool, layer6)
    c6 = oracle.grad_counts(yet6, pool, layer6, S6)
    assert c6[0].tolist() == g["trial_6_alone"]


def test_kink_subgradient_and_fd(golden):
    """At an exact kink the strict subgradient is 0 while the central finite
    difference is -1/2 per occurrence sitting on the kink."""
    losses = np.array(golden["elts"], dtype=np.float64)[:1].copy()
    losses[0, 3] = 40.0
    R = 40.0
    pool = ELTPool(losses=losses, retention=np.array([R]), limit=np.array([300.0]))
    yet = make_tiny_yet([[3, 1]], 8)
    layer = Layer(np.array([0], dtype=np.int32), 0.0, INF, 0.0, INF, 0, 1)
    res = oracle.gradients(yet, pool, layer, 0.5)
    # event 1 (loss 100) is in band: -1; event 3 sits on the kink: 0
    assert res["grad_mean"][0] == -1.0
    h = 1e-3

    def f(r):
        p = ELTPool(losses=losses, retention=np.array([r]), limit=np.array([300.0]))
        return oracle.run_layer(yet, p, layer)[0][0]

    fd = (f(R + h) - f(R - h)) / (2 * h)
    assert abs(fd - (-1.5)) < 1e-9


# ---------------------------------------------------------------------------
# small random workload used by the invariant and reduction pins
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def small():
    C = 3000
    yet = make_yet(400, 40.0, C, seed=11)
    pool = make_elt_pool(6, C, 400, seed=12)
    layer = Layer(np.array([4, 0, 2, 5], dtype=np.int32), 3000.0, 5.0e5, 2.0e5, 1.5e6, 0, 400)
    return yet, pool, layer


def test_bounds_and_empty_trials(small):
    yet, pool, layer = small
    ylt, S = oracle.run_layer(yet, pool, layer)
    assert np.all(ylt >= 0.0) and np.all(ylt <= layer.agg_limit)
    assert np.all(S >= 0.0)
    empty = make_tiny_yet([[], [], []], yet.catalogue_size)
    ylt0, S0 = oracle.run_layer(empty, pool, Layer(layer.elt_index, 0.0, INF, 0.0, INF, 0, 3))
    assert ylt0.tolist() == [0.0, 0.0, 0.0] and S0.tolist() == [0.0, 0.0, 0.0]


def _with_terms(pool, R=None, Lim=None):
    return ELTPool(losses=pool.losses,
                   retention=pool.retention if R is None else R,
                   limit=pool.limit if Lim is None else Lim)


def test_monotone_in_retentions_and_limits(small):
    yet, pool, layer = small
    base, _ = oracle.run_layer(yet, pool, layer)
    for j in layer.elt_index:
        R = pool.retention.copy()
        R[j] *= 1.5
        up, _ = oracle.run_layer(yet, _with_terms(pool, R=R), layer)
        assert np.all(up <= base)
        Lim = pool.limit.copy()
        Lim[j] *= 1.5
        up, _ = oracle.run_layer(yet, _with_terms(pool, Lim=Lim), layer)
        assert np.all(up >= base)
    for field, sign in (("occ_retention", -1), ("agg_retention", -1), ("occ_limit", 1),
                        ("agg_limit", 1)):
        l2 = Layer(**{**layer.__dict__, field: getattr(layer, field) * 1.3})
        up, _ = oracle.run_layer(yet, pool, l2)
        assert np.all(sign * (up - base) >= 0.0), field


def test_power_of_two_homogeneity_is_bit_exact(small):
    yet, pool, layer = small
    base, _ = oracle.run_layer(yet, pool, layer)
    for k in (-3, 5):
        s = 2.0 ** k
        p2 = ELTPool(losses=pool.losses * s, retention=pool.retention * s, limit=pool.limit * s)
        l2 = Layer(layer.elt_index, layer.occ_retention * s, layer.occ_limit * s,
                   layer.agg_retention * s, layer.agg_limit * s, 0, layer.trial_count)
        ylt, _ = oracle.run_layer(yet, p2, l2)
        assert np.array_equal(ylt, base * s)


def test_event_permutation_and_trial_split(small):
    yet, pool, layer = small
    base, S = oracle.run_layer(yet, pool, layer)
    rng = np.random.default_rng(5)
    ids = yet.ids.copy()
    for t in range(yet.n_trials):
        seg = ids[yet.offsets[t]:yet.offsets[t + 1]]
        rng.shuffle(seg)
    perm = make_tiny_yet([ids[yet.offsets[t]:yet.offsets[t + 1]] for t in range(yet.n_trials)],
                         yet.catalogue_size)
    ylt_p, S_p = oracle.run_layer(perm, pool, layer)
    assert np.array_equal(ylt_p, base)          # exact sums do not depend on order
    ylt_seq, S_seq = oracle.run_layer(perm, pool, layer, sum_mode="sequential")
    K = np.diff(yet.offsets)
    assert np.all(np.abs(S_seq - S) <= K * 2.0 ** -53 * S + 1e-300)
    parts = []
    for b, c in ((0, 150), (150, 1), (151, 249)):
        l2 = Layer(layer.elt_index, layer.occ_retention, layer.occ_limit, layer.agg_retention,
                   layer.agg_limit, b, c)
        parts.append(oracle.run_layer(yet, pool, l2)[0])
    assert np.array_equal(np.concatenate(parts), base)


def test_aggregate_retention_above_all_totals(small):
    yet, pool, layer = small
    _, S = oracle.run_layer(yet, pool, layer)
    l2 = Layer(layer.elt_index, layer.occ_retention, layer.occ_limit, float(S.max()), INF, 0,
               layer.trial_count)
    ylt, _ = oracle.run_layer(yet, pool, l2)
    assert np.all(ylt == 0.0)


def test_sparse_matvec_reduction(small):
    """Retentions 0 and limits infinite: YLT = A (sum_j ELT_j) with A the
    trial-by-event multiplicity matrix -- a plain sparse matrix-vector product."""
    yet, pool, layer = small
    J = layer.n_elts
    p0 = ELTPool(losses=pool.losses, retention=np.zeros(pool.n_elts),
                 limit=np.full(pool.n_elts, INF))
    l0 = Layer(layer.elt_index, 0.0, INF, 0.0, INF, 0, yet.n_trials)
    ylt, _ = oracle.run_layer(yet, p0, l0)
    rows = np.repeat(np.arange(yet.n_trials), np.diff(yet.offsets))
    A = sp.csr_matrix((np.ones(yet.n_events), (rows, yet.ids.astype(np.int64))),
                      shape=(yet.n_trials, yet.catalogue_size))
    v = pool.losses[layer.elt_index].sum(axis=0)
    ref = A @ v
    assert np.allclose(ylt, ref, rtol=1e-13, atol=0.0)
    # one ELT: each occurrence's loss is the raw table value, so the year loss
    # is exactly fsum of the looked-up losses
    l1 = Layer(layer.elt_index[:1], 0.0, INF, 0.0, INF, 0, yet.n_trials)
    ylt1, _ = oracle.run_layer(yet, p0, l1)
    row = pool.losses[layer.elt_index[0]]
    for t in range(yet.n_trials):
        assert ylt1[t] == math.fsum(row[yet.trial(t).astype(np.int64)].tolist())
    assert J > 1
    with_terms, _ = oracle.run_layer(yet, pool, layer)
    _, _, _, o = oracle.run_layer_numpy(yet, pool, layer)
    S_ref = A @ o
    t = np.minimum(np.maximum(S_ref - layer.agg_retention, 0.0), layer.agg_limit)
    assert np.allclose(with_terms, t, rtol=1e-12, atol=1e-6)


def test_three_formulations_agree_bit_exact(small):
    yet, pool, layer = small
    ylt, S = oracle.run_layer(yet, pool, layer)
    ylt_np, S_np, y_np, o_np = oracle.run_layer_numpy(yet, pool, layer)
    assert np.array_equal(ylt, ylt_np) and np.array_equal(S, S_np)
    y, o = oracle.occurrence_catalogue(pool, layer)
    assert np.array_equal(y, y_np) and np.array_equal(o, o_np)
    trials = [yet.trial(t).tolist() for t in range(0, yet.n_trials, 13)]
    ylt_py, S_py = oracle.run_layer_python(trials, pool.losses, layer.elt_index,
                                           pool.retention[layer.elt_index],
                                           pool.limit[layer.elt_index], layer.occ_retention,
                                           layer.occ_limit, layer.agg_retention, layer.agg_limit)
    assert ylt_py == ylt[::13].tolist()


def test_brute_force_tiny():
    """Every trial of up to 3 events over a 6-event catalogue."""
    rng = np.random.default_rng(3)
    C = 6
    losses = np.where(rng.random((3, C)) < 0.6, rng.integers(1, 50, (3, C)) * 8.0, 0.0)
    pool = ELTPool(losses=losses, retention=np.array([16.0, 0.0, 40.0]),
                   limit=np.array([200.0, 96.0, INF]))
    trials = [list(t) for k in range(4) for t in itertools.product(range(C), repeat=k)]
    yet = make_tiny_yet(trials, C)
    for terms in ((0.0, INF, 0.0, INF), (24.0, 160.0, 40.0, 300.0), (1000.0, 8.0, 0.0, 8.0)):
        layer = Layer(np.array([2, 0, 1], dtype=np.int32), *terms, 0, yet.n_trials)
        ylt, _ = oracle.run_layer(yet, pool, layer)
        ylt_py, _ = oracle.run_layer_python(trials, losses, layer.elt_index,
                                            pool.retention[layer.elt_index],
                                            pool.limit[layer.elt_index], *terms)
        assert ylt.tolist() == ylt_py


# ---------------------------------------------------------------------------
# per-event nets (aggregate terms on the running total)
# ---------------------------------------------------------------------------

def test_closed_form_event_nets(golden):
    pool = _golden_pool(golden)
    for case in golden["cases"]:
        if "event_nets" not in case:
            continue
        yet = make_tiny_yet(case["trials"], golden["catalogue_size"])
        layer = _golden_layer(case, yet.n_trials)
        assert oracle.event_nets(yet, pool, layer).tolist() == case["event_nets"], case["name"]
        py = oracle.event_nets_python(case["trials"], pool.losses, layer.elt_index,
                                      pool.retention[layer.elt_index],
                                      pool.limit[layer.elt_index], layer.occ_retention,
                                      layer.occ_limit, layer.agg_retention, layer.agg_limit)
        assert py == case["event_nets"]
        # a sub-range starts its output at the range's first event
        sub = Layer(layer.elt_index, layer.occ_retention, layer.occ_limit,
                    layer.agg_retention, layer.agg_limit, 1, yet.n_trials - 2)
        first = int(yet.offsets[1])
        last = int(yet.offsets[yet.n_trials - 1])
        assert oracle.event_nets(yet, pool, sub).tolist() == case["event_nets"][first:last]


def test_event_nets_brute_force_tiny():
    """Every trial of up to 3 events over a 6-event catalogue, against prefix
    totals recomputed from scratch."""
    rng = np.random.default_rng(5)
    C = 6
    losses = np.where(rng.random((3, C)) < 0.6, rng.integers(1, 50, (3, C)) * 8.0, 0.0)
    pool = ELTPool(losses=losses, retention=np.array([16.0, 0.0, 40.0]),
                   limit=np.array([200.0, 96.0, INF]))
    trials = [list(t) for k in range(4) for t in itertools.product(range(C), repeat=k)]
    yet = make_tiny_yet(trials, C)
    for terms in ((0.0, INF, 0.0, INF), (24.0, 160.0, 40.0, 300.0), (0.0, INF, 100.0, 50.0)):
        layer = Layer(np.array([2, 0, 1], dtype=np.int32), *terms, 0, yet.n_trials)
        nets = oracle.event_nets(yet, pool, layer)
        py = oracle.event_nets_python(trials, losses, layer.elt_index,
                                      pool.retention[layer.elt_index],
                                      pool.limit[layer.elt_index], *terms)
        assert nets.tolist() == py


def test_event_nets_invariants(small):
    """nets >= 0; a net never exceeds its occurrence loss (clamp is
    1-Lipschitz and non-decreasing); a trial's nets add up to its year loss
    (A_0 = 0 for a non-negative retention); no aggregate limit gives back the
    occurrence losses themselves."""
    yet, pool, layer = small
    nets = oracle.event_nets(yet, pool, layer)
    ylt, _ = oracle.run_layer(yet, pool, layer)
    _, o = oracle.occurrence_catalogue(pool, layer)
    eps = np.finfo(np.float64).eps
    assert nets.shape[0] == yet.offsets[-1]
    assert np.all(nets >= 0.0)
    o_ev = o[yet.ids.astype(np.int64)]
    for t in range(yet.n_trials):
        b, e = int(yet.offsets[t]), int(yet.offsets[t + 1])
        scale = max(ylt[t], 1.0)
        assert np.all(nets[b:e] <= o_ev[b:e] + 4 * eps * layer.agg_limit)
        assert abs(math.fsum(nets[b:e].tolist()) - ylt[t]) <= (e - b + 1) * eps * scale
    free = Layer(layer.elt_index, layer.occ_retention, layer.occ_limit, 0.0, INF, 0, yet.n_trials)
    nets_free = oracle.event_nets(yet, pool, free)
    # A_d - A_{d-1} = S_d - S_{d-1} with both rounded from exact prefixes
    assert np.allclose(nets_free, o_ev, rtol=0.0, atol=1e-9 * float(o.max()))


# ---------------------------------------------------------------------------
# portfolio: programs of layers over one YET
# ---------------------------------------------------------------------------

def _golden_portfolio(golden):
    pool = _golden_pool(golden)
    pc = golden["portfolio_case"]
    yet = make_tiny_yet(pc["trials"], golden["catalogue_size"])
    by_name = {c["name"][0]: _golden_layer(c, yet.n_trials) for c in golden["cases"]}
    programs = [[by_name[name] for name in prog] for prog in pc["programs"]]
    return yet, pool, programs, pc


def test_closed_form_portfolio(golden):
    yet, pool, programs, pc = _golden_portfolio(golden)
    rows, prog_rows, pf = oracle.portfolio(yet, pool, programs)
    assert rows.tolist() == pc["layer_ylt"]
    assert prog_rows.tolist() == pc["program_ylt"]
    assert pf.tolist() == pc["portfolio_ylt"]


def test_portfolio_sums_round_once():
    """Layer year losses 2^53, 1, 1: the sum rounded once is 2^53 + 2; adding
    in turn in FP64 would give 2^53 twice over (ties to even)."""
    big = 2.0 ** 53
    pool = ELTPool(losses=np.array([[big], [1.0], [1.0]]), retention=np.zeros(3),
                   limit=np.full(3, INF))
    yet = make_tiny_yet([[0], []], 1)
    layers = [Layer(np.array([j], dtype=np.int32), 0.0, INF, 0.0, INF, 0, 2) for j in range(3)]
    rows, prog_rows, pf = oracle.portfolio(yet, pool, [layers])
    assert rows[:, 0].tolist() == [big, 1.0, 1.0]
    assert prog_rows.tolist() == [[big + 2.0, 0.0]]
    assert pf.tolist() == [big + 2.0, 0.0]
    assert (big + 1.0) + 1.0 == big      # the sequential order really does lose both


def test_portfolio_reductions(small):
    """One program of one layer is that layer; programs of integer-valued
    layers add up exactly to the portfolio; layers over other trials are
    rejected."""
    yet, pool, layer = small
    ylt, _ = oracle.run_layer(yet, pool, layer)
    rows, prog_rows, pf = oracle.portfolio(yet, pool, [[layer]])
    assert np.array_equal(rows[0], ylt) and np.array_equal(prog_rows[0], ylt)
    assert np.array_equal(pf, ylt)
    ints = ELTPool(losses=np.floor(pool.losses / 64.0), retention=np.zeros(pool.losses.shape[0]),
                   limit=np.full(pool.losses.shape[0], INF))
    lay = [Layer(np.array(ix, dtype=np.int32), 0.0, INF, 0.0, INF, 0, yet.n_trials)
           for ix in ([0, 1], [2], [3, 4, 5], [1, 3])]
    rows, prog_rows, pf = oracle.portfolio(yet, ints, [lay[:2], lay[2:]])
    assert np.array_equal(prog_rows[0], rows[0] + rows[1])
    assert np.array_equal(pf, prog_rows[0] + prog_rows[1])
    other = Layer(lay[0].elt_index, 0.0, INF, 0.0, INF, 1, yet.n_trials - 1)
    with pytest.raises(ValueError):
        oracle.portfolio(yet, ints, [[lay[0], other]])


# ---------------------------------------------------------------------------
# P5: metrics
# ---------------------------------------------------------------------------

def test_tail_count_values():
    """Hand-worked values of m = ceil(N (1 - p)) with p read as its decimal."""
    assert oracle.tail_count(1_000_000, 0.99) == 10_000      # FP64 (1-p)*N is 10000.000000000009
    assert oracle.tail_count(1_000_000, 0.996) == 4_000
    assert oracle.tail_count(10_000, 0.99) == 100
    assert oracle.tail_count(4, 0.5) == 2
    assert oracle.tail_count(3, 0.99) == 1                   # 0.03 -> 1
    assert oracle.tail_count(7, 0.5) == 4                    # 3.5 -> 4
    # 10^6 x 0.010000000001 = 10000.000001 -> 10001 (a 1e-9 snap would say 10000)
    assert oracle.tail_count(1_000_000, 0.989999999999) == 10_001
    # repr(1/3) = 0.3333333333333333: 3 x 0.6666666666666667 = 2.0000000000000001 -> 3
    assert oracle.tail_count(3, 1.0 / 3.0) == 3
    # repr(2/3) = 0.6666666666666666: 3 x 0.3333333333333334 = 1.0000000000000002 -> 2
    assert oracle.tail_count(3, 2.0 / 3.0) == 2
    assert oracle.tail_count(1, 0.999) == 1                  # clamped up to 1
    assert oracle.tail_count(10, 1e-300) == 10               # 10 - 1e-299 -> 10
    assert oracle.tail_count(2 ** 62, 0.75) == 2 ** 60       # exact at large N
    with pytest.raises(ValueError):
        oracle.tail_count(10, 1.0)
    with pytest.raises(ValueError):
        oracle.tail_count(0, 0.5)


def test_lookups_golden_tables(golden_dir):
    """oracle.lookups returns the trial's IDs in storage order and the raw
    losses [event][ELT] in the layer's ELT order (values written out by hand
    from the golden ELT rows)."""
    g = json.load(open(os.path.join(golden_dir, "closed_form_cases.json")))
    losses = np.array(g["elts"], dtype=np.float64)
    pool = ELTPool(losses, np.array(g["elt_retention"]), np.array(g["elt_limit"]))
    yet = make_tiny_yet([[1, 2, 6], [3], [], [6, 6, 2]], g["catalogue_size"])
    both = Layer(np.array([0, 1], dtype=np.int32), 0.0, INF, 0.0, INF, 0, yet.n_trials)
    rev = Layer(np.array([1, 0], dtype=np.int32), 0.0, INF, 0.0, INF, 0, yet.n_trials)
    ids, got = oracle.lookups(yet, pool, both, 0)
    assert ids.tolist() == [1, 2, 6]
    assert got.tolist() == [[100.0, 0.0], [250.0, 100.0], [500.0, 1000.0]]
    ids, got = oracle.lookups(yet, pool, rev, 0)
    assert got.tolist() == [[0.0, 100.0], [100.0, 250.0], [1000.0, 500.0]]
    ids, got = oracle.lookups(yet, pool, both, 1)
    assert ids.tolist() == [3] and got.tolist() == [[40.0, 0.0]]
    ids, got = oracle.lookups(yet, pool, both, 2)
    assert ids.tolist() == [] and got.shape == (0, 2)
    ids, got = oracle.lookups(yet, pool, both, 3)
    assert ids.tolist() == [6, 6, 2]
    assert got.tolist() == [[500.0, 1000.0], [500.0, 1000.0], [250.0, 100.0]]


def test_metrics_on_permutations():
    rng = np.random.default_rng(8)
    for n in (1, 2, 10, 997, 10_000):
        y = rng.permutation(np.arange(1, n + 1)).astype(np.float64)
        probs = [0.5, 0.9, 0.99, 0.996]
        mean, pml, tvar = oracle.risk_metrics(y, probs)
        assert mean == (n + 1) / 2
        for p, a, b in zip(probs, pml, tvar):
            m = oracle.tail_count(n, p)
            assert a == n - m + 1
            assert b == n - (m - 1) / 2


# ---------------------------------------------------------------------------
# P6: gradients
# ---------------------------------------------------------------------------

def test_gradient_closed_forms_and_fd(small):
    yet, pool, layer = small
    ylt, S = oracle.run_layer(yet, pool, layer)
    res = oracle.gradients(yet, pool, layer, 0.9, ylt=ylt, S=S)
    J = layer.n_elts
    n = yet.n_trials
    ta = S - layer.agg_retention
    assert res["num_mean"][2 * J + 3] == int(np.sum(ta > layer.agg_limit))
    assert res["num_mean"][2 * J + 2] == -int(np.sum((ta > 0) & (ta < layer.agg_limit)))
    idx = layer.elt_index

    def fwd(theta):
        R = pool.retention.copy()
        Lim = pool.limit.copy()
        R[idx] = theta[:J]
        Lim[idx] = theta[J:2 * J]
        l2 = Layer(idx, theta[2 * J], theta[2 * J + 1], theta[2 * J + 2], theta[2 * J + 3], 0, n)
        y, _ = oracle.run_layer(yet, _with_terms(pool, R, Lim), l2)
        mean, _, tvar = oracle.risk_metrics(y, [0.9])
        return mean, tvar[0]

    theta = np.concatenate([pool.retention[idx], pool.limit[idx],
                            [layer.occ_retention, layer.occ_limit, layer.agg_retention,
                             layer.agg_limit]])
    for k in range(theta.shape[0]):
        h = 1e-6 * max(abs(theta[k]), 1.0)
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        (mp, vp), (mm, vm) = fwd(tp), fwd(tm)
        fd_mean = (mp - mm) / (2 * h)
        fd_tvar = (vp - vm) / (2 * h)
        assert abs(fd_mean - res["grad_mean"][k]) <= 1e-6 * max(1.0, abs(res["grad_mean"][k])), k
        assert abs(fd_tvar - res["grad_tvar"][k]) <= 1e-6 * max(1.0, abs(res["grad_tvar"][k])), k
