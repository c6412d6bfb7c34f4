"""Python face of the CPU oracle -- TEST INFRASTRUCTURE ONLY.

Three independent renderings of the same definition (Algorithm 3 with the
term definitions of Section IV-B) live here:

* ``run_layer``        -- the C oracle (ara_oracle.c), literal loop nest;
* ``run_layer_python`` -- pure-Python loops with math.fsum, for tiny cases;
* ``run_layer_numpy``  -- NumPy elementwise ops over the catalogue, then a
  per-trial sum; a second formulation written independently of the C code.

The risk metrics (Section IV-A names PML and TVaR without defining them)
follow the return-period reading: m = ceil(N (1 - p)) with p read as the
decimal it was written as; PML_p is the m-th largest year loss; TVaR_p is the
mean of the m largest.
"""

from __future__ import annotations

import ctypes
import math
import os
from fractions import Fraction
from typing import List, Sequence, Tuple

import numpy as np

from . import build as _build

SUM_SEQUENTIAL = 0
SUM_EXACT = 1
_MODES = {"sequential": SUM_SEQUENTIAL, "exact": SUM_EXACT}

_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        lib.ara_oracle_run_layer.argtypes = [P, i64, P, i64, P, i32, i64, i32, P, P, P,
                                             f64, f64, f64, f64, i64, i64, i32, P, P, i32]
        lib.ara_oracle_run_layer.restype = i32
        lib.ara_oracle_occurrence_catalogue.argtypes = [P, i32, i64, i32, P, P, P, f64, f64,
                                                        P, P]
        lib.ara_oracle_occurrence_catalogue.restype = i32
        lib.ara_oracle_grad_counts.argtypes = [P, i64, P, i64, P, i32, i64, i32, P, P, P,
                                               f64, f64, f64, f64, i64, i64, P, P, i32]
        lib.ara_oracle_grad_counts.restype = i32
        lib.ara_oracle_event_nets.argtypes = [P, i64, P, i64, P, i32, i64, i32, P, P, P,
                                              f64, f64, f64, f64, i64, i64, P, i32]
        lib.ara_oracle_event_nets.restype = i32
        lib.ara_oracle_exact_sum.argtypes = [P, i64]
        lib.ara_oracle_exact_sum.restype = f64
        lib.ara_oracle_max_threads.argtypes = []
        lib.ara_oracle_max_threads.restype = i32
        _LIB = lib
    return _LIB


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def max_threads() -> int:
    return int(_lib().ara_oracle_max_threads())


def exact_sum(x: np.ndarray) -> float:
    """Sum of doubles rounded once (C oracle's exact accumulator).

    Pinned by: equality with math.fsum on random and adversarial inputs."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    return float(_lib().ara_oracle_exact_sum(_ptr(x), x.shape[0]))


def _layer_arrays(pool, layer):
    idx = np.ascontiguousarray(layer.elt_index, dtype=np.int32)
    R = np.ascontiguousarray(pool.retention[idx], dtype=np.float64)
    Lim = np.ascontiguousarray(pool.limit[idx], dtype=np.float64)
    return idx, R, Lim


def _range(yet, layer) -> Tuple[int, int]:
    begin = int(layer.trial_begin)
    count = int(layer.resolved_count(yet.n_trials))
    return begin, count


# ---------------------------------------------------------------------------
# year losses
# ---------------------------------------------------------------------------

def run_layer(yet, pool, layer, sum_mode: str = "exact", threads: int = 0):
    """Year losses of ``layer`` over its trial range (Algorithm 3), via the C oracle.

    Returns (ylt, S): the year losses and the pre-aggregate annual totals.
    Pinned by: the closed-form cases of tests/golden/closed_form_cases.json,
    the invariants (bounds, monotonicity, 2^k homogeneity, split invariance),
    agreement with run_layer_python and run_layer_numpy, and the sparse
    matrix-vector reduction when all retentions are 0 and limits infinite.
    """
    lib = _lib()
    offsets = np.ascontiguousarray(yet.offsets, dtype=np.int64)
    ids = np.ascontiguousarray(yet.ids, dtype=np.uint32)
    elts = np.ascontiguousarray(pool.losses, dtype=np.float64)
    idx, R, Lim = _layer_arrays(pool, layer)
    begin, count = _range(yet, layer)
    ylt = np.empty(count, dtype=np.float64)
    S = np.empty(count, dtype=np.float64)
    rc = lib.ara_oracle_run_layer(_ptr(offsets), yet.n_trials, _ptr(ids), ids.shape[0],
                                  _ptr(elts), elts.shape[0], elts.shape[1],
                                  idx.shape[0], _ptr(idx), _ptr(R), _ptr(Lim),
                                  layer.occ_retention, layer.occ_limit,
                                  layer.agg_retention, layer.agg_limit,
                                  begin, count, _MODES[sum_mode], _ptr(ylt), _ptr(S), threads)
    if rc != 0:
        raise ValueError(f"oracle rejected the input (code {rc})")
    return ylt, S


def portfolio(yet, pool, programs, threads: int = 0):
    """Year losses of a portfolio (Algorithm 1's loops over programs and their
    layers, Section IV-A), computed without any split of the YET.

    ``programs`` is a list of programs, each a list of layers over the same
    trials.  Returns (layer_ylt [n_layers][n], program_ylt [n_programs][n],
    portfolio_ylt [n]).  The paper gives no rule for combining layers; a
    program's year loss is taken as the per-trial sum of its layers' year
    losses and the portfolio's as the sum over all of its layers, each sum
    exact and rounded once (math.fsum).  Pinned by: the hand-worked portfolio
    of tests/golden/closed_form_cases.json, a case where only a once-rounded
    sum is right, and the one-layer reduction to run_layer.
    """
    layers = [layer for prog in programs for layer in prog]
    if not programs or any(len(prog) == 0 for prog in programs):
        raise ValueError("every program needs at least one layer")
    ranges = {_range(yet, layer) for layer in layers}
    if len(ranges) != 1:
        raise ValueError("the layers of a portfolio must cover the same trials")
    rows = np.stack([run_layer(yet, pool, layer, threads=threads)[0] for layer in layers])
    n = rows.shape[1]
    program_rows = np.empty((len(programs), n))
    first = 0
    for p, prog in enumerate(programs):
        block = rows[first:first + len(prog)]
        program_rows[p] = [math.fsum(block[:, k].tolist()) for k in range(n)]
        first += len(prog)
    portfolio_row = np.array([math.fsum(rows[:, k].tolist()) for k in range(n)])
    return rows, program_rows, portfolio_row


def event_nets(yet, pool, layer, threads: int = 0) -> np.ndarray:
    """Per-event net losses of ``layer`` (Section IV-B: the aggregate terms act
    on the trial's cumulative loss), via the C oracle.

    For the d-th event of a trial, A_d = clamp(S_d; AggR, AggL) with S_d the
    exact running total of the occurrence losses rounded once, and the event's
    net is A_d - A_{d-1} (A_0 = clamp(0; AggR, AggL)).  Entry i belongs to
    event offsets[trial_begin] + i.  Pinned by: the hand-worked nets of
    tests/golden/closed_form_cases.json, event_nets_python on every tiny
    trial, and the invariants (nets >= 0, each net at most its occurrence
    loss, the nets of a trial telescoping to its year loss minus A_0).
    """
    lib = _lib()
    offsets = np.ascontiguousarray(yet.offsets, dtype=np.int64)
    ids = np.ascontiguousarray(yet.ids, dtype=np.uint32)
    elts = np.ascontiguousarray(pool.losses, dtype=np.float64)
    idx, R, Lim = _layer_arrays(pool, layer)
    begin, count = _range(yet, layer)
    nets = np.empty(int(offsets[begin + count] - offsets[begin]), dtype=np.float64)
    rc = lib.ara_oracle_event_nets(_ptr(offsets), yet.n_trials, _ptr(ids), ids.shape[0],
                                   _ptr(elts), elts.shape[0], elts.shape[1],
                                   idx.shape[0], _ptr(idx), _ptr(R), _ptr(Lim),
                                   layer.occ_retention, layer.occ_limit,
                                   layer.agg_retention, layer.agg_limit,
                                   begin, count, _ptr(nets), threads)
    if rc != 0:
        raise ValueError(f"oracle rejected the input (code {rc})")
    return nets


def event_nets_python(trials: Sequence[Sequence[int]], losses, elt_index, R, Lim,
                      occ_r, occ_l, agg_r, agg_l) -> List[float]:
    """Per-event nets in plain Python: every prefix total recomputed from
    scratch with math.fsum, for tiny cases."""
    out = []
    a0 = _terms(0.0, agg_r, agg_l)
    for trial in trials:
        occ = []
        a_prev = a0
        for e in trial:
            y = 0.0
            for j, row in enumerate(elt_index):
                y = y + _terms(float(losses[row][e]), float(R[j]), float(Lim[j]))
            occ.append(_terms(y, occ_r, occ_l))
            a = _terms(math.fsum(occ), agg_r, agg_l)
            out.append(a - a_prev)
            a_prev = a
    return out


def _terms(v: float, r: float, lim: float) -> float:
    t = v - r
    if not (t > 0.0):
        t = 0.0
    if t > lim:
        t = lim
    return t


def run_layer_python(trials: Sequence[Sequence[int]], losses, elt_index, R, Lim,
                     occ_r, occ_l, agg_r, agg_l, sum_mode: str = "exact"):
    """Algorithm 3 in plain Python floats, for hand-built and brute-force cases."""
    ylt, S_all = [], []
    for trial in trials:
        occ = []
        for e in trial:
            y = 0.0
            for j, row in enumerate(elt_index):
                y = y + _terms(float(losses[row][e]), float(R[j]), float(Lim[j]))
            occ.append(_terms(y, occ_r, occ_l))
        if sum_mode == "exact":
            S = math.fsum(occ)
        else:
            S = 0.0
            for o in occ:
                S = S + o
        S_all.append(S)
        ylt.append(_terms(S, agg_r, agg_l))
    return ylt, S_all


def run_layer_numpy(yet, pool, layer):
    """Second formulation: occurrence-net loss for every catalogue event with
    NumPy elementwise ops (same operations, same ELT order), then each trial's
    total as math.fsum over its events.  For small tables only."""
    idx, R, Lim = _layer_arrays(pool, layer)
    y = np.zeros(pool.catalogue_size, dtype=np.float64)
    for j, row in enumerate(idx):
        x = pool.losses[row] - R[j]
        x = np.where(x > 0.0, x, 0.0)
        x = np.where(x > Lim[j], Lim[j], x)
        y = y + x
    o = y - layer.occ_retention
    o = np.where(o > 0.0, o, 0.0)
    o = np.where(o > layer.occ_limit, layer.occ_limit, o)
    begin, count = _range(yet, layer)
    S = np.empty(count, dtype=np.float64)
    for k in range(count):
        t = begin + k
        S[k] = math.fsum(o[yet.ids[yet.offsets[t]:yet.offsets[t + 1]]].tolist())
    t = S - layer.agg_retention
    t = np.where(t > 0.0, t, 0.0)
    ylt = np.where(t > layer.agg_limit, layer.agg_limit, t)
    return ylt, S, y, o


def occurrence_catalogue(pool, layer):
    """(y, o) for every catalogue event E: ELT-combined net loss and the
    occurrence-net loss.  Pinned by: agreement with run_layer_numpy's
    elementwise arrays and the closed-form cases."""
    lib = _lib()
    elts = np.ascontiguousarray(pool.losses, dtype=np.float64)
    idx, R, Lim = _layer_arrays(pool, layer)
    C = elts.shape[1]
    y = np.empty(C, dtype=np.float64)
    o = np.empty(C, dtype=np.float64)
    rc = lib.ara_oracle_occurrence_catalogue(_ptr(elts), elts.shape[0], C, idx.shape[0],
                                             _ptr(idx), _ptr(R), _ptr(Lim),
                                             layer.occ_retention, layer.occ_limit,
                                             _ptr(y), _ptr(o))
    if rc != 0:
        raise ValueError(f"oracle rejected the layer (code {rc})")
    return y, o


def lookups(yet, pool, layer, trial: int):
    """Event IDs of a trial in storage (time) order and the raw ELT losses
    looked up for them: losses[k][j] = ELT_{elt_index[j]}[ids[k]] (direct
    access, Section IV-B), shape [K][J].  Pinned by the golden tables (ids
    and losses of hand-built trials, written out by hand)."""
    ids = np.asarray(yet.trial(trial), dtype=np.uint32)
    idx = np.asarray(layer.elt_index, dtype=np.int64)
    losses = pool.losses[idx][:, ids.astype(np.int64)].T.copy()
    return ids.copy(), losses


# ---------------------------------------------------------------------------
# risk metrics
# ---------------------------------------------------------------------------

def tail_count(n: int, p: float) -> int:
    """m = ceil(n (1 - p)) with p taken as the decimal it was written as
    (its shortest round-trip representation, repr), in exact rational
    arithmetic, clamped to [1, n].

    Pinned by hand values: N=1e6 gives m=10000 at 0.99 and 4000 at 0.996
    (where the FP64 product would give 10001), 10001 at 0.989999999999 (where
    snapping to the nearest integer would give 10000), 3 for N=3 at 1/3 and
    2 at 2/3 (their repr digits leave a remainder above the integer)."""
    if not (0.0 < p < 1.0):
        raise ValueError("p must lie in (0, 1)")
    if n < 1:
        raise ValueError("need at least one trial")
    q = Fraction(repr(float(p)))
    m = math.ceil(n * (1 - q))
    return int(min(max(m, 1), n))


def risk_metrics(ylt: np.ndarray, probs: Sequence[float]):
    """Mean annual loss, PML_p and TVaR_p by sorting the year losses.

    Returns (mean, [pml], [tvar]).  Pinned by: permutations of 1..N
    (PML = N - m + 1, TVaR = N - (m - 1)/2) and the closed-form Case C values.
    """
    y = np.asarray(ylt, dtype=np.float64)
    n = y.shape[0]
    mean = math.fsum(y.tolist()) / n
    desc = np.sort(y)[::-1]
    pml, tvar = [], []
    for p in probs:
        m = tail_count(n, p)
        pml.append(float(desc[m - 1]))
        tvar.append(math.fsum(desc[:m].tolist()) / m)
    return mean, pml, tvar


# ---------------------------------------------------------------------------
# gradients
# ---------------------------------------------------------------------------

def grad_counts(yet, pool, layer, S: np.ndarray, threads: int = 0) -> np.ndarray:
    """Per-trial integer derivative vectors of the year loss, int32
    [trial_count][2J+4] over theta = [R_1..R_J, Lim_1..Lim_J, OccR, OccL,
    AggR, AggL] (strict-subgradient convention at kinks)."""
    lib = _lib()
    offsets = np.ascontiguousarray(yet.offsets, dtype=np.int64)
    ids = np.ascontiguousarray(yet.ids, dtype=np.uint32)
    elts = np.ascontiguousarray(pool.losses, dtype=np.float64)
    idx, R, Lim = _layer_arrays(pool, layer)
    begin, count = _range(yet, layer)
    S = np.ascontiguousarray(S, dtype=np.float64)
    J = idx.shape[0]
    counts = np.empty((count, 2 * J + 4), dtype=np.int32)
    rc = lib.ara_oracle_grad_counts(_ptr(offsets), yet.n_trials, _ptr(ids), ids.shape[0],
                                    _ptr(elts), elts.shape[0], elts.shape[1], J,
                                    _ptr(idx), _ptr(R), _ptr(Lim),
                                    layer.occ_retention, layer.occ_limit,
                                    layer.agg_retention, layer.agg_limit,
                                    begin, count, _ptr(S), _ptr(counts), threads)
    if rc != 0:
        raise ValueError(f"oracle rejected the input (code {rc})")
    return counts


def gradients(yet, pool, layer, tvar_p: float, ylt=None, S=None, threads: int = 0):
    """Gradients of the mean annual loss and of TVaR_p over theta.

    mean: sum over trials of the integer vectors, divided by N.
    TVaR: the m largest year losses; trials strictly above the m-th largest
    value v weigh 1, trials equal to v share the remaining m - c_gt slots
    equally (weight (m - c_gt)/c_eq); the weighted sum is an integer over
    m * c_eq.  Returns dict with float gradients and the exact integer
    numerators/denominators.
    """
    if ylt is None or S is None:
        ylt, S = run_layer(yet, pool, layer, threads=threads)
    counts = grad_counts(yet, pool, layer, S, threads=threads).astype(np.int64)
    n = ylt.shape[0]
    num_mean = counts.sum(axis=0)
    m = tail_count(n, tvar_p)
    v = float(np.sort(ylt)[::-1][m - 1])
    gt = ylt > v
    eq = ylt == v
    c_gt = int(gt.sum())
    c_eq = int(eq.sum())
    num_tvar = c_eq * counts[gt].sum(axis=0) + (m - c_gt) * counts[eq].sum(axis=0)
    den_tvar = m * c_eq
    grad_mean = num_mean.astype(np.float64) / float(n)
    grad_tvar = num_tvar.astype(np.float64) / float(den_tvar)
    return dict(grad_mean=grad_mean, grad_tvar=grad_tvar, num_mean=num_mean, den_mean=n,
                num_tvar=num_tvar, den_tvar=den_tvar, m=m, threshold=v, c_gt=c_gt, c_eq=c_eq)
