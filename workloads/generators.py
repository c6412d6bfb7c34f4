"""Seeded generators for Year Event Tables, Event Loss Tables and terms.

Shapes follow the paper's description of its inputs (Section IV-A): trials of
roughly 800-1500 time-ordered (event, timestamp) pairs (Eq. 1), direct-access
ELTs holding 10k-30k event losses each (Eq. 2), layers covering 3-30 ELTs
(Eq. 3).  The industrial data is not public; these draws stand in for it:

* trial lengths K_t ~ Poisson(lam);
* event IDs i.i.d. uniform over the catalogue [0, C);
* per ELT, `nnz` distinct catalogue positions drawn without replacement,
  losses ~ lognormal(mu=10, sigma=2), every other entry 0.0;
* per-ELT retention R = midpoint of the order statistics k, k+1 with
  k = ceil(0.20 n) of that ELT's losses, limit Lim = the same midpoint at 0.95;
* layer occurrence/aggregate terms are read from ``layer_terms.json``, a
  file of constants calibrated once from quantiles (see ``describe_recipe``).

Nothing here applies a financial term or sums a loss.

Every draw uses NumPy's PCG64 seeded from ``SEED_BASE + config index`` through
``SeedSequence.spawn``, in independent blocks, so a prefix of trials can be
generated without the rest and big tables are drawn on several threads with
identical results.
"""

from __future__ import annotations

import json
import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

SEED_BASE = 160604473
_TRIAL_BLOCK = 65536          # trials per independent id-drawing block
_TERMS_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "layer_terms.json")

CONFIG_NAMES = ("config0", "config1", "config2", "config3", "config4")


def _threads() -> int:
    n = os.cpu_count() or 1
    return max(1, min(16, n))


def _rng(seed_seq: np.random.SeedSequence) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed_seq))


# ---------------------------------------------------------------------------
# data classes
# ---------------------------------------------------------------------------

@dataclass
class YET:
    """Year Event Table in CSR form (Eq. 1).

    ``offsets[t] .. offsets[t+1]`` index trial t's events in ``ids``, stored
    in ascending time-stamp order.  ``offsets`` is int64 of length N+1,
    ``ids`` uint32.
    """

    offsets: np.ndarray
    ids: np.ndarray
    catalogue_size: int
    timestamps: Optional[np.ndarray] = None

    @property
    def n_trials(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def n_events(self) -> int:
        return int(self.ids.shape[0])

    def trial(self, t: int) -> np.ndarray:
        return self.ids[self.offsets[t]:self.offsets[t + 1]]


@dataclass
class ELTPool:
    """Dense direct-access ELTs: ``losses[j, E]`` is ELT j's loss for event E.

    Row-major float64 ``[n_elts, C]``; 0.0 marks an event absent from an ELT.
    ``retention[j]`` / ``limit[j]`` are the per-ELT financial terms.
    """

    losses: np.ndarray
    retention: np.ndarray
    limit: np.ndarray

    @property
    def n_elts(self) -> int:
        return int(self.losses.shape[0])

    @property
    def catalogue_size(self) -> int:
        return int(self.losses.shape[1])


@dataclass
class Layer:
    """A layer (Eq. 3): the ELTs it covers plus the four layer terms."""

    elt_index: np.ndarray                  # int32[J], rows of the pool, layer order
    occ_retention: float
    occ_limit: float
    agg_retention: float
    agg_limit: float
    trial_begin: int = 0
    trial_count: int = -1                  # -1: up to the end of the YET

    @property
    def n_elts(self) -> int:
        return int(self.elt_index.shape[0])

    def resolved_count(self, n_trials: int) -> int:
        return n_trials - self.trial_begin if self.trial_count < 0 else self.trial_count


@dataclass
class Workload:
    name: str
    yet: YET
    pool: ELTPool
    layers: List[Layer]
    probs: Sequence[float] = (0.99,)
    meta: dict = field(default_factory=dict)


# ---------------------------------------------------------------------------
# Year Event Table
# ---------------------------------------------------------------------------

def make_yet(n_trials: int, lam: float, catalogue_size: int, seed: int,
             n_prefix: Optional[int] = None, with_timestamps: bool = False) -> YET:
    """Draw a YET of ``n_trials`` trials, K_t ~ Poisson(lam), IDs uniform.

    ``n_prefix`` returns only the first trials; they are identical to the same
    trials of the full table.  Because the IDs of a trial are i.i.d., pairing
    them in draw order with independently drawn sorted time stamps gives the
    same joint law as sorting i.i.d. (event, time) pairs by time.
    """
    root = np.random.SeedSequence(seed)
    s_len, s_ids, s_ts = root.spawn(3)
    lengths = _rng(s_len).poisson(lam, size=n_trials).astype(np.int64)
    n_keep = n_trials if n_prefix is None else min(n_prefix, n_trials)
    offsets = np.zeros(n_keep + 1, dtype=np.int64)
    np.cumsum(lengths[:n_keep], out=offsets[1:])
    n_events = int(offsets[-1])
    ids = np.empty(n_events, dtype=np.uint32)
    n_blocks = (n_keep + _TRIAL_BLOCK - 1) // _TRIAL_BLOCK
    block_seeds = s_ids.spawn((n_trials + _TRIAL_BLOCK - 1) // _TRIAL_BLOCK)

    def fill(b: int) -> None:
        t0 = b * _TRIAL_BLOCK
        t1 = min(t0 + _TRIAL_BLOCK, n_keep)
        t1_full = min(t0 + _TRIAL_BLOCK, n_trials)
        lo = int(offsets[t0])
        # draw the whole block's events so a prefix equals the full table
        block_events = int(lengths[t0:t1_full].sum())
        draw = _rng(block_seeds[b]).integers(0, catalogue_size, size=block_events,
                                             dtype=np.uint32)
        hi = int(offsets[t1])
        ids[lo:hi] = draw[:hi - lo]

    if n_blocks <= 1:
        for b in range(n_blocks):
            fill(b)
    else:
        with ThreadPoolExecutor(_threads()) as ex:
            list(ex.map(fill, range(n_blocks)))
    yet = YET(offsets=offsets, ids=ids, catalogue_size=int(catalogue_size))
    if with_timestamps:
        yet.timestamps = make_timestamps(offsets, s_ts)
    return yet


def make_timestamps(offsets: np.ndarray, seed_seq) -> np.ndarray:
    """Sorted uniform float32 time stamps in [0, 365) within each trial."""
    if not isinstance(seed_seq, np.random.SeedSequence):
        seed_seq = np.random.SeedSequence(seed_seq)
    n_events = int(offsets[-1])
    ts = _rng(seed_seq).uniform(0.0, 365.0, size=n_events).astype(np.float32)
    ts = np.minimum(ts, np.float32(np.nextafter(np.float32(365.0), np.float32(0.0))))
    trial_of = np.repeat(np.arange(offsets.shape[0] - 1, dtype=np.int64), np.diff(offsets))
    order = np.lexsort((ts, trial_of))
    return ts[order]


def make_tiny_yet(trials: Sequence[Sequence[int]], catalogue_size: int) -> YET:
    """Build a YET from explicit lists of event IDs (hand-built cases)."""
    lengths = np.array([len(t) for t in trials], dtype=np.int64)
    offsets = np.zeros(len(trials) + 1, dtype=np.int64)
    np.cumsum(lengths, out=offsets[1:])
    ids = np.array([e for t in trials for e in t], dtype=np.uint32)
    return YET(offsets=offsets, ids=ids, catalogue_size=int(catalogue_size))


# ---------------------------------------------------------------------------
# Event Loss Tables and per-ELT terms
# ---------------------------------------------------------------------------

def elt_terms_from_losses(values: np.ndarray, r_q: float = 0.20, l_q: float = 0.95):
    """Per-ELT retention and limit from the ELT's own nonzero losses.

    Each is the midpoint of the order statistics k and k+1 (1-based) with
    k = ceil(q n), so no term sits exactly on a data point.  Percentages are
    handled in integer arithmetic to avoid ceil() of an inexact product.
    """
    v = np.sort(np.asarray(values, dtype=np.float64))
    n = v.shape[0]
    if n < 2:
        return 0.0, math.inf

    def mid(q: float) -> float:
        num = int(round(q * 1000))
        k = (num * n + 999) // 1000            # ceil(q n) for q on a 0.1% grid
        k = min(max(k, 1), n - 1)
        return float((v[k - 1] + v[k]) * 0.5)

    return mid(r_q), mid(l_q)


def make_elt_pool(n_elts: int, catalogue_size: int, nnz: int, seed: int,
                  mu: float = 10.0, sigma: float = 2.0) -> ELTPool:
    """Dense pool of ``n_elts`` ELTs, each with ``nnz`` lognormal losses."""
    root = np.random.SeedSequence(seed)
    kids = root.spawn(n_elts)
    losses = np.zeros((n_elts, catalogue_size), dtype=np.float64)
    retention = np.zeros(n_elts, dtype=np.float64)
    limit = np.zeros(n_elts, dtype=np.float64)

    def fill(j: int) -> None:
        rng = _rng(kids[j])
        pos = rng.choice(catalogue_size, size=nnz, replace=False)
        vals = rng.lognormal(mean=mu, sigma=sigma, size=nnz)
        losses[j, pos] = vals
        retention[j], limit[j] = elt_terms_from_losses(vals)

    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(fill, range(n_elts)))
    return ELTPool(losses=losses, retention=retention, limit=limit)


# ---------------------------------------------------------------------------
# Layer terms (constants calibrated once; see describe_recipe)
# ---------------------------------------------------------------------------

def load_layer_terms() -> dict:
    if not os.path.exists(_TERMS_FILE):
        return {}
    with open(_TERMS_FILE) as f:
        return json.load(f)


def _terms_or_placeholder(entry: Optional[dict]):
    if entry is None:
        return (0.0, math.inf, 0.0, math.inf)
    return (float(entry["occ_retention"]), float(entry["occ_limit"]),
            float(entry["agg_retention"]), float(entry["agg_limit"]))


def layer_library(n_layers: int, pool_size: int, n_trials: int, seed: int,
                  j_max: int = 32, n_min: int = 10_000, n_max: int = 1_000_000,
                  calibrated: bool = True) -> List[Layer]:
    """The batched-layer set: J ~ U{1..j_max} distinct pool ELTs per layer,
    n_l ~ U[n_min, n_max] trials starting at U[0, n_trials - n_l]."""
    rng = _rng(np.random.SeedSequence(seed).spawn(4)[3])
    terms = load_layer_terms().get("library", []) if calibrated else []
    layers = []
    n_max = min(n_max, n_trials)
    n_min = min(n_min, n_max)
    for i in range(n_layers):
        J = int(rng.integers(1, j_max + 1))
        idx = rng.choice(pool_size, size=J, replace=False).astype(np.int32)
        n_l = int(rng.integers(n_min, n_max + 1))
        begin = int(rng.integers(0, n_trials - n_l + 1))
        entry = terms[i] if i < len(terms) else None
        if entry is not None and list(entry["elt_index"]) != idx.tolist():
            raise RuntimeError("layer_terms.json does not match the layer draws")
        occ_r, occ_l, agg_r, agg_l = _terms_or_placeholder(entry)
        layers.append(Layer(idx, occ_r, occ_l, agg_r, agg_l, begin, n_l))
    return layers


# ---------------------------------------------------------------------------
# named configurations
# ---------------------------------------------------------------------------

_CFG = {
    "config0": dict(n_trials=10_000, lam=100.0, C=100_000, n_elts=4, nnz=10_000,
                    probs=(0.99,)),
    "config1": dict(n_trials=1_000_000, lam=1000.0, C=2_000_000, n_elts=16, nnz=20_000,
                    probs=(0.99, 0.996)),
    "config2": dict(n_trials=1_000_000, lam=1000.0, C=2_000_000, n_elts=256, nnz=20_000,
                    probs=(0.99,), n_layers=64),
}


def _seed_of(name: str) -> int:
    return SEED_BASE + int(name[-1])


def make_config(name: str, n_prefix: Optional[int] = None, calibrated: bool = True,
                with_timestamps: bool = False) -> Workload:
    """Build a named workload.

    config0  small: 1e4 trials x Poisson(100), C=1e5, 1 layer over 4 ELTs.
    config1  paper-scale one-GPU share: 1e6 x Poisson(1000), C=2e6, 16 ELTs.
    config2  64 layers over a 256-ELT pool and one shared YET.
    config3  config1's data (the adjoint runs on it).
    ``n_prefix`` keeps only the first trials (same values as the full table).
    """
    base = "config1" if name == "config3" else name
    base = "config2" if name == "config4" else base
    cfg = _CFG[base]
    seed = _seed_of(base)
    yet = make_yet(cfg["n_trials"], cfg["lam"], cfg["C"], seed, n_prefix=n_prefix,
                   with_timestamps=with_timestamps)
    pool = make_elt_pool(cfg["n_elts"], cfg["C"], cfg["nnz"], seed + 10_000)
    terms = load_layer_terms() if calibrated else {}
    if base == "config2":
        layers = layer_library(cfg["n_layers"], cfg["n_elts"], cfg["n_trials"], seed,
                               calibrated=calibrated)
        if n_prefix is not None:
            layers = [_clip_layer(l, yet.n_trials) for l in layers]
            layers = [l for l in layers if l.trial_count > 0]
    else:
        occ_r, occ_l, agg_r, agg_l = _terms_or_placeholder(terms.get(base))
        layers = [Layer(np.arange(cfg["n_elts"], dtype=np.int32), occ_r, occ_l, agg_r, agg_l,
                        0, yet.n_trials)]
    meta = dict(cfg)
    meta["seed"] = seed
    return Workload(name=name, yet=yet, pool=pool, layers=layers, probs=cfg["probs"], meta=meta)


def portfolio_programs(layers: Sequence[Layer], n_programs: int, trial_begin: int,
                       trial_count: int, seed: int) -> List[List[Layer]]:
    """Group ``layers`` in order into ``n_programs`` programs of at least one
    layer each (sizes from a seeded uniform split), every layer re-ranged to
    the portfolio's trials [trial_begin, trial_begin + trial_count)."""
    n = len(layers)
    if not 1 <= n_programs <= n:
        raise ValueError("need 1 <= n_programs <= number of layers")
    rng = _rng(np.random.SeedSequence(seed))
    cuts = np.sort(rng.choice(np.arange(1, n), size=n_programs - 1, replace=False)) if n_programs > 1 \
        else np.zeros(0, dtype=np.int64)
    bounds = [0, *[int(c) for c in cuts], n]
    ranged = [Layer(l.elt_index, l.occ_retention, l.occ_limit, l.agg_retention, l.agg_limit,
                    trial_begin, trial_count) for l in layers]
    return [ranged[bounds[p]:bounds[p + 1]] for p in range(n_programs)]


def _clip_layer(layer: Layer, n_trials: int) -> Layer:
    begin = min(layer.trial_begin, n_trials)
    count = max(0, min(layer.trial_begin + layer.trial_count, n_trials) - begin)
    return Layer(layer.elt_index, layer.occ_retention, layer.occ_limit,
                 layer.agg_retention, layer.agg_limit, begin, count)


def describe_recipe() -> str:
    return (
        "YET: K_t ~ Poisson(lam), IDs uniform on [0,C) (PCG64, seed 160604473+config); "
        "ELT: nnz distinct positions, lognormal(10,2) losses, dense rows; "
        "per-ELT R/Lim: midpoints of the 20th/95th-percentile order statistics; "
        "layer OccR = q10 of the nonzero ELT-combined losses over the catalogue, "
        "OccL = q99 - OccR; AggR = q50 of the annual loss S over a trial sample, "
        "AggL = q99.9 - AggR (constants in workloads/layer_terms.json)."
    )
