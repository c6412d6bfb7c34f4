"""Multi-tenant request loop on one GPU.

The paper runs several clients ("tenants") on virtual GPUs mapped onto one
physical GPU, so that one tenant's host-to-device transfer overlaps another's
kernel, and compares two transfer modes (Section V-D): *concurrent* (every
device receives its data at once, sharing the link) and *sequential* (one
transfer at a time at full link bandwidth while others compute).  Here a
tenant is a worker thread with its own HIP stream; tenants share one GPU, the
resident ELT pool and, in "resident" mode, the resident YET.

Each request is an analysis: a slice of trials of the YET and 1-16 layers.
Shipped modes copy the slice to the device (Algorithm 2) -- concurrently or
under a FIFO transfer token -- and build tables for it that share the
resident ELT pool (ara_create_yet); resident mode runs the layers on trial
ranges of the resident YET.  Admission is by device memory: a request waits
(FIFO) until its footprint fits the budget, then runs as soon as its tenant is
free, overlapping with the other tenants' work (continuous batching: requests
are admitted as slots and memory free up, not in fixed batches).  Results
carry arrival, admission, start and finish times; latency is finish minus
arrival.
"""

from __future__ import annotations

import math
import threading
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import numpy as np

MODES = ("concurrent", "sequential", "resident")


# ---------------------------------------------------------------------------
# admission by device memory (no GPU needed)
# ---------------------------------------------------------------------------

class AdmissionController:
    """FIFO admission against a byte budget.

    acquire(n) blocks until every earlier waiter has been admitted and
    used + n <= budget; a request larger than the whole budget is refused
    (returns False) instead of waiting forever.
    """

    def __init__(self, budget_bytes: int):
        self.budget = int(budget_bytes)
        self.used = 0
        self.peak = 0
        self._cv = threading.Condition()
        self._queue: deque = deque()
        self.waits: List[float] = []

    def acquire(self, nbytes: int, timeout: Optional[float] = None) -> bool:
        nbytes = int(nbytes)
        if nbytes > self.budget:
            return False
        t0 = time.perf_counter()
        me = object()
        with self._cv:
            self._queue.append(me)
            deadline = None if timeout is None else t0 + timeout
            while not (self._queue[0] is me and self.used + nbytes <= self.budget):
                remaining = None if deadline is None else deadline - time.perf_counter()
                if remaining is not None and remaining <= 0:
                    self._queue.remove(me)
                    self._cv.notify_all()
                    return False
                self._cv.wait(remaining)
            self._queue.popleft()
            self.used += nbytes
            self.peak = max(self.peak, self.used)
            self.waits.append(time.perf_counter() - t0)
            self._cv.notify_all()
        return True

    def release(self, nbytes: int) -> None:
        with self._cv:
            self.used -= int(nbytes)
            assert self.used >= 0
            self._cv.notify_all()


# ---------------------------------------------------------------------------
# requests
# ---------------------------------------------------------------------------

@dataclass
class Request:
    rid: int
    tenant: int
    arrival: float              # seconds after the start of the run
    trial_begin: int
    n_trials: int
    layer_ids: List[int]


@dataclass
class Result:
    rid: int
    tenant: int
    arrival: float
    admitted: float = math.nan
    started: float = math.nan
    finished: float = math.nan
    footprint: int = 0
    metrics: List[List[float]] = field(default_factory=list)   # per layer [mean, pml.., tvar..]
    error: Optional[str] = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def make_requests(n_tenants: int, per_tenant: int, rate_per_tenant: float, n_yet_trials: int,
                  n_library: int, seed: int, n_min: int = 10_000, n_max: int = 1_000_000,
                  layers_max: int = 16) -> List[Request]:
    """Poisson arrivals per tenant (seed + 1000 * tenant), n ~ log-uniform
    [n_min, n_max] trials at a uniform offset, 1..layers_max layers drawn
    without replacement from the layer library."""
    reqs: List[Request] = []
    n_max = min(n_max, n_yet_trials)
    n_min = min(n_min, n_max)
    rid = 0
    for k in range(n_tenants):
        rng = np.random.Generator(np.random.PCG64(seed + 1000 * k))
        t = 0.0
        for _ in range(per_tenant):
            t += float(rng.exponential(1.0 / rate_per_tenant)) if rate_per_tenant > 0 else 0.0
            n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
            n = min(max(n, 1), n_yet_trials)
            begin = int(rng.integers(0, n_yet_trials - n + 1))
            nl = int(rng.integers(1, layers_max + 1))
            lids = rng.choice(n_library, size=min(nl, n_library), replace=False).tolist()
            reqs.append(Request(rid, k, t, begin, n, lids))
            rid += 1
    reqs.sort(key=lambda r: (r.arrival, r.rid))
    return reqs


def percentile(x: Sequence[float], q: float) -> float:
    a = np.sort(np.asarray(x, dtype=np.float64))
    if a.shape[0] == 0:
        return math.nan
    k = max(0, min(a.shape[0] - 1, int(math.ceil(q / 100.0 * a.shape[0])) - 1))
    return float(a[k])


def summarize(results: Sequence[Result], wall: float) -> Dict[str, float]:
    ok = [r for r in results if r.error is None]
    lat = [r.latency for r in ok]
    return {
        "requests": len(results),
        "completed": len(ok),
        "rejected": len(results) - len(ok),
        "wall_s": wall,
        "throughput_req_s": len(ok) / wall if wall > 0 else math.nan,
        "p50_ms": percentile(lat, 50) * 1e3,
        "p99_ms": percentile(lat, 99) * 1e3,
        "mean_ms": float(np.mean(lat)) * 1e3 if lat else math.nan,
    }


# ---------------------------------------------------------------------------
# the GPU server
# ---------------------------------------------------------------------------

def pin_ids(ids: np.ndarray):
    """Event IDs in pinned host memory (as int32 bit patterns), the source of
    every shipped request slice."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(ids, dtype=np.uint32).view(np.int32)).pin_memory()


class Server:
    """Runs requests for n_tenants tenants on one GPU.

    base:     resident tables (ELT pool and, for resident mode, the YET);
    offsets, ids: the host YET the requests slice (ids pinned by the server);
    library:  LayerSpec list (trial ranges are replaced per request);
    probs:    risk-metric probabilities reported per layer.
    """

    def __init__(self, base, offsets: np.ndarray, ids: np.ndarray, library, n_tenants: int,
                 mode: str, budget_bytes: int, probs=(0.99,), pinned_ids=None):
        import torch
        from . import ara
        if mode not in MODES:
            raise ValueError(mode)
        self.torch = torch
        self.ara = ara
        self.base = base
        self.offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        self.library = list(library)
        self.n_tenants = n_tenants
        self.mode = mode
        self.probs = list(probs)
        self.admission = AdmissionController(budget_bytes)
        self.transfer_token = threading.Lock()
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.streams = [torch.cuda.Stream() for _ in range(n_tenants)]
        self.host_ids = pinned_ids
        if mode != "resident" and self.host_ids is None:
            self.host_ids = pin_ids(ids)

    def footprint(self, req: Request) -> int:
        n_ev = int(self.offsets[req.trial_begin + req.n_trials] - self.offsets[req.trial_begin])
        out = 8 * req.n_trials * len(req.layer_ids) + 8 * (1 + 2 * len(self.probs)) * len(req.layer_ids)
        scratch = 8 * self.base.catalogue_size * 2 + 8 * 1024 * 1024   # occurrence losses, images, compact
        if self.mode == "resident":
            return out + scratch
        yet = 4 * n_ev + 8 * (req.n_trials + 1)
        # staging copy + owned copy + partitioned copy (~ the IDs again, padded)
        return 2 * yet + 5 * n_ev + 16 * req.n_trials + out + scratch

    def _layers_for(self, req: Request, begin: int):
        specs = []
        for lid in req.layer_ids:
            s = self.library[lid]
            specs.append(self.ara.LayerSpec(s.elt_index, s.elt_retention, s.elt_limit, s.occ_retention,
                                            s.occ_limit, s.agg_retention, s.agg_limit, begin, req.n_trials))
        return specs

    def _serve_one(self, req: Request, res: Result, t0: float) -> None:
        torch, ara = self.torch, self.ara
        stream = self.streams[req.tenant]
        nb = self.footprint(req)
        res.footprint = nb
        if not self.admission.acquire(nb):
            res.error = "footprint exceeds the device-memory budget"
            res.finished = time.perf_counter() - t0
            return
        res.admitted = time.perf_counter() - t0
        tables = None
        try:
            with torch.cuda.stream(stream):
                res.started = time.perf_counter() - t0
                if self.mode == "resident":
                    tables, begin = self.base, req.trial_begin
                else:
                    lo = int(self.offsets[req.trial_begin])
                    hi = int(self.offsets[req.trial_begin + req.n_trials])
                    off = torch.from_numpy(self.offsets[req.trial_begin:req.trial_begin + req.n_trials + 1] - lo)
                    off = off.pin_memory()
                    d_ids = torch.empty(hi - lo, dtype=torch.int32, device=self.device)
                    d_off = torch.empty(req.n_trials + 1, dtype=torch.int64, device=self.device)
                    if self.mode == "sequential":
                        with self.transfer_token:
                            d_ids.copy_(self.host_ids[lo:hi], non_blocking=True)
                            d_off.copy_(off, non_blocking=True)
                            stream.synchronize()
                    else:
                        d_ids.copy_(self.host_ids[lo:hi], non_blocking=True)
                        d_off.copy_(off, non_blocking=True)
                    tables = ara.create_yet(self.base, d_off, d_ids, stream=stream)
                    del d_ids, d_off
                    begin = 0
                specs = self._layers_for(req, begin)
                k = len(self.probs)
                ylt = torch.empty(req.n_trials, dtype=torch.float64, device=self.device)
                out = torch.empty((len(specs), 1 + 2 * k), dtype=torch.float64, device=self.device)
                for i, s in enumerate(specs):
                    ara.run_layers(tables, [s], out=ylt, stream=stream)
                    ara.risk_metrics(ylt, self.probs, outputs=out[i], stream=stream)
                host = out.cpu()              # waits for this tenant's stream only
                res.metrics = host.numpy().tolist()
        except Exception as exc:              # a poisoned request fails alone
            res.error = f"{type(exc).__name__}: {exc}"
        finally:
            if tables is not None and tables is not self.base:
                tables.close()
            res.finished = time.perf_counter() - t0
            self.admission.release(nb)

    def run(self, requests: Sequence[Request], time_scale: float = 1.0) -> List[Result]:
        """Serve `requests` (arrival times scaled by time_scale).  One worker
        per tenant takes that tenant's requests in arrival order."""
        per_tenant: Dict[int, List[Request]] = {k: [] for k in range(self.n_tenants)}
        for r in requests:
            per_tenant[r.tenant % self.n_tenants].append(r)
        results = {r.rid: Result(r.rid, r.tenant, r.arrival * time_scale) for r in requests}
        t0 = time.perf_counter()

        def worker(k: int) -> None:
            for r in per_tenant[k]:
                wait = r.arrival * time_scale - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(wait)
                rr = Request(r.rid, k, r.arrival, r.trial_begin, r.n_trials, r.layer_ids)
                self._serve_one(rr, results[r.rid], t0)

        threads = [threading.Thread(target=worker, args=(k,)) for k in range(self.n_tenants)]
        for th in threads:
            th.start()
        for th in threads:
            th.join()
        self.torch.cuda.synchronize()
        self.wall = time.perf_counter() - t0
        return [results[r.rid] for r in requests]


def run_tenant_study(base, offsets, ids, library, n_tenants: int = 8, per_tenant: int = 6,
                     seed: int = 160604478, budget_bytes: int = 160 << 30, probs=(0.99,),
                     load: float = 0.7, modes: Sequence[str] = ("concurrent", "sequential", "resident"),
                     log=None) -> Dict[str, object]:
    """Config-4 study: requests with Poisson arrivals at `load` times the
    single-tenant capacity, served by n_tenants tenants in each transfer mode
    and by one tenant; p50/p99 latency and throughput for each."""
    n_yet = int(offsets.shape[0] - 1)
    pinned = pin_ids(ids)
    # capacity: one tenant, requests back to back, shipped concurrently
    probe = make_requests(1, 6, 0.0, n_yet, len(library), seed=seed + 77)
    for r in probe:
        r.arrival = 0.0
    srv = Server(base, offsets, ids, library, 1, "concurrent", budget_bytes, probs, pinned)
    srv.run(probe[:1], 0.0)                                   # warm-up
    res = srv.run(probe, 0.0)
    service = srv.wall / max(len(res), 1)
    rate_total = load / service
    reqs = make_requests(n_tenants, per_tenant, rate_total / n_tenants, n_yet, len(library), seed=seed)
    out: Dict[str, object] = {"service_ms_one_tenant": service * 1e3, "arrival_rate_req_s": rate_total,
                              "load": load, "tenants": n_tenants, "requests": len(reqs)}
    for mode in modes:
        for k in (1, n_tenants):
            s = Server(base, offsets, ids, library, k, mode, budget_bytes, probs, pinned)
            r = s.run(reqs, 1.0)
            summ = summarize(r, s.wall)
            summ["admission_peak_bytes"] = s.admission.peak
            out[f"{mode}_{k}t"] = summ
            if log:
                log(f"serving {mode} tenants={k}: p50 {summ['p50_ms']:.1f} ms p99 {summ['p99_ms']:.1f} ms "
                    f"{summ['throughput_req_s']:.2f} req/s")
    return out


# ---------------------------------------------------------------------------
# one analysis split over v tenants: measured time and energy beside the
# deployment model of Section V-F (Eqs. 4-10), fitted on one tenant
# ---------------------------------------------------------------------------

class PowerSampler:
    """Samples the GPU's socket power (W) and graphics activity (%) every
    `period` seconds through amdsmi (read-only queries), in a thread.  If
    amdsmi is unavailable the sampler records nothing and reports None."""

    def __init__(self, device_index: int = 0, period: float = 0.05):
        self.period = period
        self.samples: List[tuple] = []
        self._stop = threading.Event()
        self._thread = None
        self._h = None
        try:
            import amdsmi
            amdsmi.amdsmi_init()
            self._smi = amdsmi
            self._h = amdsmi.amdsmi_get_processor_handles()[device_index]
            self.read()
        except Exception:            # no library, no permission, or no such query on this driver
            self._h = None

    @property
    def available(self) -> bool:
        return self._h is not None

    def read(self):
        p = self._smi.amdsmi_get_power_info(self._h)
        w = p.get("current_socket_power", p.get("average_socket_power"))
        try:
            act = self._smi.amdsmi_get_gpu_activity(self._h).get("gfx_activity")
        except Exception:
            act = None
        return float(w), (float(act) if isinstance(act, (int, float)) else None)

    def _run(self) -> None:
        while not self._stop.is_set():
            try:
                w, a = self.read()
                self.samples.append((time.perf_counter(), w, a))
            except Exception:
                pass
            self._stop.wait(self.period)

    def __enter__(self):
        self.samples = []
        if self.available:
            self._stop.clear()
            self._thread = threading.Thread(target=self._run, daemon=True)
            self._thread.start()
        return self

    def __exit__(self, *exc):
        if self._thread is not None:
            self._stop.set()
            self._thread.join()
            self._thread = None
        return False

    def summary(self) -> Optional[Dict[str, float]]:
        """Energy (J, trapezoid over the samples), mean power (W) and mean
        graphics activity (%) of the last sampled interval."""
        s = self.samples
        if len(s) < 2:
            return None
        e = sum(0.5 * (s[i][1] + s[i + 1][1]) * (s[i + 1][0] - s[i][0]) for i in range(len(s) - 1))
        dt = s[-1][0] - s[0][0]
        acts = [a for _, _, a in s if a is not None]
        return {"energy_j": e, "mean_power_w": e / dt if dt > 0 else float("nan"),
                "mean_gfx_activity_pct": (sum(acts) / len(acts)) if acts else None, "samples": len(s)}


def split_ranges(n: int, v: int) -> List[tuple]:
    """v contiguous trial ranges covering [0, n), sizes differing by at most one."""
    q, r = divmod(n, v)
    out, b = [], 0
    for k in range(v):
        c = q + (1 if k < r else 0)
        out.append((b, c))
        b += c
    return out


def fit_split_model(transfer_s: float, compute_s: float, fixed_s: float, w_idle: float, w_busy: float):
    """Eqs. 4-10 on one physical GPU with v tenants: T_transfer(v) = v
    fixed_s + transfer_s (the YET is split, the per-tenant costs are not),
    T_comp(v) = compute_s / v, time = max(Eq. 7, Eq. 8), energy by Eq. 10 with
    the measured idle and busy power."""
    from .perf_model import Platform
    return Platform(compute_s, fixed_s, 0.0, 0.0, 0.0, transfer_s, w_idle=w_idle, w_compute=w_busy)


def split_study(base, offsets, pinned_ids, library, layer_ids: Sequence[int], tenants=(1, 2, 4, 8),
                modes=("concurrent", "sequential"), probs=(0.99,), repeats: int = 2, log=None) -> Dict[str, object]:
    """The whole YET analysed with `layer_ids`, split over v tenants on one
    GPU (each ships its slice, builds its tables, runs the layers and the
    metrics), for each transfer mode; wall time, energy and activity per
    (mode, v), and the model's prediction from single-tenant components."""
    import torch
    from . import ara
    from .perf_model import Platform   # noqa: F401  (documents the dependency)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    n = int(offsets.shape[0] - 1)
    dev = torch.device("cuda", torch.cuda.current_device())
    sampler = PowerSampler(torch.cuda.current_device())

    def specs_for(begin: int, count: int):
        out = []
        for lid in layer_ids:
            s = library[lid]
            out.append(ara.LayerSpec(s.elt_index, s.elt_retention, s.elt_limit, s.occ_retention, s.occ_limit,
                                     s.agg_retention, s.agg_limit, begin, count))
        return out

    def ship(lo_t: int, cnt: int, stream):
        lo, hi = int(offsets[lo_t]), int(offsets[lo_t + cnt])
        off = torch.from_numpy(offsets[lo_t:lo_t + cnt + 1] - lo).pin_memory()
        d_ids = torch.empty(hi - lo, dtype=torch.int32, device=dev)
        d_off = torch.empty(cnt + 1, dtype=torch.int64, device=dev)
        d_ids.copy_(pinned_ids[lo:hi], non_blocking=True)
        d_off.copy_(off, non_blocking=True)
        return d_off, d_ids

    def compute(tables, begin: int, cnt: int, stream) -> None:
        ylt = torch.empty(cnt, dtype=torch.float64, device=dev)
        res = torch.empty(1 + 2 * len(probs), dtype=torch.float64, device=dev)
        for s in specs_for(begin, cnt):
            ara.run_layers(tables, [s], out=ylt, stream=stream)
            ara.risk_metrics(ylt, list(probs), outputs=res, stream=stream)

    # single-tenant components for the fit
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        for _ in range(2):
            t0 = time.perf_counter()
            d_off, d_ids = ship(0, n, st)
            st.synchronize()
            t_ship = time.perf_counter() - t0
            t0 = time.perf_counter()
            tab = ara.create_yet(base, d_off, d_ids, stream=st)
            st.synchronize()
            t_build = time.perf_counter() - t0
            del d_off, d_ids
            t0 = time.perf_counter()
            compute(tab, 0, n, st)
            st.synchronize()
            t_comp = time.perf_counter() - t0
            tab.close()
        # per-tenant fixed cost: a one-trial slice shipped and built
        t0 = time.perf_counter()
        d_off, d_ids = ship(0, 1, st)
        tab = ara.create_yet(base, d_off, d_ids, stream=st)
        st.synchronize()
        t_fixed = time.perf_counter() - t0
        tab.close()
        del d_off, d_ids
    torch.cuda.synchronize()
    w_idle = w_busy = None
    if sampler.available:
        # the power reading is an average over about a second: sample 2 s windows
        time.sleep(1.0)
        with sampler:
            time.sleep(2.0)
        idle = sampler.summary()
        with sampler:
            t0 = time.perf_counter()
            while time.perf_counter() - t0 < 2.0:
                compute(base, 0, n, None)
                torch.cuda.synchronize()
        busy = sampler.summary()
        w_idle = idle["mean_power_w"] if idle else None
        w_busy = busy["mean_power_w"] if busy else None
    # the build runs on the GPU and splits with the trials: count it as compute
    model = fit_split_model(t_ship, t_comp + t_build, t_fixed, w_idle or 0.0, w_busy or 0.0)
    out: Dict[str, object] = {"trials": n, "layers": list(layer_ids), "fit": {
        "transfer_s": t_ship, "compute_s": t_comp, "build_s": t_build, "fixed_per_tenant_s": t_fixed,
        "power_idle_w": w_idle, "power_busy_w": w_busy}, "runs": {}}

    for mode in modes:
        for v in tenants:
            streams = [torch.cuda.Stream() for _ in range(v)]
            token = threading.Lock()
            errors: List[str] = []

            built: List[object] = []

            def tenant(k: int, b: int, c: int) -> None:
                try:
                    s = streams[k]
                    with torch.cuda.stream(s):
                        if mode == "sequential":
                            with token:
                                d_off, d_ids = ship(b, c, s)
                                s.synchronize()
                        else:
                            d_off, d_ids = ship(b, c, s)
                        tab = ara.create_yet(base, d_off, d_ids, stream=s)
                        del d_off, d_ids
                        compute(tab, 0, c, s)
                        s.synchronize()
                        built.append(tab)     # freed after the run: a free waits for the whole device
                except Exception as exc:  # reported, not raised inside the thread
                    errors.append(f"{type(exc).__name__}: {exc}")

            def once() -> float:
                torch.cuda.synchronize()
                ths = [threading.Thread(target=tenant, args=(k, b, c))
                       for k, (b, c) in enumerate(split_ranges(n, v))]
                t0 = time.perf_counter()
                for th in ths:
                    th.start()
                for th in ths:
                    th.join()
                torch.cuda.synchronize()
                wall = time.perf_counter() - t0
                for tab in built:
                    tab.close()
                built.clear()
                return wall

            best = once()
            # energy: the analysis back to back for >= 2 s inside one sampling
            # window (the power readings are too coarse for a single run); the
            # tables' frees between runs fall inside the window too
            k_runs = max(repeats, int(math.ceil(2.0 / max(best, 1e-3))))
            energy = None
            with sampler:
                for _ in range(k_runs):
                    best = min(best, once())
            summ = sampler.summary()
            if summ:
                # the window also holds the frees and thread starts between runs:
                # energy per analysis = the window's mean power x the analysis time
                energy = {"mean_power_w": summ["mean_power_w"],
                          "mean_gfx_activity_pct": summ["mean_gfx_activity_pct"],
                          "energy_j": summ["mean_power_w"] * best, "window_energy_j": summ["energy_j"],
                          "runs_in_window": k_runs, "samples": summ["samples"]}
            rec = {"time_s": best, "model_time_s": model.exec_time(1, v),
                   "model_fully_overlapped_s": model.time_fully_overlapped(1, v),
                   "model_not_overlapped_s": model.time_not_overlapped(1, v)}
            if energy:
                rec.update(energy)
                rec["model_energy_j"] = model.energy(1, v)
            if errors:
                rec["errors"] = errors[:3]
            out["runs"][f"{mode}_{v}"] = rec
            if log:
                en = f", {energy['energy_j']:.1f} J" if energy else ""
                log(f"split {mode} v={v}: {best * 1e3:.1f} ms (model {rec['model_time_s'] * 1e3:.1f} ms){en}")
    best_key = min(out["runs"], key=lambda k: out["runs"][k]["time_s"])
    model_v = min(tenants, key=lambda v: model.exec_time(1, v))
    out["best_measured"] = best_key
    out["best_model_tenants"] = model_v
    return out
