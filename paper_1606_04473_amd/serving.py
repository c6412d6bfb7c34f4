"""Multi-tenant request loop on one GPU.

The paper runs several clients ("tenants") on virtual GPUs mapped onto one
physical GPU, so that one tenant's host-to-device transfer overlaps another's
kernel, and compares two transfer modes (Section V-D): *concurrent* (every
device receives its data at once, sharing the link) and *sequential* (one
transfer at a time at full link bandwidth while others compute).  Here the
tenants' requests share a pool of slots, each a worker thread with its own
HIP stream; slots share one GPU, the resident ELT pool and, in "resident"
mode, the resident YET.

Each request is an analysis: a slice of trials of the YET and 1-16 layers.
Shipped modes copy the slice to the device (Algorithm 2) -- concurrently or
under a FIFO transfer token -- and build tables for it that share the
resident ELT pool (ara_create_yet); resident mode runs the layers on trial
ranges of the resident YET.  Admission is by device memory: a request waits
(FIFO) until its footprint -- the library's own count of what it will hold --
fits the budget, then runs in the slot that took it, overlapping with the
other slots' work (continuous batching: requests are admitted as slots and
memory free up, not in fixed batches).  Results carry arrival, admission,
start and finish times; latency is finish minus arrival.
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

# Device staging for shipped slices, one (IDs, offsets) pair per (device, slot),
# sized for the whole YET and kept for the process: servers made one after the
# other reuse them.  Allocating a slice buffer per request would leave blocks
# of every size cached under each slot's stream by torch's allocator; once
# those caches fill the device, an allocation makes the allocator free them,
# and each free waits for the whole device (other slots' copies included).
_SLICE_BUFFERS: Dict[tuple, tuple] = {}


def slice_buffers(device, slot: int, n_ids: int, n_off: int):
    """Slot `slot`'s device staging on `device`: an int32 tensor of at least
    n_ids IDs and an int64 tensor of at least n_off offsets, allocated on first
    use (or when too small) and then reused."""
    import torch
    key = (device.index, slot)
    bufs = _SLICE_BUFFERS.get(key)
    if bufs is None or bufs[0].numel() < n_ids or bufs[1].numel() < n_off:
        _SLICE_BUFFERS.pop(key, None)
        torch.cuda.synchronize(device)
        bufs = (torch.empty(max(n_ids, 1), dtype=torch.int32, device=device),
                torch.empty(max(n_off, 1), dtype=torch.int64, device=device))
        _SLICE_BUFFERS[key] = bufs
    return bufs


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
    phases: Dict[str, float] = field(default_factory=dict)     # seconds: ship, build, compute
    stream_layout: bool = False           # the request's tables hold the 16-bit copy

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
    phases = {f"{k}_ms_mean": float(np.mean([r.phases[k] for r in ok if k in r.phases])) * 1e3
              for k in ("ship", "build", "compute") if any(k in r.phases for r in ok)}
    return {
        **phases,
        "fast_layout_requests": sum(1 for r in ok if r.stream_layout),
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
    """Serves requests on one GPU from a shared pool of `n_slots` slots.

    base:     resident tables (ELT pool and, for resident mode, the YET);
    offsets, ids: the host YET the requests slice (ids pinned by the server);
    library:  LayerSpec list (trial ranges are replaced per request);
    probs:    risk-metric probabilities reported per layer;
    budget_bytes: the device bytes requests may hold at once; None = the
              device's free memory when the server starts, less `reserve`.

    Requests wait in one arrival-ordered queue whatever their tenant; a free
    slot (a worker thread with its own HIP stream) takes the oldest arrived
    one, waits for admission by device memory (FIFO, the request's footprint
    from the library's own counts), then ships its YET slice (or uses the
    resident YET), runs its layers and metrics, and frees its memory.
    Requests that arrive while others run are admitted as slots and memory
    free up, and their work overlaps on the device.  A shipped slice lands in
    the slot's device staging (kept for the process and reused, see
    _SLICE_BUFFERS), from which the library copies it into the request's
    tables; the footprint still counts the slice.
    """

    def __init__(self, base, offsets: np.ndarray, ids: np.ndarray, library, n_slots: int,
                 mode: str, budget_bytes: Optional[int] = None, probs=(0.99,), pinned_ids=None,
                 reserve: int = 2 << 30):
        import torch
        from . import ara
        if mode not in MODES:
            raise ValueError(mode)
        self.torch = torch
        self.ara = ara
        self.base = base
        self.offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        self.library = list(library)
        self.n_slots = n_slots
        self.mode = mode
        self.probs = list(probs)
        self.free_bytes_at_start = int(torch.cuda.mem_get_info()[0])
        if budget_bytes is None:
            budget_bytes = max(self.free_bytes_at_start - reserve, 0)
        self.admission = AdmissionController(budget_bytes)
        self.transfer_token = threading.Lock()
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.streams = [torch.cuda.Stream() for _ in range(n_slots)]
        self.host_ids = pinned_ids
        if mode != "resident" and self.host_ids is None:
            self.host_ids = pin_ids(ids)
        if mode != "resident":
            for k in range(n_slots):
                self._slice_buffers(k)

    def _slice_buffers(self, slot: int):
        """The slot's device staging for a shipped slice, sized for the whole
        YET (see _SLICE_BUFFERS)."""
        return slice_buffers(self.device, slot, int(self.offsets[-1]), int(self.offsets.shape[0]))

    def footprint(self, req: Request) -> int:
        """Device bytes the request holds at its peak, from the library's counts:
        its shipped YET (the device copy it is shipped into, then the tables
        built from it, with their build temporaries), the scratch of its
        largest ara_run_layers call, the metrics scratch and its outputs."""
        ara = self.ara
        n = req.n_trials
        n_ev = int(self.offsets[req.trial_begin + n] - self.offsets[req.trial_begin])
        k = len(self.probs)
        b = 8 * n + 8 * (1 + 2 * k) * len(req.layer_ids)                 # YLT and metrics outputs
        b += ara.metrics_footprint(n, k, ara.ARA_DEVICE_PTR)
        specs = self._layers_for(req, 0 if self.mode != "resident" else req.trial_begin)
        b += max(ara.footprint(self.base, [s], ara.ARA_DEVICE_PTR) for s in specs)
        if self.mode != "resident":
            b += 4 * n_ev + 8 * (n + 1)                                    # the shipped slice
            b += ara.yet_footprint(n, n_ev, self.base.catalogue_size)
        return b

    def _layers_for(self, req: Request, begin: int):
        specs = []
        for lid in req.layer_ids:
            s = self.library[lid]
            specs.append(self.ara.LayerSpec(s.elt_index, s.elt_retention, s.elt_limit, s.occ_retention,
                                            s.occ_limit, s.agg_retention, s.agg_limit, begin, req.n_trials))
        return specs

    def _serve_one(self, req: Request, res: Result, slot: int, t0: float) -> None:
        torch, ara = self.torch, self.ara
        stream = self.streams[slot]
        try:
            nb = self.footprint(req)
        except Exception as exc:              # e.g. a layer the library rejects
            res.error = f"{type(exc).__name__}: {exc}"
            res.finished = time.perf_counter() - t0
            return
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
                    res.stream_layout = tables.layout()["stream_parts"] > 0
                else:
                    lo = int(self.offsets[req.trial_begin])
                    hi = int(self.offsets[req.trial_begin + req.n_trials])
                    off = torch.from_numpy(self.offsets[req.trial_begin:req.trial_begin + req.n_trials + 1] - lo)
                    off = off.pin_memory()
                    ids_buf, off_buf = self._slice_buffers(slot)
                    d_ids = ids_buf[:hi - lo]
                    d_off = off_buf[:req.n_trials + 1]
                    tp = time.perf_counter()
                    if self.mode == "sequential":
                        with self.transfer_token:
                            d_ids.copy_(self.host_ids[lo:hi], non_blocking=True)
                            d_off.copy_(off, non_blocking=True)
                            stream.synchronize()
                    else:
                        d_ids.copy_(self.host_ids[lo:hi], non_blocking=True)
                        d_off.copy_(off, non_blocking=True)
                    tb = time.perf_counter()
                    tables = ara.create_yet(self.base, d_off, d_ids, stream=stream)
                    res.phases["ship"] = tb - tp
                    res.phases["build"] = time.perf_counter() - tb
                    res.stream_layout = tables.layout()["stream_parts"] > 0
                    del d_ids, d_off
                    begin = 0
                specs = self._layers_for(req, begin)
                k = len(self.probs)
                tc = time.perf_counter()
                ylt = torch.empty(req.n_trials, dtype=torch.float64, device=self.device)
                out = torch.empty((len(specs), 1 + 2 * k), dtype=torch.float64, device=self.device)
                for i, s in enumerate(specs):
                    ara.run_layers(tables, [s], out=ylt, stream=stream)
                    ara.risk_metrics(ylt, self.probs, outputs=out[i], stream=stream)
                host = out.cpu()              # waits for this slot's stream only
                res.phases["compute"] = time.perf_counter() - tc
                res.metrics = host.numpy().tolist()
        except Exception as exc:              # a poisoned request fails alone
            res.error = f"{type(exc).__name__}: {exc}"
        finally:
            if tables is not None and tables is not self.base:
                tables.close()
            res.finished = time.perf_counter() - t0
            self.admission.release(nb)

    def run(self, requests: Sequence[Request], time_scale: float = 1.0) -> List[Result]:
        """Serve `requests`, each arriving at arrival * time_scale seconds
        (time_scale 0: all at once, a closed loop at saturation)."""
        queue = deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        results = {r.rid: Result(r.rid, r.tenant, r.arrival * time_scale) for r in requests}
        lock = threading.Lock()
        t0 = time.perf_counter()

        def slot(k: int) -> None:
            while True:
                with lock:
                    if not queue:
                        return
                    r = queue.popleft()
                wait = r.arrival * time_scale - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(wait)
                self._serve_one(r, results[r.rid], k, t0)

        threads = [threading.Thread(target=slot, args=(k,)) for k in range(self.n_slots)]
        for th in threads:
            th.start()
        for th in threads:
            th.join()
        self.torch.cuda.synchronize()
        self.wall = time.perf_counter() - t0
        return [results[r.rid] for r in requests]


def admission_summary(results: Sequence[Result], controller: AdmissionController) -> Dict[str, float]:
    """Admission by device memory: how many requests waited for memory and how
    long (from taking a slot to admission), the budget and the peak held, and
    the p99 of arrival to admission (waits for a slot and for memory)."""
    waits = [w for w in controller.waits]
    queued = [r.admitted - r.arrival for r in results if r.error is None and not math.isnan(r.admitted)]
    return {"budget_bytes": controller.budget, "peak_bytes": controller.peak,
            "admission_waits_over_1ms": int(sum(1 for w in waits if w > 1e-3)),
            "admission_wait_p50_ms": percentile(waits, 50) * 1e3,
            "admission_wait_p99_ms": percentile(waits, 99) * 1e3,
            "queue_to_admission_p99_ms": percentile(queued, 99) * 1e3}


def run_tenant_study(base, offsets, ids, library, n_tenants: int = 8, per_tenant: int = 6,
                     seed: int = 160604478, budget_bytes: Optional[int] = 16 << 30, probs=(0.99,),
                     load: float = 0.7, modes: Sequence[str] = ("concurrent", "sequential", "resident"),
                     log=None) -> Dict[str, object]:
    """Config-4 study.  Requests of n_tenants tenants (Poisson arrivals at
    `load` times the one-slot capacity) served from one slot and from
    n_tenants slots in each transfer mode: p50/p99 latency, throughput and
    admission waits under a device-memory budget (16 GiB by default, standing
    in for a GPU shared with other work, so that admission binds; None = the
    free memory).  Then the same requests all at once (closed loop), twice:
    the capacity in requests per second of each mode and slot count from the
    second run (the first is reported beside it)."""
    n_yet = int(offsets.shape[0] - 1)
    pinned = pin_ids(ids)
    # one-slot capacity, requests back to back, shipped concurrently
    probe = make_requests(1, 6, 0.0, n_yet, len(library), seed=seed + 77)
    srv = Server(base, offsets, ids, library, 1, "concurrent", budget_bytes, probs, pinned)
    srv.run(probe[:1], 0.0)                                   # warm-up
    res = srv.run(probe, 0.0)
    service = srv.wall / max(len(res), 1)
    rate_total = load / service
    reqs = make_requests(n_tenants, per_tenant, rate_total / n_tenants, n_yet, len(library), seed=seed)
    out: Dict[str, object] = {"service_ms_one_slot": service * 1e3, "arrival_rate_req_s": rate_total,
                              "load": load, "tenants": n_tenants, "requests": len(reqs),
                              "budget_bytes": srv.admission.budget,
                              "free_device_bytes": srv.free_bytes_at_start}
    for mode in modes:
        for k in (1, n_tenants):
            s = Server(base, offsets, ids, library, k, mode, budget_bytes, probs, pinned)
            r = s.run(reqs, 1.0)
            summ = summarize(r, s.wall)
            summ.update(admission_summary(r, s.admission))
            # steady state: the first closed-loop run grows the device caches to
            # this concurrency and is not counted
            closed = Server(base, offsets, ids, library, k, mode, budget_bytes, probs, pinned)
            rc0 = closed.run(reqs, 0.0)
            summ["capacity_first_run_req_s"] = summarize(rc0, closed.wall)["throughput_req_s"]
            closed = Server(base, offsets, ids, library, k, mode, budget_bytes, probs, pinned)
            rc = closed.run(reqs, 0.0)
            summ["capacity_req_s"] = summarize(rc, closed.wall)["throughput_req_s"]
            summ["capacity_admission_waits_over_1ms"] = admission_summary(rc, closed.admission)[
                "admission_waits_over_1ms"]
            out[f"{mode}_{k}t"] = summ
            if log:
                log(f"serving {mode} slots={k}: p50 {summ['p50_ms']:.1f} ms p99 {summ['p99_ms']:.1f} ms, "
                    f"{summ['throughput_req_s']:.2f} req/s offered, capacity {summ['capacity_req_s']:.2f} req/s "
                    f"(first run {summ['capacity_first_run_req_s']:.2f}), "
                    f"{summ['admission_waits_over_1ms']} admission waits (p99 {summ['admission_wait_p99_ms']:.1f} ms)")
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
                modes=("concurrent", "sequential"), probs=(0.99,), repeats: int = 3, window_s: float = 1.5,
                log=None) -> Dict[str, object]:
    """The whole YET analysed with `layer_ids`, split over v tenants on one
    GPU (each ships its slice, builds its tables, runs the layers and the
    metrics), for each transfer mode; wall time, energy and activity per
    (mode, v), and the model's prediction from single-tenant components.
    Energy per analysis comes from `repeats` rounds (every (mode, v) once per
    round, in rotated order) of a fixed window of back-to-back analyses:
    median and range over the rounds, gross and above the idle power."""
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

    def ship(lo_t: int, cnt: int, stream, slot: int = 0):
        lo, hi = int(offsets[lo_t]), int(offsets[lo_t + cnt])
        off = torch.from_numpy(offsets[lo_t:lo_t + cnt + 1] - lo).pin_memory()
        ids_buf, off_buf = slice_buffers(dev, slot, int(offsets[-1]), n + 1)
        d_ids = ids_buf[:hi - lo]
        d_off = off_buf[:cnt + 1]
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

    def make_runner(mode: str, v: int):
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
                            d_off, d_ids = ship(b, c, s, k)
                            s.synchronize()
                    else:
                        d_off, d_ids = ship(b, c, s, k)
                    tab = ara.create_yet(base, d_off, d_ids, stream=s)
                    del d_off, d_ids
                    compute(tab, 0, c, s)
                    s.synchronize()
                    built.append(tab)     # freed after the run: a free waits for the whole device
            except Exception as exc:  # reported, not raised inside the thread
                errors.append(f"{type(exc).__name__}: {exc}")

        def once() -> float:
            torch.cuda.synchronize()
            ths = [threading.Thread(target=tenant, args=(k, b, c)) for k, (b, c) in enumerate(split_ranges(n, v))]
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

        return once, errors

    combos = [(mode, v) for mode in modes for v in tenants]
    runners = {c: make_runner(*c) for c in combos}
    times = {c: [] for c in combos}
    energy = {c: [] for c in combos}
    for c in combos:
        times[c].append(runners[c][0]())                     # warm-up, timed
    # energy: every (mode, v) in turn, `repeats` rounds in rotated order, each a
    # fixed window of back-to-back analyses sampled as one: energy per analysis
    # = mean power x window / analyses, gross and above idle power
    for rnd in range(repeats):
        order = combos[rnd % len(combos):] + combos[:rnd % len(combos)]
        for c in order:
            once = runners[c][0]
            with sampler:
                t_start = time.perf_counter()
                k_runs = 0
                while time.perf_counter() - t_start < window_s:
                    times[c].append(once())
                    k_runs += 1
                span = time.perf_counter() - t_start
            summ = sampler.summary()
            if summ:
                e = {"gross_j": summ["mean_power_w"] * span / k_runs, "mean_power_w": summ["mean_power_w"],
                     "activity_pct": summ["mean_gfx_activity_pct"], "analyses": k_runs}
                if w_idle is not None:
                    e["net_j"] = (summ["mean_power_w"] - w_idle) * span / k_runs
                energy[c].append(e)
    for c in combos:
        mode, v = c
        t = times[c]
        rec = {"time_s": min(t), "time_median_s": float(np.median(t)), "runs": len(t),
               "model_time_s": model.exec_time(1, v), "model_fully_overlapped_s": model.time_fully_overlapped(1, v),
               "model_not_overlapped_s": model.time_not_overlapped(1, v)}
        es = energy[c]
        if es:
            g = [e["gross_j"] for e in es]
            rec.update({"energy_j": float(np.median(g)), "energy_j_min": min(g), "energy_j_max": max(g),
                        "mean_power_w": float(np.median([e["mean_power_w"] for e in es])),
                        "rounds": len(es), "analyses_per_window": [e["analyses"] for e in es],
                        "model_energy_j": model.energy(1, v)})
            acts = [e["activity_pct"] for e in es if e["activity_pct"] is not None]
            rec["mean_gfx_activity_pct"] = float(np.median(acts)) if acts else None
            if "net_j" in es[0]:
                nj = [e["net_j"] for e in es]
                rec.update({"energy_above_idle_j": float(np.median(nj)), "energy_above_idle_j_min": min(nj),
                            "energy_above_idle_j_max": max(nj)})
        if runners[c][1]:
            rec["errors"] = runners[c][1][:3]
        out["runs"][f"{mode}_{v}"] = rec
        if log:
            en = (f", {rec['energy_j']:.1f} J [{rec['energy_j_min']:.1f}, {rec['energy_j_max']:.1f}]"
                  if "energy_j" in rec else "")
            log(f"split {mode} v={v}: {rec['time_s'] * 1e3:.1f} ms (model {rec['model_time_s'] * 1e3:.1f} ms){en}")
    best_key = min(out["runs"], key=lambda k: out["runs"][k]["time_s"])
    model_v = min(tenants, key=lambda v: model.exec_time(1, v))
    out["best_measured"] = best_key
    out["best_model_tenants"] = model_v
    return out
