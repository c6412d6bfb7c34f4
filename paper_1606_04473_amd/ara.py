"""ctypes binding of libara (include/ara.h): argument marshalling only.

Every computation happens in the HIP library.  Inputs may be NumPy arrays
(host memory) or torch CUDA tensors (device memory); the binding passes the
pointer, the matching ARA_DEVICE_PTR flag and torch's current stream.  If the
library is missing the first call raises -- there is no CPU fallback.
"""

from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libara.so")

ARA_OK = 0
ARA_ERR_INVALID_ARG = 1
ARA_ERR_OUT_OF_RANGE = 2
ARA_ERR_BUFFER_TOO_SMALL = 3
ARA_ERR_NO_MEMORY = 4
ARA_ERR_DEVICE = 5
ARA_ERR_NOT_READY = 6
ARA_ERR_UNSUPPORTED = 7

ARA_DEVICE_PTR = 1 << 0
ARA_LITERAL = 1 << 1
ARA_CHECKPOINT_S = 1 << 2
ARA_PER_LAYER = 1 << 3
ARA_GRAPH = 1 << 4
ARA_PROFILE = 1 << 5
ARA_PLAIN_LAYOUT = 1 << 6
ARA_CHECKPOINT_STRIDE = 1 << 7

KERNEL_FOLD = 0
KERNEL_TRIAL_PASS = 1
KERNEL_BATCHED = 2
KERNEL_COMBINE = 3
KERNEL_AGGREGATE = 4

MAX_LAYER_ELTS = 64
CHECKPOINT_EVERY = 64

EXPORTED = (
    "ara_create_tables", "ara_destroy_tables", "ara_run_layers", "ara_risk_metrics", "ara_backward",
    "ara_last_error", "ara_status_string", "ara_table_bytes", "ara_footprint", "ara_debug_lookups",
    "ara_event_nets", "ara_run_portfolio",
    "ara_read_checkpoints", "ara_set_tuning", "ara_get_tuning", "ara_device_info",
    "ara_kernel_stats", "ara_create_yet", "ara_tail_count", "ara_layout_info_get",
)


class AraError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_STATUS_NAMES = {
    1: "ARA_ERR_INVALID_ARG", 2: "ARA_ERR_OUT_OF_RANGE", 3: "ARA_ERR_BUFFER_TOO_SMALL",
    4: "ARA_ERR_NO_MEMORY", 5: "ARA_ERR_DEVICE", 6: "ARA_ERR_NOT_READY", 7: "ARA_ERR_UNSUPPORTED",
}


class CLayer(ctypes.Structure):
    _fields_ = [
        ("n_elts", ctypes.c_int32),
        ("elt_index", ctypes.c_void_p),
        ("elt_retention", ctypes.c_void_p),
        ("elt_limit", ctypes.c_void_p),
        ("occ_retention", ctypes.c_double),
        ("occ_limit", ctypes.c_double),
        ("agg_retention", ctypes.c_double),
        ("agg_limit", ctypes.c_double),
        ("trial_begin", ctypes.c_int64),
        ("trial_count", ctypes.c_int64),
    ]


class CProgram(ctypes.Structure):
    _fields_ = [("n_layers", ctypes.c_int32), ("layers", ctypes.POINTER(CLayer))]


class CPortfolioOut(ctypes.Structure):
    _fields_ = [
        ("layer_ylt", ctypes.c_void_p), ("layer_capacity", ctypes.c_int64),
        ("program_ylt", ctypes.c_void_p), ("program_capacity", ctypes.c_int64),
        ("portfolio_ylt", ctypes.c_void_p), ("portfolio_capacity", ctypes.c_int64),
    ]


class CTuning(ctypes.Structure):
    _fields_ = [
        ("block_threads", ctypes.c_int32),
        ("part_lanes_per_trial", ctypes.c_int32),
        ("lanes_per_trial", ctypes.c_int32),
        ("blocks_per_cu", ctypes.c_int32),
        ("fold_events_per_thread", ctypes.c_int32),
        ("schedule", ctypes.c_int32),
        ("pass_variant", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]



class CLayoutInfo(ctypes.Structure):
    _fields_ = [
        ("image_parts", ctypes.c_int32),
        ("stream_parts", ctypes.c_int32),
        ("stream_group_trials", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("partitioned_ids", ctypes.c_int64),
        ("partitioned_bytes", ctypes.c_int64),
        ("stream_groups", ctypes.c_int64),
        ("stream_ids", ctypes.c_int64),
        ("stream_bytes", ctypes.c_int64),
    ]

_LIB = None


def lib():
    """Load libara.so; raise if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "or python paper_1606_04473_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64, u32, f64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                             ctypes.c_double)
    L.ara_create_tables.argtypes = [P, i64, P, i64, P, i32, i64, u32, P, ctypes.POINTER(P)]
    L.ara_create_tables.restype = i32
    L.ara_create_yet.argtypes = [P, P, i64, P, i64, u32, P, ctypes.POINTER(P)]
    L.ara_create_yet.restype = i32
    L.ara_destroy_tables.argtypes = [P]
    L.ara_destroy_tables.restype = None
    L.ara_run_layers.argtypes = [P, ctypes.POINTER(CLayer), i32, P, i64, u32, P]
    L.ara_run_layers.restype = i32
    L.ara_risk_metrics.argtypes = [P, i64, P, i32, P, P, P, u32, P]
    L.ara_risk_metrics.restype = i32
    L.ara_yet_footprint.argtypes = [i64, i64, i64, u32, ctypes.POINTER(i64)]
    L.ara_yet_footprint.restype = i32
    L.ara_metrics_footprint.argtypes = [i64, i32, u32, ctypes.POINTER(i64)]
    L.ara_metrics_footprint.restype = i32
    L.ara_debug_read.argtypes = [P, P, i32, P, i64, ctypes.POINTER(i64), P]
    L.ara_debug_read.restype = i32
    L.ara_risk_metrics_noalloc.argtypes = [P, i64, P, i32, P, P, P, P]
    L.ara_risk_metrics_noalloc.restype = i32
    L.ara_backward.argtypes = [P, ctypes.POINTER(CLayer), f64, P, P, u32, P]
    L.ara_backward.restype = i32
    L.ara_last_error.argtypes = []
    L.ara_last_error.restype = ctypes.c_char_p
    L.ara_status_string.argtypes = [i32]
    L.ara_status_string.restype = ctypes.c_char_p
    L.ara_table_bytes.argtypes = [P, ctypes.POINTER(i64)]
    L.ara_table_bytes.restype = i32
    L.ara_analyze.argtypes = [P, ctypes.POINTER(CLayer), P, i32, P, i64, P, u32, P]
    L.ara_analyze.restype = i32
    L.ara_cached_memory.argtypes = [ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.ara_cached_memory.restype = i32
    L.ara_release_cached_memory.argtypes = [ctypes.POINTER(i64)]
    L.ara_release_cached_memory.restype = i32
    L.ara_footprint.argtypes = [P, ctypes.POINTER(CLayer), i32, u32, ctypes.POINTER(i64)]
    L.ara_footprint.restype = i32
    L.ara_debug_lookups.argtypes = [P, ctypes.POINTER(CLayer), i64, P, P, i64, ctypes.POINTER(i64), P]
    L.ara_debug_lookups.restype = i32
    L.ara_run_portfolio.argtypes = [P, ctypes.POINTER(CProgram), i32, i32, ctypes.POINTER(CPortfolioOut),
                                    u32, P]
    L.ara_run_portfolio.restype = i32
    L.ara_event_nets.argtypes = [P, ctypes.POINTER(CLayer), P, i64, ctypes.POINTER(i64), u32, P]
    L.ara_event_nets.restype = i32
    L.ara_read_checkpoints.argtypes = [P, i32, P, i64, ctypes.POINTER(i64)]
    L.ara_read_checkpoints.restype = i32
    L.ara_set_tuning.argtypes = [P, ctypes.POINTER(CTuning)]
    L.ara_set_tuning.restype = i32
    L.ara_get_tuning.argtypes = [P, ctypes.POINTER(CTuning)]
    L.ara_get_tuning.restype = i32
    L.ara_kernel_stats.argtypes = [P, i32, ctypes.POINTER(i64), ctypes.POINTER(f64), i32]
    L.ara_kernel_stats.restype = i32
    L.ara_layout_info_get.argtypes = [P, ctypes.POINTER(CLayoutInfo)]
    L.ara_layout_info_get.restype = i32
    L.ara_device_info.argtypes = [ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.ara_device_info.restype = i32
    L.ara_tail_count.argtypes = [i64, f64, ctypes.POINTER(i64)]
    L.ara_tail_count.restype = i32
    _LIB = L
    return L


def _check(status: int) -> None:
    if status != ARA_OK:
        msg = lib().ara_last_error().decode(errors="replace")
        raise AraError(status, msg)


# ---------------------------------------------------------------------------
# array marshalling
# ---------------------------------------------------------------------------

def _is_device(x) -> bool:
    return hasattr(x, "is_cuda") and bool(x.is_cuda)


def _ptr(x, dtype=None):
    """(pointer, keepalive, on_device) for a NumPy array or torch tensor."""
    if x is None:
        return None, None, False
    if hasattr(x, "data_ptr"):
        if dtype is not None:
            import torch
            want = {np.float64: torch.float64, np.int64: torch.int64, np.uint32: None,
                    np.int32: torch.int32}[dtype]
            if want is not None and x.dtype != want:
                raise TypeError(f"expected {want}, got {x.dtype}")
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return ctypes.c_void_p(x.data_ptr()), x, _is_device(x)
    a = np.ascontiguousarray(x, dtype=dtype) if dtype is not None else np.ascontiguousarray(x)
    return a.ctypes.data_as(ctypes.c_void_p), a, False


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available() and torch.cuda.is_initialized():
                return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        except Exception:
            pass
        return ctypes.c_void_p(0)
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


@dataclass
class LayerSpec:
    """A layer as the library sees it: pool rows, per-ELT terms, layer terms
    and the trial range."""

    elt_index: np.ndarray
    elt_retention: np.ndarray
    elt_limit: np.ndarray
    occ_retention: float
    occ_limit: float
    agg_retention: float
    agg_limit: float
    trial_begin: int
    trial_count: int

    @property
    def n_elts(self) -> int:
        return int(len(self.elt_index))

    @staticmethod
    def from_layer(layer, pool, n_trials: int) -> "LayerSpec":
        idx = np.ascontiguousarray(layer.elt_index, dtype=np.int32)
        count = layer.trial_count if layer.trial_count >= 0 else n_trials - layer.trial_begin
        return LayerSpec(idx, np.ascontiguousarray(pool.retention[idx], dtype=np.float64),
                         np.ascontiguousarray(pool.limit[idx], dtype=np.float64),
                         float(layer.occ_retention), float(layer.occ_limit),
                         float(layer.agg_retention), float(layer.agg_limit),
                         int(layer.trial_begin), int(count))

    def theta(self) -> np.ndarray:
        return np.concatenate([self.elt_retention, self.elt_limit,
                               [self.occ_retention, self.occ_limit, self.agg_retention,
                                self.agg_limit]]).astype(np.float64)

    def with_theta(self, theta: Sequence[float]) -> "LayerSpec":
        J = self.n_elts
        t = np.asarray(theta, dtype=np.float64)
        return LayerSpec(self.elt_index, t[:J].copy(), t[J:2 * J].copy(), float(t[2 * J]),
                         float(t[2 * J + 1]), float(t[2 * J + 2]), float(t[2 * J + 3]),
                         self.trial_begin, self.trial_count)


def _c_layers(specs: Sequence[LayerSpec]):
    arr = (CLayer * len(specs))()
    keep = []
    for i, s in enumerate(specs):
        idx = np.ascontiguousarray(s.elt_index, dtype=np.int32)
        R = np.ascontiguousarray(s.elt_retention, dtype=np.float64)
        Lim = np.ascontiguousarray(s.elt_limit, dtype=np.float64)
        keep += [idx, R, Lim]
        arr[i] = CLayer(idx.shape[0], idx.ctypes.data_as(ctypes.c_void_p),
                        R.ctypes.data_as(ctypes.c_void_p), Lim.ctypes.data_as(ctypes.c_void_p),
                        s.occ_retention, s.occ_limit, s.agg_retention, s.agg_limit,
                        int(s.trial_begin), int(s.trial_count))
    return arr, keep


# ---------------------------------------------------------------------------
# API
# ---------------------------------------------------------------------------

class Tables:
    """Resident YET + ELT pool (ara_create_tables / ara_destroy_tables)."""

    def __init__(self, handle, n_trials: int, n_events: int, catalogue_size: int, n_pool: int):
        self._h = handle
        self.n_trials = n_trials
        self.n_events = n_events
        self.catalogue_size = catalogue_size
        self.n_pool = n_pool

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("tables destroyed")
        return self._h

    def close(self) -> None:
        if self._h is not None:
            lib().ara_destroy_tables(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def bytes(self) -> int:
        v = ctypes.c_int64()
        _check(lib().ara_table_bytes(self.handle, ctypes.byref(v)))
        return int(v.value)

    def layout(self) -> dict:
        """ara_layout_info_get: the sizes of the YET copies the passes stream."""
        v = CLayoutInfo()
        _check(lib().ara_layout_info_get(self.handle, ctypes.byref(v)))
        return {name: int(getattr(v, name)) for name, _ in CLayoutInfo._fields_ if name != "reserved"}


def create_tables(offsets, ids, elt_losses, catalogue_size: Optional[int] = None,
                  stream=None, flags: int = 0) -> Tables:
    """ara_create_tables.  NumPy inputs are host memory; CUDA tensors device memory."""
    po, ko, do = _ptr(offsets, np.int64)
    pi, ki, di = _ptr(ids, np.uint32)
    pe, ke, de = _ptr(elt_losses, np.float64)
    if not (do == di == de):
        raise ValueError("inputs must all be host arrays or all device tensors")
    n_trials = int(ko.shape[0]) - 1
    n_events = int(ki.shape[0])
    shape = tuple(ke.shape)
    n_pool = int(shape[0])
    C = int(shape[1]) if catalogue_size is None else int(catalogue_size)
    h = ctypes.c_void_p()
    _check(lib().ara_create_tables(po, n_trials, pi, n_events, pe, n_pool, C,
                                   flags | (ARA_DEVICE_PTR if do else 0), _stream(stream),
                                   ctypes.byref(h)))
    return Tables(h, n_trials, n_events, C, n_pool)


def create_yet(base: Tables, offsets, ids, stream=None, flags: int = 0) -> Tables:
    """ara_create_yet: tables owning this YET and sharing base's ELT pool.
    The returned object keeps `base` alive."""
    po, ko, do = _ptr(offsets, np.int64)
    pi, ki, di = _ptr(ids, np.uint32)
    if do != di:
        raise ValueError("offsets and ids must both be host arrays or both device tensors")
    n_trials = int(ko.shape[0]) - 1
    n_events = int(ki.shape[0])
    h = ctypes.c_void_p()
    _check(lib().ara_create_yet(base.handle, po, n_trials, pi, n_events,
                                flags | (ARA_DEVICE_PTR if do else 0), _stream(stream), ctypes.byref(h)))
    t = Tables(h, n_trials, n_events, base.catalogue_size, base.n_pool)
    t._base = base
    return t


def run_layers(tables: Tables, layers: Sequence[LayerSpec], out=None, flags: int = 0,
               stream=None):
    """ara_run_layers.  Returns the YLT (back to back per layer): a NumPy array
    when `out` is None, else `out` (NumPy or a CUDA float64 tensor)."""
    arr, keep = _c_layers(layers)
    total = int(sum(l.trial_count for l in layers))
    if out is None:
        out = np.empty(total, dtype=np.float64)
    po, ko, dev = _ptr(out, np.float64)
    f = flags | (ARA_DEVICE_PTR if dev else 0)
    _check(lib().ara_run_layers(tables.handle, arr, len(layers), po, int(ko.numel() if dev else ko.size),
                                f, _stream(stream)))
    return out


def risk_metrics(ylt, probs: Sequence[float], stream=None, outputs=None):
    """ara_risk_metrics.  Host input -> (mean, [pml], [tvar]) floats.  Device
    input -> the same computed on the device; if `outputs` is a float64 CUDA
    tensor of size 1 + 2 n_probs it receives [mean, pml..., tvar...] and the
    call stays asynchronous."""
    py, ky, dev = _ptr(ylt, np.float64)
    n = int(ky.numel() if dev else ky.size)
    p = np.ascontiguousarray(probs, dtype=np.float64)
    k = p.shape[0]
    if dev:
        import torch
        res = outputs if outputs is not None else torch.empty(1 + 2 * k, dtype=torch.float64,
                                                              device=ky.device)
        base = res.data_ptr()
        _check(lib().ara_risk_metrics(py, n, p.ctypes.data_as(ctypes.c_void_p), k,
                                      ctypes.c_void_p(base), ctypes.c_void_p(base + 8),
                                      ctypes.c_void_p(base + 8 * (1 + k)), ARA_DEVICE_PTR,
                                      _stream(stream)))
        if outputs is not None:
            return outputs
        h = res.cpu().numpy()
        return float(h[0]), h[1:1 + k].tolist(), h[1 + k:].tolist()
    mean = ctypes.c_double()
    pml = np.empty(max(k, 1), dtype=np.float64)
    tvar = np.empty(max(k, 1), dtype=np.float64)
    _check(lib().ara_risk_metrics(py, n, p.ctypes.data_as(ctypes.c_void_p), k, ctypes.byref(mean),
                                  pml.ctypes.data_as(ctypes.c_void_p),
                                  tvar.ctypes.data_as(ctypes.c_void_p), 0, _stream(stream)))
    return float(mean.value), pml[:k].tolist(), tvar[:k].tolist()


def risk_metrics_noalloc(ylt, probs: Sequence[float], outputs, stream=None):
    """ara_risk_metrics_noalloc: `ylt` a float64 CUDA tensor, `outputs` a
    float64 CUDA tensor of size 1 + 2 n_probs that receives [mean, pml...,
    tvar...]; asynchronous on `stream`.  The library allocates nothing."""
    py, ky, dev = _ptr(ylt, np.float64)
    po, ko, dev_o = _ptr(outputs, np.float64)
    if not (dev and dev_o):
        raise ValueError("ara_risk_metrics_noalloc takes device tensors")
    p = np.ascontiguousarray(probs, dtype=np.float64)
    k = p.shape[0]
    if ko.numel() < 1 + 2 * k:
        raise ValueError("outputs must hold 1 + 2 n_probs doubles")
    base = outputs.data_ptr()
    _check(lib().ara_risk_metrics_noalloc(py, int(ky.numel()), p.ctypes.data_as(ctypes.c_void_p), k,
                                          ctypes.c_void_p(base), ctypes.c_void_p(base + 8),
                                          ctypes.c_void_p(base + 8 * (1 + k)), _stream(stream)))
    return outputs


def backward(tables: Tables, layer: LayerSpec, tvar_p: float, grad_mean=None, grad_tvar=None,
             stream=None):
    """ara_backward.  Returns (grad_mean, grad_tvar) as NumPy arrays of 2J+4
    unless CUDA tensors are passed to receive them."""
    arr, keep = _c_layers([layer])
    P = 2 * layer.n_elts + 4
    if grad_mean is None and grad_tvar is None:
        gm = np.empty(P, dtype=np.float64)
        gt = np.empty(P, dtype=np.float64)
        _check(lib().ara_backward(tables.handle, arr, float(tvar_p),
                                  gm.ctypes.data_as(ctypes.c_void_p),
                                  gt.ctypes.data_as(ctypes.c_void_p), 0, _stream(stream)))
        return gm, gt
    pm, km, dm = _ptr(grad_mean, np.float64)
    pt, kt, dt = _ptr(grad_tvar, np.float64)
    dev = dm or dt
    _check(lib().ara_backward(tables.handle, arr, float(tvar_p), pm, pt,
                              ARA_DEVICE_PTR if dev else 0, _stream(stream)))
    return grad_mean, grad_tvar


def debug_lookups(tables: Tables, layer: LayerSpec, trial: int, capacity: int = 4096, stream=None):
    """ara_debug_lookups: (ids[K], losses[K][J]) as the device looks them up."""
    arr, keep = _c_layers([layer])
    J = layer.n_elts
    ids = np.empty(capacity, dtype=np.uint32)
    losses = np.empty(capacity * max(J, 1), dtype=np.float64)
    n = ctypes.c_int64()
    _check(lib().ara_debug_lookups(tables.handle, arr, int(trial), ids.ctypes.data_as(ctypes.c_void_p),
                                   losses.ctypes.data_as(ctypes.c_void_p), capacity, ctypes.byref(n),
                                   _stream(stream)))
    K = int(n.value)
    return ids[:K].copy(), losses[:K * J].reshape(K, J).copy()


DEBUG_OCCURRENCE = 0
DEBUG_COMPACT = 1
DEBUG_IMAGES = 2
DEBUG_STREAM_IDS = 3
DEBUG_STREAM_BASE = 4
DEBUG_STREAM_GSTART = 5
DEBUG_STREAM_GEND = 6
_DEBUG_DTYPES = {DEBUG_OCCURRENCE: np.float64, DEBUG_COMPACT: np.float64, DEBUG_IMAGES: np.uint8,
                 DEBUG_STREAM_IDS: np.uint16, DEBUG_STREAM_BASE: np.int64, DEBUG_STREAM_GSTART: np.uint32,
                 DEBUG_STREAM_GEND: np.uint16}


def debug_read(tables: Tables, what: int, layer: Optional[LayerSpec] = None, stream=None) -> np.ndarray:
    """ara_debug_read: the fold's o(E), compact values or part images for
    `layer`, or the arrays of the 16-bit stream copy, as a NumPy array."""
    arr = None
    if layer is not None:
        arr, keep = _c_layers([layer])
    n = ctypes.c_int64()
    st = lib().ara_debug_read(tables.handle, arr, int(what), None, 0, ctypes.byref(n), _stream(stream))
    if st not in (ARA_OK, ARA_ERR_BUFFER_TOO_SMALL):
        _check(st)
    out = np.empty(int(n.value) // np.dtype(_DEBUG_DTYPES[what]).itemsize, dtype=_DEBUG_DTYPES[what])
    _check(lib().ara_debug_read(tables.handle, arr, int(what), out.ctypes.data_as(ctypes.c_void_p), out.nbytes,
                                ctypes.byref(n), _stream(stream)))
    return out


PORTFOLIO_OUTPUTS = ("layer", "program", "portfolio")


def run_portfolio(tables: Tables, programs: Sequence[Sequence[LayerSpec]], n_splits: int = 1,
                  outs=None, flags: int = 0, stream=None):
    """ara_run_portfolio: a portfolio given as a list of programs, each a list
    of layers over the same trials.  With `outs` None, returns host arrays
    {"layer": [n_layers, n], "program": [n_programs, n], "portfolio": [n]}.
    Otherwise `outs` maps some of those names to NumPy arrays or CUDA float64
    tensors (all host or all device) and only those are written."""
    progs = (CProgram * len(programs))()
    keep = []
    for i, layers in enumerate(programs):
        arr, k = _c_layers(layers) if len(layers) else ((CLayer * 1)(), [])
        keep += [arr, k]
        progs[i] = CProgram(len(layers), ctypes.cast(arr, ctypes.POINTER(CLayer)))
    if outs is None:
        n = int(programs[0][0].trial_count) if programs and programs[0] else 0
        n_layers = sum(len(p) for p in programs)
        outs = {"layer": np.empty((n_layers, n)), "program": np.empty((len(programs), n)),
                "portfolio": np.empty(n)}
    unknown = set(outs) - set(PORTFOLIO_OUTPUTS)
    if unknown:
        raise KeyError(f"unknown outputs {sorted(unknown)}")
    c = CPortfolioOut()
    devs = set()
    for name in PORTFOLIO_OUTPUTS:
        if outs.get(name) is None:
            continue
        po, ko, dev = _ptr(outs[name], np.float64)
        if not dev and ko is not outs[name]:
            raise ValueError(f"output {name!r} must be a contiguous float64 array")
        devs.add(dev)
        keep.append(ko)
        setattr(c, f"{name}_ylt", po)
        setattr(c, f"{name}_capacity", int(ko.numel() if dev else ko.size))
    if len(devs) > 1:
        raise ValueError("outputs must be all host or all device")
    f = flags | (ARA_DEVICE_PTR if devs == {True} else 0)
    _check(lib().ara_run_portfolio(tables.handle, progs, len(programs), int(n_splits), ctypes.byref(c), f,
                                   _stream(stream)))
    return outs


def analyze(tables: Tables, layer: LayerSpec, probs, ylt=None, metrics=None, flags: int = 0, stream=None):
    """ara_analyze: the layer's year losses and [mean, PML_p..., TVaR_p...].
    With CUDA tensors for `ylt` and `metrics` the call is asynchronous on
    `stream` (ARA_GRAPH replays one graph); otherwise NumPy arrays are
    returned.  Returns (ylt, metrics)."""
    arr, keep = _c_layers([layer])
    p = np.ascontiguousarray(probs, dtype=np.float64)
    k = int(p.shape[0])
    if ylt is None:
        ylt = np.empty(layer.trial_count, dtype=np.float64)
    if metrics is None:
        metrics = np.empty(1 + 2 * k, dtype=np.float64)
    py, ky, dy = _ptr(ylt, np.float64)
    pm, km, dm = _ptr(metrics, np.float64)
    if dy != dm:
        raise ValueError("ylt and metrics must both be host arrays or both device tensors")
    cap = int(ky.numel() if dy else ky.size)
    mcap = int(km.numel() if dm else km.size)
    if mcap < 1 + 2 * k:
        raise ValueError("metrics holds fewer than 1 + 2 * len(probs) values")
    _check(lib().ara_analyze(tables.handle, arr, p.ctypes.data_as(ctypes.c_void_p), k, py, cap, pm,
                             flags | (ARA_DEVICE_PTR if dy else 0), _stream(stream)))
    return ylt, metrics


def event_nets(tables: Tables, layer: LayerSpec, out=None, stream=None):
    """ara_event_nets: per-event net losses of the layer's trials in time
    order.  Returns a NumPy array, or fills `out` (NumPy or a CUDA float64
    tensor) and returns it."""
    arr, keep = _c_layers([layer])
    n = ctypes.c_int64()
    if out is None:
        st = lib().ara_event_nets(tables.handle, arr, None, 0, ctypes.byref(n), 0, _stream(stream))
        if st not in (ARA_OK, ARA_ERR_BUFFER_TOO_SMALL):
            _check(st)
        out = np.empty(max(int(n.value), 1), dtype=np.float64)
        _check(lib().ara_event_nets(tables.handle, arr, out.ctypes.data_as(ctypes.c_void_p), out.shape[0],
                                    ctypes.byref(n), 0, _stream(stream)))
        return out[:int(n.value)]
    po, ko, dev = _ptr(out, np.float64)
    cap = int(ko.numel() if dev else ko.size)
    _check(lib().ara_event_nets(tables.handle, arr, po, cap, ctypes.byref(n), ARA_DEVICE_PTR if dev else 0,
                                _stream(stream)))
    return out


def read_checkpoints(tables: Tables, what: int):
    n = ctypes.c_int64()
    st = lib().ara_read_checkpoints(tables.handle, what, None, 0, ctypes.byref(n))
    if st not in (ARA_OK, ARA_ERR_BUFFER_TOO_SMALL):
        _check(st)
    out = np.empty(max(int(n.value), 1), dtype=np.float64)
    _check(lib().ara_read_checkpoints(tables.handle, what, out.ctypes.data_as(ctypes.c_void_p),
                                      out.shape[0], ctypes.byref(n)))
    return out[:int(n.value)]


def footprint(tables: Tables, layers: Sequence[LayerSpec], flags: int = 0) -> int:
    arr, keep = _c_layers(layers)
    v = ctypes.c_int64()
    _check(lib().ara_footprint(tables.handle, arr, len(layers), flags, ctypes.byref(v)))
    return int(v.value)


def yet_footprint(n_trials: int, n_events: int, catalogue_size: int, flags: int = 0) -> int:
    """ara_yet_footprint: device bytes of tables built for a YET of these sizes."""
    v = ctypes.c_int64()
    _check(lib().ara_yet_footprint(int(n_trials), int(n_events), int(catalogue_size), int(flags), ctypes.byref(v)))
    return int(v.value)


def metrics_footprint(n_trials: int, n_probs: int, flags: int = ARA_DEVICE_PTR) -> int:
    """ara_metrics_footprint: scratch bytes of one ara_risk_metrics call."""
    v = ctypes.c_int64()
    _check(lib().ara_metrics_footprint(int(n_trials), int(n_probs), int(flags), ctypes.byref(v)))
    return int(v.value)


TUNING_FIELDS = ("part_lanes_per_trial", "lanes_per_trial", "blocks_per_cu", "schedule", "pass_variant")


def set_tuning(tables: Tables, lanes_per_trial: int = 0, blocks_per_cu: int = 0,
               part_lanes_per_trial: int = 0, schedule: int = 0, pass_variant: int = 0) -> None:
    """Launch-shape knobs for later calls on `tables` (0 = default)."""
    t = CTuning(0, part_lanes_per_trial, lanes_per_trial, blocks_per_cu, 0, schedule, pass_variant)
    _check(lib().ara_set_tuning(tables.handle, ctypes.byref(t)))


def get_tuning(tables: Tables) -> dict:
    t = CTuning()
    _check(lib().ara_get_tuning(tables.handle, ctypes.byref(t)))
    return {k: int(getattr(t, k)) for k in TUNING_FIELDS}


def kernel_stats(tables: Tables, kernel: int, reset: bool = False):
    """(launches, total_ms) of one kernel class over ARA_PROFILE runs."""
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    _check(lib().ara_kernel_stats(tables.handle, kernel, ctypes.byref(n), ctypes.byref(ms),
                                  1 if reset else 0))
    return int(n.value), float(ms.value)


def device_info():
    n = ctypes.c_int32()
    d = ctypes.c_int32()
    _check(lib().ara_device_info(ctypes.byref(n), ctypes.byref(d)))
    return int(n.value), int(d.value)


def tail_count(n_trials: int, p: float) -> int:
    """The m that PML_p and TVaR_p are taken over (host only, no device)."""
    m = ctypes.c_int64()
    _check(lib().ara_tail_count(int(n_trials), float(p), ctypes.byref(m)))
    return int(m.value)


def cached_memory():
    """ara_cached_memory on the current device: (held_bytes, idle_bytes)."""
    held, idle = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().ara_cached_memory(ctypes.byref(held), ctypes.byref(idle)))
    return held.value, idle.value


def release_cached_memory() -> int:
    """ara_release_cached_memory on the current device: bytes released."""
    freed = ctypes.c_int64()
    _check(lib().ara_release_cached_memory(ctypes.byref(freed)))
    return freed.value


def status_string(status: int) -> str:
    return lib().ara_status_string(status).decode()
