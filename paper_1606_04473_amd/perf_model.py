"""Performance and energy model for multi-tenant deployments (Section V-F).

Eq. 4:  total = T_transfer(g) + T_computation(g)
Eq. 5:  T_computation(g) = ComputationTime_1pGPU / g        (perfect scaling)
Eq. 6:  T_transfer(g) = g (T_alloc + T_small + T_4MB + T_120MB) + T_4GB
        (per-device allocation and replicated ELT/portfolio copies; the
        YET is split, so its transfer does not grow with g)
Eq. 7:  fully overlapped multi-tenancy with v tenants per physical GPU:
        T_transfer(p v) / v + v T_computation(p v)
Eq. 8:  not fully overlapped: T_transfer(p v) + T_computation(p v)
Eq. 9:  time = max(Eq. 7, Eq. 8)
Eq. 10: energy = p (T_computation(p) W_compute
                    + (time - T_computation(p)) W_idle)

`Platform` carries the constants (Table II for the paper's K20 + InfiniBand
platforms; `fit_one_gpu` re-fits them from tenant measurements on one GPU).
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, Iterable, List, Optional, Sequence, Tuple


@dataclass(frozen=True)
class Platform:
    compute_1gpu: float          # ComputationTime_1pGPU (s)
    t_alloc: float               # T_cudaMalloc
    t_small: float               # T_small_transfers
    t_4mb: float                 # T_transfer_4MB   (portfolio, replicated)
    t_120mb: float               # T_transfer_120MB (ELTs, replicated)
    t_4gb: float                 # T_transfer_4GB   (the YET, split)
    w_idle: float = 47.0         # idle or receiving (W)
    w_compute: float = 102.0     # computing (W)

    def t_computation(self, n_gpus: int) -> float:
        return self.compute_1gpu / n_gpus

    def t_transfer(self, n_gpus: int) -> float:
        return n_gpus * (self.t_alloc + self.t_small + self.t_4mb + self.t_120mb) + self.t_4gb

    def time_fully_overlapped(self, p: int, v: int) -> float:
        g = p * v
        return self.t_transfer(g) / v + v * self.t_computation(g)

    def time_not_overlapped(self, p: int, v: int) -> float:
        g = p * v
        return self.t_transfer(g) + self.t_computation(g)

    def exec_time(self, p: int, v: int) -> float:
        return max(self.time_fully_overlapped(p, v), self.time_not_overlapped(p, v))

    def energy(self, p: int, v: int) -> float:
        t = self.exec_time(p, v)
        tc = self.t_computation(p)
        return p * (tc * self.w_compute + (t - tc) * self.w_idle)


def from_table(row: Dict[str, float], compute_1gpu: float, w_idle: float = 47.0,
               w_compute: float = 102.0) -> Platform:
    return Platform(compute_1gpu, row["cudaMalloc"], row["small_transfers"], row["transfer_4MB"],
                    row["transfer_120MB"], row["transfer_4GB"], w_idle, w_compute)


def grid(platform: Platform, max_p: int = 16, max_v: int = 12,
         max_v_per_p: Optional[int] = None) -> List[Tuple[int, int, float, float]]:
    out = []
    for p in range(1, max_p + 1):
        for v in range(1, max_v + 1):
            if max_v_per_p is not None and v > max_v_per_p:
                continue
            out.append((p, v, platform.exec_time(p, v), platform.energy(p, v)))
    return out


def best_time(platform: Platform, **kw) -> Tuple[int, int, float]:
    p, v, t, _ = min(grid(platform, **kw), key=lambda r: (r[2], r[0] * r[1]))
    return p, v, t


def best_energy(platform: Platform, **kw) -> Tuple[int, int, float]:
    p, v, _, e = min(grid(platform, **kw), key=lambda r: (r[3], r[0] * r[1]))
    return p, v, e


def fit_one_gpu(compute_s: float, transfer_s: float, fixed_s: float = 0.0) -> Platform:
    """Constants for tenants sharing one GPU, from measurements: the whole
    analysis' device time (compute_s), the time to ship its YET (transfer_s)
    and any per-tenant fixed cost (allocation, table build: fixed_s).  The
    replicated-table terms vanish: the ELT pool stays resident."""
    return Platform(compute_s, fixed_s, 0.0, 0.0, 0.0, transfer_s)


def tenants_on_one_gpu(platform: Platform, max_tenants: int = 16) -> List[Tuple[int, float]]:
    """Eq. 9 with p = 1: predicted time of one analysis split over v tenants."""
    return [(v, platform.exec_time(1, v)) for v in range(1, max_tenants + 1)]
