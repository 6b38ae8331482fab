"""Continuous-batching server for independent XL-BOMD systems on one GPU.

Requests (a System and an arrival time) are admitted while their estimated
HBM footprint fits the budget and a slot is free; each admitted system keeps
its whole state resident on the device (its library handle) and is stepped
by its own worker thread on its own HIP stream, so the kernels of all active
systems overlap on the GPU.  Requests that arrive while others run are
admitted as slots and memory free up.  Per-step latency (completion of step
s minus completion of step s-1, or of the initial state for s = 1) and the
queueing delay (arrival to admission) are recorded.

Only scheduling lives here; every step runs in the HIP library.
"""
from __future__ import annotations

import sys
import threading
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from .binding import MIXED, MIXED_BF16X3, FP32, FP64, XLBOMD

_ESZ = {FP64: (8, 8), FP32: (4, 4), MIXED: (8, 4), MIXED_BF16X3: (8, 4)}


def footprint_bytes(system, precision=MIXED, levels=10) -> int:
    """Upper estimate of the device memory one system holds (no energy
    evaluation, which the server does not request).

    Expansion matrices: Z_0..Z_L, Y_0..Y_{L-1}, A_0..A_{L-1}, the seed
    powers Y, Y^2, Y^3 and four work matrices; responses: three matrices per
    direction (nine on the split path: four work matrices, the split rows
    of Y D, Y^2 D, Y^3 D and the FP64 Y D Y^3), plus the response-precision
    copies of the
    expansion operands (Z, Y, Y..Y^4) when the two precisions differ, and
    on the split path the split Y, Y^2, Y^3, Z_L^2 and four level work
    matrices.
    """
    n = system.n_atoms * system.n_orb
    npad = -(-n // 128) * 128
    ef, er = _ESZ[precision]
    m = max(1, system.rank)
    mats_f = 3 * levels + 8
    if precision == MIXED_BF16X3:
        mats_r = 9 * m + 2 * levels + 13
    else:
        mats_r = 3 * m + ((2 * levels + 5) if ef != er else 0)
    vecs = 64 * system.n_atoms * 8 + 16 * npad * 8
    return npad * npad * (mats_f * ef + mats_r * er) + vecs


@dataclass
class RequestStats:
    name: str
    n_orb_total: int
    arrival: float
    admitted: float = 0.0
    ready: float = 0.0            # initial state done
    finished: float = 0.0
    step_latency: List[float] = field(default_factory=list)
    final: Optional[dict] = None
    error: Optional[str] = None


class Server:
    def __init__(self, hbm_budget: int, max_slots: int = 8, precision=MIXED,
                 steps: int = 100, scf_tol: Optional[float] = None,
                 verbose: bool = False):
        self.verbose = verbose
        self._done = 0
        self.budget = int(hbm_budget)
        self.max_slots = int(max_slots)
        self.precision = precision
        self.steps = int(steps)
        self.scf_tol = scf_tol
        self._lock = threading.Condition()
        self._used = 0
        self._active = 0
        self.peak_used = 0
        self.peak_active = 0

    def _worker(self, system, st: RequestStats, need: int, t0: float):
        try:
            g = XLBOMD(system, precision=self.precision, scf_tol=self.scf_tol)
            st.ready = time.perf_counter() - t0
            last = st.ready
            rep = None
            for _ in range(self.steps):
                rep = g.step(1, report=False)
                now = time.perf_counter() - t0
                st.step_latency.append(now - last)
                last = now
            n, q = g.charges()
            st.final = dict(q=q, n=n)
            g.close()
        except Exception as e:          # reported, never hidden
            st.error = repr(e)
        finally:
            st.finished = time.perf_counter() - t0
            with self._lock:
                self._used -= need
                self._active -= 1
                self._done += 1
                done = self._done
                self._lock.notify_all()
            if self.verbose:
                print(f"[serve] t={st.finished:7.2f}s done {done}: {st.name} "
                      f"({'error ' + st.error if st.error else 'ok'})",
                      file=sys.stderr, flush=True)

    def run(self, requests: Sequence[Tuple[float, object]], realtime=True):
        """Serve a stream of (arrival_s, System); returns (stats, summary)."""
        reqs = sorted(requests, key=lambda x: x[0])
        t0 = time.perf_counter()
        stats: List[RequestStats] = []
        threads = []
        for arrival, system in reqs:
            need = footprint_bytes(system, self.precision)
            if need > self.budget:
                raise ValueError(f"{system.name} needs {need} bytes > budget")
            st = RequestStats(name=system.name,
                              n_orb_total=system.n_atoms * system.n_orb,
                              arrival=arrival)
            stats.append(st)
            if realtime:
                wait = arrival - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(wait)
            with self._lock:
                while (self._used + need > self.budget
                       or self._active >= self.max_slots):
                    self._lock.wait()
                self._used += need
                self._active += 1
                self.peak_used = max(self.peak_used, self._used)
                self.peak_active = max(self.peak_active, self._active)
            st.admitted = time.perf_counter() - t0
            th = threading.Thread(target=self._worker,
                                  args=(system, st, need, t0), daemon=True)
            th.start()
            threads.append(th)
        for th in threads:
            th.join()
        wall = time.perf_counter() - t0
        lat = np.array([x for s in stats for x in s.step_latency])
        queue = np.array([s.admitted - s.arrival for s in stats])
        summary = dict(
            requests=len(stats), errors=sum(1 for s in stats if s.error),
            wall_s=wall, total_steps=int(lat.size),
            steps_per_s=lat.size / wall if wall > 0 else 0.0,
            p50_step_ms=float(np.percentile(lat, 50) * 1e3) if lat.size else None,
            p99_step_ms=float(np.percentile(lat, 99) * 1e3) if lat.size else None,
            p50_queue_ms=float(np.percentile(queue, 50) * 1e3),
            p99_queue_ms=float(np.percentile(queue, 99) * 1e3),
            peak_hbm_bytes=self.peak_used, hbm_budget=self.budget,
            peak_active=self.peak_active)
        return stats, summary
