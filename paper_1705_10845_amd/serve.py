"""Continuous-batching server for independent XL-BOMD systems on one GPU.

Requests (a System and an arrival time) are admitted while their estimated
HBM footprint fits the budget and a slot is free.  An admitted system is set
up (ground state by the kernel SCF) by a worker thread, then joins the
running set: its whole state stays resident on the device (its library
handle) and it steps on its own stream, each system's next step starting
as soon as its last one is done, so the device overlaps the steps of every
running system and a small system is never held back by a large one.  Two
ways of stepping:

  step_mode 0 (default): steps with host decisions, each taken by a worker
      thread of its own system;
  step_mode 2: planned steps (every decision on the device), each replayed
      from the system's captured HIP graph, all enqueued and polled by the
      one host thread that runs the loop.

Step mode 0 serves the 16-512-atom stream faster: a planned step always
launches its rerun expansion (returning at once when no rerun is needed),
and these steps are bound by the GPU, not by the host.  Requests that
arrive while others run are admitted as slots and memory free up.
Per-step latency (completion of step s minus completion of step s-1, or of
the initial state for s = 1) and the queueing delay (arrival to admission)
are recorded.

Only scheduling lives here; every step runs in the HIP library.
"""
from __future__ import annotations

import sys
import time
from collections import deque
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

from .binding import MIXED, MIXED_BF16X3, MIXED_BF16, FP32, FP64, XLBOMD

_ESZ = {FP64: (8, 8), FP32: (4, 4), MIXED: (8, 4), MIXED_BF16X3: (8, 4), MIXED_BF16: (8, 4)}


def footprint_bytes(system, precision=MIXED, levels=10, planned=True) -> int:
    """Upper estimate of the device memory one system holds (no energy
    evaluation, which the server does not request).

    Expansion matrices: Z_0..Z_L, Y_0..Y_{L-1}, A_0..A_{L-1}, the seed
    powers Y, Y^2, Y^3 and four work matrices; responses: three matrices per
    direction (nine on the split path: four work matrices, the split rows
    of Y D, Y^2 D, Y^3 D and the FP64 Y D Y^3), plus the response-precision
    copies of the expansion operands (Z, Y, Y..Y^4) when the two precisions
    differ, and on the split path the split Y, Y^2, Y^3, Z_L^2 and four
    level work matrices.  Planned steps hold a second set of the expansion
    buffers (the rerun at the corrected chemical potential) and Z_L^3.  A
    non-orthogonal basis adds eight FP64 matrices (S, S^-1/2, S^1/2, H, H',
    D', two work matrices) and a fourth response batch buffer.
    """
    n = system.n_atoms * system.n_orb
    npad = -(-n // 128) * 128
    ef, er = _ESZ[precision]
    m = max(1, system.rank)
    mats_f = 3 * levels + 8
    if precision in (MIXED_BF16X3, MIXED_BF16):
        mats_r = 9 * m + 2 * levels + 13
        set_r = 2 * levels + 9
    else:
        mats_r = 3 * m + ((2 * levels + 5) if ef != er else 0)
        set_r = (2 * levels + 5) if ef != er else 0
    if planned:
        mats_f += 3 * levels + 8
        mats_r += set_r
    if getattr(system, "overlap_block", None) is not None:
        mats_f += 8
        mats_r += m
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


@dataclass
class _Running:
    g: XLBOMD
    st: RequestStats
    need: int
    done: int = 0
    last: float = 0.0
    fut: object = None     # step with host decisions in flight (step mode 0)


class Server:
    def __init__(self, hbm_budget: int, max_slots: int = 8, precision=MIXED,
                 steps: int = 100, scf_tol: Optional[float] = None,
                 verbose: bool = False, step_mode: int = 0, init_workers: int = 4):
        self.verbose = verbose
        self.budget = int(hbm_budget)
        self.max_slots = int(max_slots)
        self.precision = precision
        self.steps = int(steps)
        self.scf_tol = scf_tol
        self.step_mode = int(step_mode)
        self.init_workers = int(init_workers)
        self.peak_used = 0
        self.peak_active = 0
        # planned-step counters summed over the finished systems
        self.plan_stats = {"planned": 0, "replays": 0, "captures": 0, "fallbacks": 0}

    def _init(self, system):
        g = XLBOMD(system, precision=self.precision, scf_tol=self.scf_tol)
        if self.step_mode:
            g.set_step_mode(self.step_mode)
        return g

    def run(self, requests: Sequence[Tuple[float, object]], realtime=True):
        """Serve a stream of (arrival_s, System); returns (stats, summary)."""
        reqs = sorted(requests, key=lambda x: x[0])
        stats: List[RequestStats] = []
        queue = deque()
        for arrival, system in reqs:
            need = footprint_bytes(system, self.precision, planned=self.step_mode != 0)
            if need > self.budget:
                raise ValueError(f"{system.name} needs {need} bytes > budget")
            st = RequestStats(name=system.name, n_orb_total=system.n_atoms * system.n_orb,
                              arrival=arrival)
            stats.append(st)
            queue.append((arrival, system, st, need))
        used = 0
        starting = []                       # (future, st, need)
        running: List[_Running] = []
        pool = ThreadPoolExecutor(max_workers=self.init_workers)
        # step mode 0 (host decisions, a host synchronisation per decision):
        # each running system's step is taken by a worker thread
        steppers = None if self.step_mode else ThreadPoolExecutor(max_workers=self.max_slots)

        def begin(r):
            if steppers is None:
                r.g.step_begin()
            else:
                r.fut = steppers.submit(r.g.step, 1, False)

        def end(r):
            if steppers is None:
                return bool(r.g.step_end(wait=False))
            if not r.fut.done():
                return False
            r.fut.result()
            return True

        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0   # noqa: E731

        def retire(st, need, g=None):
            nonlocal used
            if g is not None:
                try:
                    g.close()
                except Exception as e:      # reported, never hidden
                    st.error = st.error or repr(e)
            used -= need
            st.finished = now()
            if self.verbose:
                print(f"[serve] t={st.finished:7.2f}s done: {st.name} "
                      f"({'error ' + st.error if st.error else 'ok'})", file=sys.stderr, flush=True)

        try:
            while queue or starting or running:
                progressed = False
                # admission: arrived, fits the budget, a slot is free
                while queue:
                    arrival, system, st, need = queue[0]
                    if realtime and arrival > now():
                        break
                    if used + need > self.budget or \
                            len(starting) + len(running) >= self.max_slots:
                        break
                    queue.popleft()
                    used += need
                    st.admitted = now()
                    starting.append((pool.submit(self._init, system), st, need))
                    self.peak_used = max(self.peak_used, used)
                    self.peak_active = max(self.peak_active, len(starting) + len(running))
                    progressed = True
                # systems whose initial state is ready start stepping
                for item in list(starting):
                    fut, st, need = item
                    if not fut.done():
                        continue
                    starting.remove(item)
                    progressed = True
                    try:
                        g = fut.result()
                    except Exception as e:
                        st.error = repr(e)
                        retire(st, need)
                        continue
                    st.ready = now()
                    r = _Running(g=g, st=st, need=need, last=st.ready)
                    try:
                        begin(r)
                        running.append(r)
                    except Exception as e:
                        st.error = repr(e)
                        retire(st, need, g)
                # poll running steps; start each system's next step at once
                for r in list(running):
                    try:
                        if not end(r):
                            continue
                        t = now()
                        r.st.step_latency.append(t - r.last)
                        r.last = t
                        r.done += 1
                        progressed = True
                        if r.done < self.steps:
                            begin(r)
                            continue
                        n, q = r.g.charges()
                        r.st.final = dict(q=q, n=n)
                        if self.step_mode:
                            for k, v in r.g.step_stats().items():
                                if k in self.plan_stats:
                                    self.plan_stats[k] += int(v)
                    except Exception as e:
                        r.st.error = repr(e)
                    running.remove(r)
                    retire(r.st, r.need, r.g)
                if not progressed:
                    time.sleep(20e-6)
        finally:
            pool.shutdown(wait=True)
            if steppers is not None:
                steppers.shutdown(wait=True)
        wall = now()
        lat = np.array([x for s in stats for x in s.step_latency])
        qd = np.array([s.admitted - s.arrival for s in stats])
        summary = dict(
            requests=len(stats), errors=sum(1 for s in stats if s.error),
            wall_s=wall, total_steps=int(lat.size),
            steps_per_s=lat.size / wall if wall > 0 else 0.0,
            p50_step_ms=float(np.percentile(lat, 50) * 1e3) if lat.size else None,
            p99_step_ms=float(np.percentile(lat, 99) * 1e3) if lat.size else None,
            p50_queue_ms=float(np.percentile(qd, 50) * 1e3),
            p99_queue_ms=float(np.percentile(qd, 99) * 1e3),
            peak_hbm_bytes=self.peak_used, hbm_budget=self.budget,
            peak_active=self.peak_active, step_mode=self.step_mode,
            plan_stats=dict(self.plan_stats) if self.step_mode else None)
        return stats, summary
