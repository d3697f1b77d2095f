"""Continuous-batching service for shot simulations on one GPU.

Requests (grid, model, source, receivers, step count, storage type) arrive
over time.  The loop admits a request as soon as its device arena fits the
HBM budget (sized with `wave_bytes_required`), adds it to the running batch
of its storage type, and keeps advancing every batch by blocks of steps; a
request that arrives while others are on the GPU joins at the next block, and
a finished one is read out and its memory released right away.  All
numerical work happens in the HIP library through `wave`; this module only
schedules.

A request's result is identical to a run of the same shot on its own: batch
members take exactly the steps and arithmetic of a solo run.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Dict, List, Optional

import numpy as np

from . import wave as W


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float            # seconds from the start of the run
    shot: object              # a synth.Shot-like object (grid, vel, src, wavelet, rec, steps)
    storage: str = "f32"
    # filled in by the server
    admitted: Optional[float] = None
    finished: Optional[float] = None
    traces: Optional[np.ndarray] = None
    field: Optional[np.ndarray] = None
    error: Optional[str] = None

    @property
    def latency(self) -> Optional[float]:
        return None if self.finished is None else self.finished - self.arrival

    @property
    def points(self) -> int:
        s = self.shot
        return int(s.nx) * int(s.ny) * int(s.nz)


class Executor:
    """The device side of the server (a seam so that scheduling can be tested
    on the CPU with a fake).  `start` allocates and admits a request into its
    batch, `advance` runs every batch by up to n steps and waits, `remaining`
    and `finish` read a request out and release it."""

    def bytes_for(self, req: Request) -> int:
        raise NotImplementedError

    def start(self, req: Request) -> None:
        raise NotImplementedError

    def advance(self, n: int) -> None:
        raise NotImplementedError

    def remaining(self, req: Request) -> int:
        raise NotImplementedError

    def finish(self, req: Request, keep_field: bool) -> None:
        raise NotImplementedError


class GpuExecutor(Executor):
    def __init__(self, device="cuda:0", graph_steps=0, max_shots=128):
        import torch
        self.torch = torch
        self.device = device
        self.graph_steps = graph_steps
        self.max_shots = max_shots
        self.batches: Dict[str, W.Batch] = {}
        self.shots: Dict[int, W.Shot] = {}

    def bytes_for(self, req: Request) -> int:
        s = req.shot
        nrec = 0 if s.rec is None else len(s.rec)
        d = W.make_desc(s.nx, s.ny, s.nz, s.w, s.dx, s.dy, s.dz, s.dt, req.storage,
                        max_src=max(1, len(s.src)), max_rec=nrec, max_steps=int(s.steps))
        return W.wave_bytes_required(d)

    def _batch(self, storage: str) -> W.Batch:
        b = self.batches.get(storage)
        if b is None:
            b = W.Batch(storage=storage, max_shots=self.max_shots, device=self.device)
            b.set_graph(self.graph_steps)
            self.batches[storage] = b
        return b

    def start(self, req: Request) -> None:
        sh = W.shot_from_synth(req.shot, storage=req.storage, device=self.device)
        self._batch(req.storage).add(sh, int(req.shot.steps))
        self.shots[req.rid] = sh

    def advance(self, n: int) -> None:
        for b in self.batches.values():
            if b.members:
                b.run(n)
        self.torch.cuda.synchronize(self.device)

    def remaining(self, req: Request) -> int:
        sh = self.shots[req.rid]
        return self.batches[req.storage].remaining(sh)

    def finish(self, req: Request, keep_field: bool) -> None:
        sh = self.shots.pop(req.rid)
        self.batches[req.storage].remove(sh)
        req.traces = sh.traces()
        if keep_field:
            req.field = sh.read(W.WAVE_FIELD_U)
        sh.close()

    def close(self):
        for b in self.batches.values():
            b.close()
        self.batches.clear()


class Server:
    """Continuous batching under an HBM budget.

    run(requests) replays the requests' arrival times against the wall clock
    (time_scale < 1 compresses them) and returns the requests with their
    latencies.  A request larger than the whole budget is rejected."""

    def __init__(self, executor: Executor, budget_bytes: int, block_steps: int = 50,
                 clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.block = int(block_steps)
        self.clock = clock
        self.sleep = sleep
        self.in_use = 0
        self.peak_in_use = 0
        self.log: List[tuple] = []

    def run(self, requests: List[Request], time_scale: float = 1.0, keep_fields=()) -> List[Request]:
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting: collections.deque = collections.deque()   # arrived, not admitted
        active: List[Request] = []
        sizes: Dict[int, int] = {}
        done: List[Request] = []
        t0 = self.clock()
        now = lambda: (self.clock() - t0) / time_scale
        while pending or waiting or active:
            t = now()
            while pending and pending[0].arrival <= t:
                waiting.append(pending.popleft())
            # admit in arrival order while the budget allows (no overtaking)
            while waiting:
                r = waiting[0]
                nb = self.ex.bytes_for(r)
                if nb == 0 or nb > self.budget:
                    waiting.popleft()
                    r.error = "rejected: larger than the memory budget"
                    r.finished = now()
                    done.append(r)
                    continue
                if self.in_use + nb > self.budget:
                    break
                waiting.popleft()
                self.ex.start(r)
                sizes[r.rid] = nb
                self.in_use += nb
                self.peak_in_use = max(self.peak_in_use, self.in_use)
                r.admitted = now()
                active.append(r)
                self.log.append(("admit", r.rid, r.admitted, self.in_use))
            if not active:
                if pending:
                    self.sleep(max(0.0, (pending[0].arrival - now()) * time_scale))
                continue
            self.ex.advance(self.block)
            for r in list(active):
                if self.ex.remaining(r) == 0:
                    self.ex.finish(r, keep_field=r.rid in keep_fields)
                    r.finished = now()
                    active.remove(r)
                    self.in_use -= sizes.pop(r.rid)
                    done.append(r)
                    self.log.append(("finish", r.rid, r.finished, self.in_use))
        return sorted(done, key=lambda r: r.rid)


def summarize(done: List[Request], wall: float) -> dict:
    ok = [r for r in done if r.error is None]
    lat = np.array([r.latency for r in ok]) if ok else np.zeros(1)
    pts = sum(r.points * int(r.shot.steps) for r in ok)
    return {
        "requests": len(done), "served": len(ok), "rejected": len(done) - len(ok),
        "wall_s": round(wall, 3),
        "shots_per_s": round(len(ok) / wall, 3) if wall > 0 else None,
        "gpoints_per_s": round(pts / wall / 1e9, 3) if wall > 0 else None,
        "p50_s": round(float(np.percentile(lat, 50)), 4),
        "p99_s": round(float(np.percentile(lat, 99)), 4),
    }
