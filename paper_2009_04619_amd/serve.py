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
members take exactly the steps and arithmetic of a solo run.  Set-up and
read-out of requests overlap with the blocks running on the GPU.
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
    on the CPU with a fake).

    start     allocate a request and add it to the batch of its storage type
    launch    enqueue up to n steps for every admitted request, return a token
    wait      block until the launch behind a token has completed
    remaining steps a request has left after everything launched so far
    detach    take a request with no steps left out of its batch (no wait)
    finish    read a detached request out and release it (after the launch
              that completed it has been waited for)
    """

    def bytes_for(self, req: Request) -> int:
        raise NotImplementedError

    def admit(self, req: Request, in_use: int, budget: int):
        """(status, bytes, fits now) under the budget, with the library's
        status codes: WAVE_OK (admissible; `fits now` says whether beside
        `in_use`), WAVE_EBUDGET (larger than the whole budget), WAVE_EINVAL."""
        nb = int(self.bytes_for(req))
        if nb <= 0:
            return W.WAVE_EINVAL, 0, False
        if nb > budget:
            return W.WAVE_EBUDGET, nb, False
        return W.WAVE_OK, nb, in_use + nb <= budget

    def start(self, req: Request) -> None:
        raise NotImplementedError

    def launch(self, n: int):
        raise NotImplementedError

    def wait(self, token) -> None:
        raise NotImplementedError

    def remaining(self, req: Request) -> int:
        raise NotImplementedError

    def detach(self, req: Request) -> None:
        raise NotImplementedError

    def finish(self, req: Request, keep_field: bool) -> None:
        raise NotImplementedError


class GpuExecutor(Executor):
    """Batches per storage type on the caller's stream; set-up and read-out
    of requests on a stream of their own, so that they overlap with the
    blocks the batches are running (the library orders the two with
    events).

    `tiles` gives each storage type's batch sweep tile as
    wave_batch_set_kernel takes it; the defaults are what the batch tuner
    picked for mixed 128-384^3 shots on MI355X (one point per lane, 64 x 8,
    for float32; two points per lane, 128 x 8, for 16-bit storage)."""

    TILES = {"f32": (1, 8), "bf16": (0, 8), "f16": (0, 8)}

    def __init__(self, device="cuda:0", graph_steps=0, max_shots=128, tiles=None):
        import torch
        self.torch = torch
        self.device = device
        self.graph_steps = graph_steps
        self.max_shots = max_shots
        self.tiles = dict(self.TILES, **(tiles or {}))
        self.batches: Dict[str, W.Batch] = {}
        self.shots: Dict[int, W.Shot] = {}
        self.run_stream = torch.cuda.current_stream(device)
        self.io_stream = torch.cuda.Stream(device=device)

    def _desc(self, req: Request):
        s = req.shot
        nrec = 0 if s.rec is None else len(s.rec)
        return W.make_desc(s.nx, s.ny, s.nz, s.w, s.dx, s.dy, s.dz, s.dt, req.storage,
                           max_src=max(1, len(s.src)), max_rec=nrec, max_steps=int(s.steps))

    def bytes_for(self, req: Request) -> int:
        return W.wave_bytes_required(self._desc(req))

    def admit(self, req: Request, in_use: int, budget: int):
        return W.wave_admit(self._desc(req), budget, in_use)

    def _batch(self, storage: str) -> W.Batch:
        b = self.batches.get(storage)
        if b is None:
            b = W.Batch(storage=storage, max_shots=self.max_shots, device=self.device,
                        stream=self.run_stream)
            b.set_graph(self.graph_steps)
            b.set_kernel(*self.tiles[storage])
            self.batches[storage] = b
        return b

    def start(self, req: Request) -> None:
        sh = W.shot_from_synth(req.shot, storage=req.storage, device=self.device,
                               stream=self.io_stream)
        self._batch(req.storage).add(sh, int(req.shot.steps))
        self.shots[req.rid] = sh

    def launch(self, n: int):
        for b in self.batches.values():
            if b.members:
                b.run(n)
        ev = self.torch.cuda.Event()
        ev.record(self.run_stream)      # the caller's stream waits on every run
        return ev

    def wait(self, token) -> None:
        token.synchronize()

    def remaining(self, req: Request) -> int:
        sh = self.shots[req.rid]
        b = self.batches[req.storage]
        return b.remaining(sh) if sh in b.members else 0

    def detach(self, req: Request) -> None:
        self.batches[req.storage].remove(self.shots[req.rid])

    def finish(self, req: Request, keep_field: bool) -> None:
        sh = self.shots.pop(req.rid)
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
    latencies.  A request larger than the whole budget is rejected
    (WAVE_EBUDGET from the executor's admission check).

    The loop keeps one block in flight: it admits what has arrived, enqueues
    the next block, takes the requests that this block completes out of
    their batches, and only then waits for the previous block and reads out
    the requests it completed, so the GPU has queued work while the host
    does set-up and read-out.  A finished request holds its memory until it
    has been read out."""

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
        inflight = None                  # (token, requests that block completes)
        t0 = self.clock()
        now = lambda: (self.clock() - t0) / time_scale
        while pending or waiting or active or inflight is not None:
            t = now()
            while pending and pending[0].arrival <= t:
                waiting.append(pending.popleft())
            # admit in arrival order while the budget allows (no overtaking)
            while waiting:
                r = waiting[0]
                rc, nb, fits = self.ex.admit(r, self.in_use, self.budget)
                if rc != W.WAVE_OK:
                    waiting.popleft()
                    r.error = f"rejected: {W.wave_strerror(rc)}"
                    r.finished = now()
                    done.append(r)
                    continue
                if not fits:
                    break
                waiting.popleft()
                self.ex.start(r)
                sizes[r.rid] = nb
                self.in_use += nb
                self.peak_in_use = max(self.peak_in_use, self.in_use)
                r.admitted = now()
                active.append(r)
                self.log.append(("admit", r.rid, r.admitted, self.in_use))
            launched = None
            if active:
                token = self.ex.launch(self.block)
                ending = [r for r in active if self.ex.remaining(r) == 0]
                for r in ending:
                    self.ex.detach(r)
                    active.remove(r)
                launched = (token, ending)
            if inflight is not None:
                token, ending = inflight
                self.ex.wait(token)
                for r in ending:
                    self.ex.finish(r, keep_field=r.rid in keep_fields)
                    r.finished = now()
                    self.in_use -= sizes.pop(r.rid)
                    done.append(r)
                    self.log.append(("finish", r.rid, r.finished, self.in_use))
            inflight = launched
            if not active and inflight is None and not waiting and pending:
                self.sleep(max(0.0, (pending[0].arrival - now()) * time_scale))
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
