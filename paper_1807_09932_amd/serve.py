"""Serving: fitness-evaluation requests from many concurrent EBIC runs.

Many evolutionary runs share one GPU and a few resident matrices. Each run
submits one population evaluation per generation and waits for its counts
(the host-side evolutionary loop of the EBIC paper's Introduction; the
evaluation of Methods, "Handling missing values").

The server does continuous batching:

* Admission. A request reserves the device bytes it will hold: its CSR
  population, its outputs, and its masks if asked for. It is admitted only
  while the reserved total stays within the HBM budget. A request larger than
  the whole budget is refused at submission with EBIC_EBUDGET.
* Launch. Each admitted request's population is copied to the device on a
  free stream slot. Whenever a slot is free, every admitted request waiting
  for one is launched there as one batch: one ebic_eval_batch call, one HIP
  graph replay. Requests that arrive while other batches run on other slots
  are admitted and launched as soon as a slot and memory free up, so their
  work overlaps on the device.
* Completion. When a slot's batch has finished (its event has completed), its
  results go back to the host, each request's future is completed, its latency
  is recorded, and its reservation and slot are released.

Each request's counts and masks are exactly those of an evaluation of the
same population alone: the batched kernel runs the same per-item code, and
integer atomics make the accumulation order-independent.
"""
from __future__ import annotations

import concurrent.futures
import dataclasses
import threading
import time
from collections import deque
from typing import Deque, Dict, List, Optional

import numpy as np
import torch

from . import ebic


@dataclasses.dataclass
class Result:
    matched: np.ndarray
    negative: np.ndarray
    matched_mask: Optional[np.ndarray]
    negative_mask: Optional[np.ndarray]
    latency_s: float


@dataclasses.dataclass
class _Req:
    run: int
    matrix: int
    offsets: np.ndarray
    cols: np.ndarray
    include: bool
    negative: bool
    masks: bool
    bytes: int
    future: concurrent.futures.Future
    t_submit: float
    n: int = 0
    checks: int = 0
    # device state once admitted
    pop: Optional[ebic.Population] = None
    out: Optional[tuple] = None


class _Slot:
    def __init__(self, device):
        self.stream = torch.cuda.Stream(device=device)  # default priority
        self.event: Optional[torch.cuda.Event] = None
        self.batch: List[_Req] = []

    @property
    def busy(self) -> bool:
        return bool(self.batch)


class Server:
    """Continuous-batching front end over one Context and its resident matrices."""

    def __init__(self, ctx: ebic.Context, hbm_budget_bytes: int = 1 << 30, slots: int = 4,
                 max_batch: int = 256):
        self.ctx = ctx
        self.budget = int(hbm_budget_bytes)
        self.reserved = 0
        self.high_water = 0
        self.max_batch = max_batch
        self.slots = [_Slot(ctx.device) for _ in range(max(1, slots))]
        self._waiting: Deque[_Req] = deque()     # submitted, not yet admitted
        self._admitted: Deque[_Req] = deque()    # on the device, not yet launched
        self._cv = threading.Condition()
        self._stop = False
        self._thread = threading.Thread(target=self._loop, name="ebic-server", daemon=True)
        self.latencies: List[float] = []
        self.completed = 0
        self.checks_done = 0
        self.batches = 0
        self._thread.start()

    # -- client side ----------------------------------------------------------
    def request_bytes(self, matrix: int, n: int, nnz: int, masks: bool) -> int:
        rows, _ = self.ctx.matrices[matrix]
        words = ebic.ebic_mask_words(rows)
        b = 4 * (n + 1) + 4 * max(1, nnz) + 8 * n
        if masks:
            b += 2 * 8 * n * words
        return b

    def submit(self, run: int, matrix: int, offsets: np.ndarray, cols: np.ndarray,
               include: bool = False, negative: bool = True,
               masks: bool = False) -> concurrent.futures.Future:
        """Queue one population evaluation; the future yields a Result."""
        offsets = np.ascontiguousarray(offsets, dtype=np.int32)
        cols = np.ascontiguousarray(cols, dtype=np.int32)
        n = offsets.size - 1
        if offsets.size < 1 or int(offsets.min()) < 0 or int(offsets.max()) > cols.size:
            raise ValueError("offsets reach outside the column array")
        nbytes = self.request_bytes(matrix, n, cols.size, masks)
        if nbytes > self.budget:
            raise ebic.EbicError(ebic.EBIC_EBUDGET,
                                 f"request needs {nbytes} bytes, budget is {self.budget}")
        rows, _ = self.ctx.matrices[matrix]
        fut: concurrent.futures.Future = concurrent.futures.Future()
        r = _Req(run, matrix, offsets, cols, include, negative, masks, nbytes, fut,
                 time.perf_counter(), n=n, checks=rows * int(offsets[-1]))
        with self._cv:
            if self._stop:
                raise RuntimeError("server is closed")
            self._waiting.append(r)
            self._cv.notify()
        return fut

    def close(self, wait: bool = True):
        with self._cv:
            self._stop = True
            self._cv.notify()
        if wait:
            self._thread.join()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def stats(self) -> Dict[str, float]:
        lat = np.array(self.latencies) if self.latencies else np.zeros(1)
        return {"completed": self.completed, "batches": self.batches,
                "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3),
                "mean_batch": self.completed / max(1, self.batches),
                "admitted_bytes_high_water": self.high_water,
                "checks": self.checks_done}

    # -- scheduler ------------------------------------------------------------
    def _admit(self) -> bool:
        """Move waiting requests onto the device while the budget allows."""
        moved = False
        while self._waiting and self.reserved + self._waiting[0].bytes <= self.budget:
            r = self._waiting.popleft()
            self.reserved += r.bytes
            self.high_water = max(self.high_water, self.reserved)
            self._admitted.append(r)
            moved = True
        return moved

    def _launch(self, slot: _Slot):
        batch = []
        while self._admitted and len(batch) < self.max_batch:
            batch.append(self._admitted.popleft())
        if not batch:
            return
        with torch.cuda.stream(slot.stream):
            reqs = []
            for r in batch:
                r.pop = self.ctx.population(offsets=r.offsets, cols=r.cols)
                r.out = self.ctx.outputs(r.matrix, r.n, masks=r.masks, negative=True)
                reqs.append(self.ctx.request(r.matrix, r.pop, r.out, include=r.include,
                                             negative=r.negative))
            self.ctx.eval_batch(reqs, stream=slot.stream)
            ev = torch.cuda.Event()
            ev.record(slot.stream)
        slot.event = ev
        slot.batch = batch
        self.batches += 1

    def _complete(self, slot: _Slot):
        now = time.perf_counter()
        for r in slot.batch:
            m, g, mm, nm = r.out
            res = Result(m.cpu().numpy(), g.cpu().numpy(),
                         None if mm is None else mm.cpu().numpy().view(np.uint64),
                         None if nm is None else nm.cpu().numpy().view(np.uint64),
                         now - r.t_submit)
            self.reserved -= r.bytes
            self.latencies.append(res.latency_s)
            self.completed += 1
            self.checks_done += r.checks
            r.pop = r.out = None
            r.future.set_result(res)
        slot.batch = []
        slot.event = None

    def _loop(self):
        torch.cuda.set_device(self.ctx.device)
        while True:
            with self._cv:
                progressed = self._admit()
                free = [s for s in self.slots if not s.busy]
                if self._admitted and free:
                    self._launch(free[0])
                    progressed = True
                for s in self.slots:
                    if s.busy and s.event.query():
                        self._complete(s)
                        progressed = True
                        self._admit()
                idle = not self._waiting and not self._admitted and \
                    not any(s.busy for s in self.slots)
                if self._stop and idle:
                    return
                if not progressed:
                    if idle:
                        self._cv.wait(timeout=0.05)
                    else:
                        self._cv.wait(timeout=50e-6)
