"""Serving: fitness-evaluation requests from many concurrent EBIC runs.

Many evolutionary runs share one GPU and a few resident matrices. Each run
submits one population evaluation per generation and waits for its counts
(the host-side evolutionary loop of the EBIC paper's Introduction; the
evaluation of Methods, "Handling missing values").

The scheduling runs in the library's native serving engine
(``ebic_server_*`` in include/ebic.h): admission against an HBM budget
(a device arena of exactly that size), continuous batching of waiting
requests onto stream slots (one ``ebic_eval_batch`` graph replay per batch,
one copy in and one copy out), a completion thread per slot and latency
accounting. This module only marshals arguments: ``submit`` hands the host
CSR and host output arrays to the engine and returns a future; one poller
thread turns completed tags into results.

Each request's counts and masks are exactly those of an evaluation of the
same population alone: the batched kernel runs the same per-item code, and
integer atomics make the accumulation order-independent.
"""
from __future__ import annotations

import concurrent.futures
import dataclasses
import itertools
import threading
import time
from typing import Dict, Optional

import numpy as np

from . import ebic


@dataclasses.dataclass
class Result:
    matched: np.ndarray
    negative: np.ndarray
    matched_mask: Optional[np.ndarray]
    negative_mask: Optional[np.ndarray]
    latency_s: float


@dataclasses.dataclass
class _Pending:
    future: concurrent.futures.Future
    keep: tuple                  # the arrays the engine reads or writes
    t_submit: float
    tag: int = 0


class Server:
    """Continuous-batching front end over one Context and its resident matrices."""

    def __init__(self, ctx: ebic.Context, hbm_budget_bytes: int = 1 << 30, slots: int = 4,
                 max_batch: int = 256):
        self.ctx = ctx
        self.budget = int(hbm_budget_bytes)
        self.handle = ebic.ebic_server_create(ctx.handle, self.budget, slots, max_batch)
        self._tags = itertools.count(1)
        self._pending: Dict[int, _Pending] = {}
        self._mu = threading.Lock()
        self._closing = False
        self._final_stats = None
        self._poller = threading.Thread(target=self._poll_loop, name="ebic-server-poll", daemon=True)
        self._poller.start()

    # -- client side ----------------------------------------------------------
    def request_bytes(self, matrix: int, n: int, nnz: int, masks: bool) -> int:
        """Device bytes a request holds while in flight (what admission counts):
        its CSR, both count arrays and, with masks, both mask arrays."""
        flags = ebic.Context.flags(False, True)
        return ebic.ebic_server_request_bytes(self.ctx.handle, matrix, n, nnz, flags, masks)

    def submit(self, run: int, matrix: int, offsets: np.ndarray, cols: np.ndarray,
               include: bool = False, negative: bool = True,
               masks: bool = False) -> concurrent.futures.Future:
        """Queue one population evaluation; the future yields a Result.
        Raises EbicError(EBIC_EBUDGET) for a request larger than the budget."""
        del run  # requests of all runs share the queue (FIFO)
        offsets = np.ascontiguousarray(offsets, dtype=np.int32)
        cols = np.ascontiguousarray(cols, dtype=np.int32)
        n = offsets.size - 1
        if n < 0:
            raise ValueError("offsets must have n + 1 entries")
        if n and (int(offsets.min()) < 0 or int(offsets.max()) > cols.size):
            raise ValueError("offsets reach outside the column array")
        rows, _ = self.ctx.matrices[matrix]
        words = ebic.ebic_mask_words(rows)
        # Like Context.eval: both count arrays, and both masks when asked for
        # (the negative ones are zero when negative trends are not counted).
        m = np.empty(n, np.int32)
        g = np.empty(n, np.int32)
        mm = np.empty((n, words), np.uint64) if masks else None
        nm = np.empty((n, words), np.uint64) if masks else None
        flags = ebic.Context.flags(include, negative)
        fut: concurrent.futures.Future = concurrent.futures.Future()
        tag = next(self._tags)
        ptr = lambda a: None if a is None else a.ctypes.data
        with self._mu:
            if self._closing:
                raise RuntimeError("server is closed")
            self._pending[tag] = _Pending(fut, (offsets, cols, m, g, mm, nm), time.perf_counter(), tag)
        fut.ebic_tag = tag  # (for cancel)
        try:
            ebic.ebic_server_submit(self.handle, matrix, n, offsets.ctypes.data,
                                    cols.ctypes.data if cols.size else None, flags, m.ctypes.data,
                                    ptr(g), ptr(mm), ptr(nm), tag)
        except Exception:
            with self._mu:
                self._pending.pop(tag, None)
            raise
        return fut

    def cancel(self, fut: concurrent.futures.Future) -> bool:
        """Cancel a request that has not been launched yet. True if it was
        (its future ends cancelled), False if it is already on the device
        or done (it then completes normally)."""
        try:
            ebic.ebic_server_cancel(self.handle, fut.ebic_tag)
            return True
        except ebic.EbicError as e:
            if e.status in (ebic.EBIC_EBUSY, ebic.EBIC_ENOENT):
                return False
            raise

    def pause(self, paused: bool = True) -> None:
        """Stop launching new batches (requests keep queueing), or resume."""
        ebic.ebic_server_set_paused(self.handle, paused)

    def _poll_loop(self):
        tags = np.zeros(256, np.uint64)
        sts = np.zeros(256, np.int32)
        while True:
            k = ebic.ebic_server_poll(self.handle, tags, sts, 20000)
            now = time.perf_counter()
            for i in range(k):
                with self._mu:
                    p = self._pending.pop(int(tags[i]))
                _, _, m, g, mm, nm = p.keep
                if sts[i] == ebic.EBIC_ECANCELED:
                    p.future.cancel()
                elif sts[i] != ebic.EBIC_OK:
                    p.future.set_exception(ebic.EbicError(int(sts[i]), "batch launch failed"))
                else:
                    p.future.set_result(Result(m, g, mm, nm, now - p.t_submit))
            with self._mu:
                if self._closing and not self._pending:
                    return

    def close(self):
        """Complete every submitted request, then stop the engine."""
        if self.handle is None:
            return
        with self._mu:
            self._closing = True
        self._poller.join()
        self._final_stats = self._raw_stats()
        ebic.ebic_server_destroy(self.handle)
        self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _raw_stats(self, reset: bool = False):
        st = ebic.ebic_server_get_stats(self.handle, reset)
        return {"completed": st.completed, "batches": st.batches, "pending": st.pending,
                "p50_ms": st.latency_p50_ms, "p99_ms": st.latency_p99_ms,
                "max_ms": st.latency_max_ms, "graph_captures": st.graph_captures,
                "staging_grows": st.staging_grows, "queue_p99_ms": st.queue_p99_ms,
                "mean_batch": st.mean_batch,
                "admitted_bytes_high_water": st.high_water_bytes,
                "reserved_bytes": st.reserved_bytes, "budget_bytes": st.budget_bytes,
                "checks": st.nominal_checks, "cancelled": st.cancelled}

    def stats(self, reset: bool = False) -> Dict[str, float]:
        """Engine counters (latency from submission to completion in the
        engine); reset=True starts a new measurement window."""
        if self.handle is None:
            return dict(self._final_stats or {})
        return self._raw_stats(reset)

    @property
    def high_water(self) -> int:
        return int(self.stats()["admitted_bytes_high_water"])
