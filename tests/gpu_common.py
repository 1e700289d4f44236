"""Helpers shared by the GPU parity tests: run the HIP path and the CPU oracle
on the same seeded inputs and compare them element by element."""
from __future__ import annotations

import os
import sys

import numpy as np

import oracle

ORACLE_THREADS = max(1, min(16, os.cpu_count() or 1))


def announce(*what):
    """Name the case before a GPU step, so a fault can be traced to it."""
    print("[gpu-case]", *what, flush=True)
    sys.stdout.flush()


def to_np(t):
    if t is None:
        return None
    a = t.cpu().numpy()
    return a.view(np.uint64) if a.dtype == np.int64 else a


def gpu_eval(ctx, mat, offs, cols, *, include=False, negative=True, masks=True):
    import torch
    pop = ctx.population(offsets=offs, cols=cols)
    out = ctx.eval(mat, pop, include=include, negative=negative, masks=masks)
    torch.cuda.synchronize()
    return tuple(to_np(t) for t in out)


def oracle_eval(X, offs, cols, *, include=False, negative=True, masks=True,
                sentinel=float("nan"), fill=0.0):
    return oracle.eval_population(X, offs, cols, include=include, negative=negative,
                                  sentinel=sentinel, fill=fill, masks=masks,
                                  threads=ORACLE_THREADS)


def assert_same(got, want, what=""):
    """Bit-exact: counts and mask words must be identical."""
    gm, gn, gmm, gnm = got
    om, on, omm, onm = want
    n = om.size
    if not np.array_equal(gm, om):
        bad = np.nonzero(gm != om)[0][:8]
        raise AssertionError(f"{what}: matched differs at {bad.tolist()} "
                             f"gpu={gm[bad].tolist()} oracle={om[bad].tolist()} (n={n})")
    if gn is not None and not np.array_equal(gn, on):
        bad = np.nonzero(gn != on)[0][:8]
        raise AssertionError(f"{what}: negative differs at {bad.tolist()} "
                             f"gpu={gn[bad].tolist()} oracle={on[bad].tolist()}")
    if gmm is not None and omm is not None:
        if not np.array_equal(gmm, omm):
            bad = np.argwhere(gmm != omm)[:8]
            raise AssertionError(f"{what}: matched mask differs at {bad.tolist()}")
        if not np.array_equal(gnm, onm):
            bad = np.argwhere(gnm != onm)[:8]
            raise AssertionError(f"{what}: negative mask differs at {bad.tolist()}")
