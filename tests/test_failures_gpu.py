"""Error paths forced from the host (EBIC_FAULT), releases of matrices in
use, and serving-request cancellation. No kernel is made to fault: an
injected failure is raised on the host before anything is enqueued."""
import os
import threading

import numpy as np
import pytest

from paper_1807_09932_amd import gen
from tests.gpu_common import announce, assert_same, oracle_eval, to_np

pytestmark = pytest.mark.gpu


def _context(fault=None):
    from paper_1807_09932_amd.ebic import Context
    old = os.environ.pop("EBIC_FAULT", None)
    if fault:
        os.environ["EBIC_FAULT"] = fault
    try:
        return Context(0)  # the plan is read at creation
    finally:
        os.environ.pop("EBIC_FAULT", None)
        if old is not None:
            os.environ["EBIC_FAULT"] = old


def _small():
    w = gen.make_matrix(31, 3_001, 64, "beta", 3, (100, 300), (4, 8), directions="alternate")
    offs, cols = gen.csr(gen.make_population(31, 1, 64, 120, (1, 20), w.plants))
    return w.X, offs, cols


def _sentinel_outputs(torch, n, dev):
    return (torch.full((n,), 7, dtype=torch.int32, device=dev),
            torch.full((n,), 7, dtype=torch.int32, device=dev), None, None)


@pytest.mark.parametrize("after", range(0, 8))
def test_injected_allocation_failure_unwinds(after):
    """The (after+1)-th device allocation fails: upload or evaluation returns
    EBIC_ENOMEM, frees what it had allocated, and the next call succeeds."""
    import torch
    from paper_1807_09932_amd import ebic
    X, offs, cols = _small()
    dev = torch.device("cuda", 0)
    ctx = _context(f"alloc:{after}")
    try:
        torch.cuda.synchronize()
        base = torch.cuda.memory_allocated(dev)
        announce("alloc fault", after)
        try:
            mat = ctx.upload(X, fill=0.5, keep_fill_copy=True)
        except ebic.EbicError as e:
            assert e.status == ebic.EBIC_ENOMEM and "EBIC_FAULT" in str(e)
            torch.cuda.synchronize()
            assert torch.cuda.memory_allocated(dev) == base, "a failed upload leaked device memory"
            mat = ctx.upload(X, fill=0.5, keep_fill_copy=True)  # the fault fired once
        pop = ctx.population(offsets=offs, cols=cols)
        out = _sentinel_outputs(torch, pop.n, dev)
        try:
            ctx.eval(mat, pop, out=out)
        except ebic.EbicError as e:
            assert e.status == ebic.EBIC_ENOMEM
            torch.cuda.synchronize()
            assert int(out[0].min()) == 7 and int(out[0].max()) == 7  # nothing was enqueued
            ctx.eval(mat, pop, out=out)
        torch.cuda.synchronize()
        want = oracle_eval(X, offs, cols, masks=False)
        assert np.array_equal(to_np(out[0]), want[0]) and np.array_equal(to_np(out[1]), want[1])
        ctx.release(mat)
    finally:
        ctx.close()


@pytest.mark.parametrize("after", [0, 1])
def test_injected_launch_failure(after):
    """The (after+1)-th launch fails with EBIC_EHIP before anything is
    enqueued; earlier and later launches give the oracle's counts."""
    import torch
    from paper_1807_09932_amd import ebic
    X, offs, cols = _small()
    dev = torch.device("cuda", 0)
    ctx = _context(f"launch:{after}")
    try:
        mat = ctx.upload(X)
        pop = ctx.population(offsets=offs, cols=cols)
        want = oracle_eval(X, offs, cols, masks=False)
        failed = 0
        for call in range(3):
            out = _sentinel_outputs(torch, pop.n, dev)
            announce("launch fault", after, call)
            try:
                ctx.eval(mat, pop, out=out)
            except ebic.EbicError as e:
                assert e.status == ebic.EBIC_EHIP and "EBIC_FAULT" in ebic.ebic_last_error() + str(e)
                assert call == after
                failed += 1
                torch.cuda.synchronize()
                assert int(out[0].min()) == 7 and int(out[0].max()) == 7
                continue
            torch.cuda.synchronize()
            assert np.array_equal(to_np(out[0]), want[0])
        assert failed == 1
        # batched launches go through the same check
        ctx.close()
        ctx = _context("launch:0")
        mat = ctx.upload(X)
        pop = ctx.population(offsets=offs, cols=cols)
        o = ctx.outputs(mat, pop.n)
        with pytest.raises(ebic.EbicError) as e:
            ctx.eval_batch([ctx.request(mat, pop, o)])
        assert e.value.status == ebic.EBIC_EHIP
        ctx.eval_batch([ctx.request(mat, pop, o)])
        torch.cuda.synchronize()
        assert np.array_equal(to_np(o[0]), want[0])
    finally:
        ctx.close()


def test_release_waits_for_callers_and_refuses_while_held():
    """Evaluations on one thread and a release on another: every evaluation
    either returns the oracle's counts or finds the matrix gone (ENOENT);
    the release never frees memory a call has planned with."""
    import torch
    from paper_1807_09932_amd import ebic
    X, offs, cols = _small()
    want = oracle_eval(X, offs, cols, masks=False)
    ctx = _context()
    try:
        for trial in range(5):
            mat = ctx.upload(X)
            pop = ctx.population(offsets=offs, cols=cols)
            results, errors = [], []
            stop = threading.Event()

            out = ctx.outputs(mat, pop.n)

            def worker():
                s = torch.cuda.Stream()
                while not stop.is_set():
                    try:
                        ctx.eval(mat, pop, out=out, stream=s)
                    except ebic.EbicError as e:
                        errors.append(e.status)
                        return
                    s.synchronize()
                    results.append((to_np(out[0]), to_np(out[1])))

            th = threading.Thread(target=worker)
            th.start()
            announce("release race", trial)
            released = False
            for _ in range(2000):
                try:
                    ctx.release(mat)
                    released = True
                    break
                except ebic.EbicError as e:
                    assert e.status == ebic.EBIC_EBUSY
            stop.set()
            th.join(timeout=60)
            assert released
            assert all(st == ebic.EBIC_ENOENT for st in errors)
            for m, g in results:
                assert np.array_equal(m, want[0]) and np.array_equal(g, want[1])
    finally:
        ctx.close()


def test_server_cancel_pause_and_busy_release():
    """Paused server: queued requests hold their matrix (release returns
    EBIC_EBUSY), cancelled ones end with EBIC_ECANCELED and are not written,
    the rest complete bit-exact after the pause; then the release succeeds."""
    import concurrent.futures

    from paper_1807_09932_amd import ebic
    from paper_1807_09932_amd.serve import Server
    X, offs, cols = _small()
    want = oracle_eval(X, offs, cols, masks=False)
    ctx = _context()
    try:
        mat = ctx.upload(X)
        other = ctx.upload(X[:1000])
        with Server(ctx, hbm_budget_bytes=16 << 20, slots=2) as srv:
            srv.pause(True)
            futs = [srv.submit(0, mat, offs, cols) for _ in range(6)]
            with pytest.raises(ebic.EbicError) as e:
                ctx.release(mat)
            assert e.value.status == ebic.EBIC_EBUSY
            ctx.release(other)  # a matrix no request uses is released at once
            assert srv.cancel(futs[1]) and srv.cancel(futs[4])
            assert not srv.cancel(futs[1])  # already cancelled
            announce("server resume")
            srv.pause(False)
            for i, f in enumerate(futs):
                if i in (1, 4):
                    with pytest.raises(concurrent.futures.CancelledError):
                        f.result(timeout=60)
                    continue
                res = f.result(timeout=60)
                assert np.array_equal(res.matched, want[0]) and np.array_equal(res.negative, want[1])
            st = srv.stats()
            assert st["completed"] == 4 and st["cancelled"] == 2
        ctx.release(mat)  # nothing holds it any more
    finally:
        ctx.close()


def test_server_launch_failure_is_per_request():
    """An injected launch failure fails the requests of that batch with
    EBIC_EHIP; the server carries on and later requests are exact."""
    from paper_1807_09932_amd import ebic
    from paper_1807_09932_amd.serve import Server
    X, offs, cols = _small()
    want = oracle_eval(X, offs, cols, masks=False)
    ctx = _context("launch:0")
    try:
        mat = ctx.upload(X)
        with Server(ctx, hbm_budget_bytes=16 << 20, slots=1) as srv:
            f1 = srv.submit(0, mat, offs, cols)
            with pytest.raises(ebic.EbicError) as e:
                f1.result(timeout=60)
            assert e.value.status == ebic.EBIC_EHIP
            for _ in range(3):
                res = srv.submit(0, mat, offs, cols).result(timeout=60)
                assert np.array_equal(res.matched, want[0])
        ctx.release(mat)
    finally:
        ctx.close()
