"""The continuous-batching server: every request's result in the mix equals
the same request evaluated alone (bit-exact), and the HBM budget is honoured."""
import time

import numpy as np
import pytest

from paper_1807_09932_amd import gen
from tests.gpu_common import announce, assert_same, oracle_eval, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def served():
    from paper_1807_09932_amd.ebic import Context
    ctx = Context(0)
    ws = gen.served_matrices(scale=0.05)
    mats = [ctx.upload(w.X) for w in ws]
    pools = gen.served_pools(pool_size=6, n_range=(20, 200))
    yield ctx, ws, mats, pools
    ctx.close()


def _alone(ctx, mat, offs, cols, negative=True, masks=False, include=False):
    import torch
    pop = ctx.population(offsets=offs, cols=cols)
    out = ctx.eval(mat, pop, negative=negative, masks=masks, include=include)
    torch.cuda.synchronize()
    return tuple(to_np(t) for t in out)


def test_results_in_the_mix_equal_results_alone(served):
    from paper_1807_09932_amd.serve import Server
    ctx, ws, mats, pools = served
    reqs = gen.served_requests(0.2, rate_hz=1000.0, pool_size=6)[:150]
    announce("serve mix", len(reqs))
    with Server(ctx, hbm_budget_bytes=64 << 20, slots=3) as srv:
        # the first 60 queue behind a pause (so that mixed batches certainly
        # form when it ends); the rest arrive on the schedule
        srv.pause(True)
        t0 = time.perf_counter()
        futs = []
        for i, r in enumerate(reqs):
            if i == 60:
                srv.pause(False)
                t0 = time.perf_counter() - r.t_arrival
            while i >= 60 and time.perf_counter() - t0 < r.t_arrival:
                time.sleep(1e-4)
            offs, cols = pools[r.matrix][r.pool_index]
            futs.append(srv.submit(r.run, mats[r.matrix], offs, cols, negative=bool(i % 2),
                                   masks=(i % 5 == 0)))
        results = [f.result(timeout=60) for f in futs]
        stats = srv.stats()
    assert stats["completed"] == len(reqs)
    assert stats["batches"] < len(reqs)  # requests were batched together
    for i, (r, res) in enumerate(zip(reqs, results)):
        offs, cols = pools[r.matrix][r.pool_index]
        alone = _alone(ctx, mats[r.matrix], offs, cols, negative=bool(i % 2), masks=(i % 5 == 0))
        assert_same((res.matched, res.negative, res.matched_mask, res.negative_mask), alone,
                    f"request {i}")
    # and a sample against the oracle
    for i in (0, 7, 33):
        r = reqs[i]
        offs, cols = pools[r.matrix][r.pool_index]
        want = oracle_eval(ws[r.matrix].X, offs, cols, negative=bool(i % 2), masks=False)
        assert np.array_equal(results[i].matched, want[0])
        assert np.array_equal(results[i].negative, want[1])


def test_budget_refuses_oversized_and_serialises_tight(served):
    from paper_1807_09932_amd import ebic
    from paper_1807_09932_amd.serve import Server
    ctx, ws, mats, pools = served
    offs, cols = pools[3][0]
    with Server(ctx, hbm_budget_bytes=1000, slots=2) as srv:
        with pytest.raises(ebic.EbicError) as e:
            srv.submit(0, mats[3], offs, cols)
        assert e.value.status == ebic.EBIC_EBUDGET
    # a budget that fits only one request at a time still completes every request
    need = max(Server.request_bytes(srv, mats[m], p[0].size - 1, p[1].size, True)
               for m in range(4) for p in pools[m])
    announce("serve tight budget")
    with Server(ctx, hbm_budget_bytes=need, slots=2) as srv:
        futs = [srv.submit(j, mats[j % 4], *pools[j % 4][j % 6], masks=True) for j in range(12)]
        res = [f.result(timeout=60) for f in futs]
        assert srv.high_water <= need
    for j, r in enumerate(res):
        offs, cols = pools[j % 4][j % 6]
        assert_same((r.matched, r.negative, r.matched_mask, r.negative_mask),
                    _alone(ctx, mats[j % 4], offs, cols, masks=True), f"tight {j}")


def test_graph_captures_stay_one_per_slot():
    """Batches of any mix of population sizes over several matrices (all
    on the pair bitmaps, whose group size travels in the batch's arena)
    replay one captured graph per slot stream; every result equals the
    request evaluated alone."""
    import torch
    from paper_1807_09932_amd.ebic import Context
    from paper_1807_09932_amd.serve import Server
    rng = np.random.default_rng(91)
    with Context(0) as ctx:
        Xs = [rng.standard_normal((r, c)).astype(np.float32) for r, c in ((3_000, 40), (9_000, 120), (20_000, 64))]
        mats = [ctx.upload(X) for X in Xs]
        jobs = []
        for i in range(90):
            j = i % 3
            n = int(rng.integers(5, 400))
            inds = [rng.permutation(Xs[j].shape[1])[: int(rng.integers(2, 20))].astype(np.int32) for _ in range(n)]
            jobs.append((j, *gen.csr(inds)))
        announce("serve graph captures", len(jobs))
        with Server(ctx, hbm_budget_bytes=64 << 20, slots=2) as srv:
            srv.pause(True)
            futs = [srv.submit(i, mats[j], o, c, negative=True) for i, (j, o, c) in enumerate(jobs[:40])]
            srv.pause(False)
            futs += [srv.submit(i, mats[j], o, c, negative=True) for i, (j, o, c) in enumerate(jobs[40:])]
            results = [f.result(timeout=60) for f in futs]
            stats = srv.stats()
        assert stats["graph_captures"] <= 2, stats
        for i in (0, 17, 45, 89):
            j, o, c = jobs[i]
            alone = _alone(ctx, mats[j], o, c)
            assert np.array_equal(results[i].matched, alone[0]) and np.array_equal(results[i].negative, alone[1])
        torch.cuda.synchronize()
        for m in mats:
            ctx.release(m)
