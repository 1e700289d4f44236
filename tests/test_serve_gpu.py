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
