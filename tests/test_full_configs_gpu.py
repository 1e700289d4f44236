"""Every configuration at full size against the oracle, element by element.

* the batched workload: all 64 populations over the 100,000 x 256 matrix in
  one batched launch (the shape the benchmark times), every count, and the
  masks of a subset of populations;
* the served workload: the four full-size resident matrices, requests
  arriving at the Poisson schedule through the serving engine, every
  request's counts;
* the methylation workload (436,444 x 64) in include mode, counts and masks;
* the paper's dataset width, 436,444 x 310 (Results, Table 1), the whole
  800-individual population, counts and masks, in the default launch shape
  and in the one the benchmark's autotuner picks.
"""
import time

import numpy as np
import pytest

from paper_1807_09932_amd import gen
from tests.gpu_common import announce, assert_same, gpu_eval, oracle_eval, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1807_09932_amd.ebic import Context
    c = Context(0)
    yield c
    c.close()


def test_batched_all_64_populations(ctx):
    import torch
    from paper_1807_09932_amd import ebic
    w, pops = gen.batched_100000x256()
    mat = ctx.upload(w.X)
    packed = [gen.csr(p) for p in pops]
    dev = [ctx.population(offsets=o, cols=c) for o, c in packed]
    with_masks = {0, 21, 42, 63}
    outs = [ctx.outputs(mat, p.n, masks=q in with_masks) for q, p in enumerate(dev)]
    reqs = [ctx.request(mat, p, o) for p, o in zip(dev, outs)]
    L, W, P, stagings, _ = ebic.ebic_plan_batch_shape(ctx.handle, reqs)
    assert (L, W) == (1, 4) and set(stagings) == {ebic.STAGE_PAIRS}
    announce("batched 64 populations", sum(p.n for p in dev))
    ctx.eval_batch(reqs)
    torch.cuda.synchronize()
    for q, ((o, c), out) in enumerate(zip(packed, outs)):
        got = tuple(to_np(t) for t in out)
        want = oracle_eval(w.X, o, c, masks=q in with_masks)
        assert_same(got, want, f"population {q}")
    ctx.release(mat)


def test_served_full_scale_every_request(ctx):
    from paper_1807_09932_amd.serve import Server
    ws = gen.served_matrices()
    assert [x.X.shape for x in ws] == [(10000, 100), (50000, 200), (200000, 64), (436444, 64)]
    mats = [ctx.upload(x.X) for x in ws]
    pools = gen.served_pools()
    reqs = gen.served_requests(0.3)
    used = sorted({(r.matrix, r.pool_index) for r in reqs})
    announce("served oracle", len(used))
    want = {}
    for m, k in used:
        o, c = pools[m][k]
        want[(m, k)] = oracle_eval(ws[m].X, o, c, masks=False)
    announce("served full scale", len(reqs))
    with Server(ctx, hbm_budget_bytes=1 << 30, slots=4) as srv:
        t0 = time.perf_counter()
        futs = []
        for r in reqs:
            while time.perf_counter() - t0 < r.t_arrival:
                time.sleep(1e-4)
            o, c = pools[r.matrix][r.pool_index]
            futs.append(srv.submit(r.run, mats[r.matrix], o, c))
        results = [f.result(timeout=120) for f in futs]
        stats = srv.stats()
    assert stats["completed"] == len(reqs)
    for i, (r, res) in enumerate(zip(reqs, results)):
        wm, wn, _, _ = want[(r.matrix, r.pool_index)]
        assert np.array_equal(res.matched, wm), f"request {i} matched"
        assert np.array_equal(res.negative, wn), f"request {i} negative"
    for m in mats:
        ctx.release(m)


def test_methylation_include_mode_full(ctx):
    w, pop = gen.methylation_436444x64()
    offs, cols = gen.csr(pop)
    mat = ctx.upload(w.X, fill=0.5)
    announce("methylation_436444x64 include")
    got = gpu_eval(ctx, mat, offs, cols, include=True, negative=True, masks=True)
    want = oracle_eval(w.X, offs, cols, include=True, negative=True, masks=True, fill=0.5)
    assert_same(got, want, "methylation_436444x64 include")
    ctx.release(mat)


@pytest.mark.parametrize("shape,staging", [(None, 6), ((3, 16, 400, 5), 5), ((6, 16, 200, 5), 5),
                                           ((2, 16, 400, 4), 4)],
                         ids=["default", "10-bit-P400", "10-bit-two-words", "16-bit"])
def test_methylation_wide_full(ctx, shape, staging):
    from paper_1807_09932_amd import ebic
    w, pop = gen.methylation_wide()
    offs, cols = gen.csr(pop)
    mat = ctx.upload(w.X)
    try:
        if shape:
            ctx.set_launch_shape(*shape, 0)
        plan = ebic.ebic_plan_shape(ctx.handle, mat, offs.size - 1)
        assert plan[3] == staging
        announce("methylation 436444x310", plan)
        got = gpu_eval(ctx, mat, offs, cols, negative=True, masks=True)
        want = oracle_eval(w.X, offs, cols, negative=True, masks=True)
        assert_same(got, want, f"436444x310 {plan}")
    finally:
        ctx.set_launch_shape()
        ctx.release(mat)
