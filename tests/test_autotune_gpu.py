"""The autotuner through the C ABI: it stores a shape for the sample's
class (plain and batched), evaluations in the tuned shapes stay bit-exact
against the oracle, the cache file it writes is read back by a later
context (EBIC_TUNE_CACHE), and a shape forced afterwards still wins over
the tuned one."""
import json
import os

import numpy as np
import pytest

from paper_1807_09932_amd import gen
from tests.gpu_common import announce, assert_same, oracle_eval, to_np

pytestmark = pytest.mark.gpu


def _workload():
    w = gen.make_matrix(41, 30_011, 64, "beta", 4, (200, 400), (4, 8), directions="alternate")
    pops = [gen.make_population(41, q, 64, n, (2, 20), w.plants) for q, n in enumerate((300, 170, 90))]
    return w.X, [gen.csr(p) for p in pops]


def test_autotune_plain_and_batch_then_cache(tmp_path):
    import torch
    from paper_1807_09932_amd import ebic
    X, packed = _workload()
    cache = str(tmp_path / "tune.json")
    ctx = ebic.Context(0)
    try:
        mat = ctx.upload(X)
        dev = [ctx.population(offsets=o, cols=c) for o, c in packed]
        outs = [ctx.outputs(mat, p.n) for p in dev]
        reqs = [ctx.request(mat, p, o) for p, o in zip(dev, outs)]
        default_plain = ebic.ebic_plan_shape(ctx.handle, mat, dev[0].n, int(packed[0][0][-1]))
        announce("autotune")
        ctx.autotune(reqs, cache)
        assert os.path.exists(cache)
        entries = json.load(open(cache))
        assert entries, "the cache holds the tuned shapes"
        tuned_plain = ebic.ebic_plan_shape(ctx.handle, mat, dev[0].n, int(packed[0][0][-1]))
        assert tuned_plain[3] in (ebic.STAGE_PAIRS, ebic.STAGE_BYTES, ebic.STAGE_CODES, ebic.STAGE_LDS,
                                  ebic.STAGE_DIRECT)
        # every population, plain and batched, in the tuned shapes: bit-exact
        for (o, c), p in zip(packed, dev):
            m, g, _, _ = ctx.eval(mat, p, negative=True)
            torch.cuda.synchronize()
            want = oracle_eval(X, o, c, negative=True, masks=False)
            assert_same((to_np(m), to_np(g), None, None), want, "tuned plain")
        ctx.eval_batch(reqs)
        torch.cuda.synchronize()
        for (o, c), out in zip(packed, outs):
            want = oracle_eval(X, o, c, negative=True, masks=False)
            assert_same((to_np(out[0]), to_np(out[1]), None, None), want, "tuned batch")
        # a forced shape wins over the tuned one, and clearing it restores the tuned one
        ctx.set_launch_shape(4, 8, 64, ebic.STAGE_BYTES, 0)
        assert tuple(ebic.ebic_plan_shape(ctx.handle, mat, dev[0].n)[:3]) == (4, 8, 64)
        ctx.set_launch_shape()
        assert ebic.ebic_plan_shape(ctx.handle, mat, dev[0].n, int(packed[0][0][-1])) == tuned_plain
        ctx.release(mat)
    finally:
        ctx.close()
    # a later context reads the cache at creation
    old = os.environ.get("EBIC_TUNE_CACHE")
    os.environ["EBIC_TUNE_CACHE"] = cache
    try:
        ctx2 = ebic.Context(0)
    finally:
        if old is None:
            os.environ.pop("EBIC_TUNE_CACHE", None)
        else:
            os.environ["EBIC_TUNE_CACHE"] = old
    try:
        mat2 = ctx2.upload(X)
        got = ebic.ebic_plan_shape(ctx2.handle, mat2, len(packed[0][0]) - 1, int(packed[0][0][-1]))
        assert got[:4] == tuned_plain[:4], (got, tuned_plain, default_plain)
        ctx2.release(mat2)
    finally:
        ctx2.close()
