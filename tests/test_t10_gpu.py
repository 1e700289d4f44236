"""10-bit rank codes (three rows per 32-bit lane word, for matrices of 129 to
512 columns) against the oracle, bit-exact, through the C ABI: tie-heavy,
tie-free and missing-valued matrices, ragged row counts around the 192-row
groups and 384-row chunks, one and two lane words per chunk, several launch
shapes, plain and batched launches."""
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


def _matrix(kind, rows, cols, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((rows, cols))
    if kind == "ties":
        X = np.round(X, 1)
    X = X.astype(np.float32)
    if kind == "missing":
        X[rng.random(X.shape) < 0.03] = np.float32(np.nan)
    return X


def _pop(rng, cols, n, kmax=30, dup=0.05, bad=0.02):
    inds = []
    for _ in range(n):
        k = int(rng.integers(1, kmax + 1))
        if rng.random() < dup:
            ind = rng.integers(0, cols, size=k)
        else:
            ind = rng.permutation(cols)[:k]
        if rng.random() < bad:
            ind = np.append(ind, cols + 1)
        inds.append(np.asarray(ind, np.int32))
    return gen.csr(inds)


SHAPES = [(3, 16, 200, 0), (3, 8, 64, 0), (3, 5, 33, 7), (3, 16, 400, 0), (3, 1, 5, 2),
          (6, 16, 200, 0), (6, 8, 64, 0), (6, 5, 33, 7), (6, 16, 400, 3), (6, 2, 5, 0)]


@pytest.mark.parametrize("cols", [129, 200, 310, 384, 512])
@pytest.mark.parametrize("kind", ["ties", "missing", "tiefree"])
def test_t10_plain(ctx, cols, kind):
    from paper_1807_09932_amd import ebic
    rows = 5_037
    X = _matrix("ties" if kind == "ties" else ("missing" if kind == "missing" else "plain"), rows, cols,
                cols + len(kind))
    rng = np.random.default_rng(cols)
    offs, cc = _pop(rng, cols, 220)
    mat = ctx.upload(X, fill=0.5)
    st = ctx.stats(mat)
    assert st["code_sets"] & ebic.SET_U10, st
    try:
        for shape in SHAPES:
            ctx.set_launch_shape(shape[0], shape[1], shape[2], ebic.STAGE_T10, shape[3])
            for include in (False, True):
                # exclude mode on a matrix with missing cells cannot use codes of
                # the filled values: the plan falls back
                plan = ebic.ebic_plan_shape(ctx.handle, mat, offs.size - 1)
                for negative in (True, False):
                    announce("t10 plain", cols, kind, shape, include, negative)
                    got = gpu_eval(ctx, mat, offs, cc, include=include, negative=negative, masks=True)
                    want = oracle_eval(X, offs, cc, include=include, negative=negative, masks=True,
                                       fill=0.5)
                    assert_same(got, want, f"cols={cols} {kind} {shape} include={include} neg={negative}")
            if kind != "missing":
                assert plan[3] == ebic.STAGE_T10, plan
    finally:
        ctx.set_launch_shape()
        ctx.release(mat)


@pytest.mark.parametrize("tiles", [3, 6])
@pytest.mark.parametrize("rows", [1, 63, 64, 65, 191, 192, 193, 383, 384, 385, 577, 769])
def test_t10_edge_rows(ctx, rows, tiles):
    from paper_1807_09932_amd import ebic
    X = _matrix("ties", rows, 150, rows)
    rng = np.random.default_rng(rows)
    offs, cc = _pop(rng, 150, 60, kmax=12, dup=0.2)
    mat = ctx.upload(X)
    try:
        ctx.set_launch_shape(tiles, 4, 16, ebic.STAGE_T10, 0)
        assert tuple(ebic.ebic_plan_shape(ctx.handle, mat, 60)[::3]) == (tiles, ebic.STAGE_T10)
        for include in (False, True):
            announce("t10 rows", rows, tiles, include)
            got = gpu_eval(ctx, mat, offs, cc, include=include, negative=True, masks=True)
            assert_same(got, oracle_eval(X, offs, cc, include=include, negative=True, masks=True),
                        f"rows={rows} include={include}")
    finally:
        ctx.set_launch_shape()
        ctx.release(mat)


@pytest.mark.parametrize("forced", [(2, 8, 128, 5), (2, 16, 1024, 5), None])
def test_t10_batched(ctx, forced):
    """Batches of several populations on wide matrices (with a narrow one in
    the mix when not forced: its requests take byte codes in the same
    launch)."""
    import torch
    from paper_1807_09932_amd import ebic
    mats, Xs = [], []
    for rows, cols, kind, seed in [(4_099, 256, "plain", 1), (2_001, 310, "ties", 2), (3_001, 64, "ties", 3)]:
        X = _matrix(kind, rows, cols, seed)
        Xs.append(X)
        mats.append(ctx.upload(X))
    rng = np.random.default_rng(99)
    jobs = []
    for q in range(12):
        k = q % (3 if forced is None else 2)
        offs, cc = _pop(rng, Xs[k].shape[1], int(rng.integers(1, 300)))
        jobs.append((k, offs, cc, bool(q & 1), bool(q & 2)))
    if forced:
        ctx.set_launch_shape(*forced, 0)
    else:
        ctx.set_launch_shape(2, 16, 1024, ebic.STAGE_T10, 0)
    try:
        held, reqs, outs = [], [], []
        for k, offs, cc, negative, masks in jobs:
            p = ctx.population(offsets=offs, cols=cc)
            o = ctx.outputs(mats[k], p.n, masks=masks)
            held.append(p)
            outs.append(o)
            reqs.append(ctx.request(mats[k], p, o, negative=negative))
        shape = ebic.ebic_plan_batch_shape(ctx.handle, reqs)
        for (k, *_), stg in zip(jobs, shape[3]):
            assert stg == (ebic.STAGE_BYTES if Xs[k].shape[1] <= 128 else ebic.STAGE_T10), shape
        announce("t10 batched", forced)
        ctx.eval_batch(reqs)
        torch.cuda.synchronize()
        for (k, offs, cc, negative, masks), o in zip(jobs, outs):
            got = tuple(to_np(t) for t in o)
            want = oracle_eval(Xs[k], offs, cc, negative=negative, masks=masks)
            assert_same(got, want, f"batched matrix {k}")
    finally:
        ctx.set_launch_shape()
        for m in mats:
            ctx.release(m)
