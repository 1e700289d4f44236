"""Individuals whose first columns repeat, on matrices whose rows hold no two
equal values, through the SWAR rank-code paths (bit-exact to the oracle).

On such a matrix every 512-row chunk of the byte or 16-bit codes is marked
tie-free, so the evaluation runs the variant without the first pair's tie
handling. An individual c, c, b, ... compares a cell with itself on its first
pair (x >= x and x <= x both hold: Methods, "Handling missing values", with
repeated columns allowed), so every row is tied there; rows that fall after
column 1 are on the negative trend only. The prep step drops the leading run
of repeats, and these tests check the result against the oracle for byte
codes (one and two lane words per row) and 16-bit codes (one and two), with
and without negative trends, masks included, in plain and batched launches.
"""
import numpy as np
import pytest

from paper_1807_09932_amd import gen
from tests.gpu_common import announce, assert_same, gpu_eval, oracle_eval, to_np

pytestmark = pytest.mark.gpu

ROWS = 9_037  # 18 chunks of 512 rows and a ragged tail


@pytest.fixture(scope="module")
def ctx():
    from paper_1807_09932_amd.ebic import Context
    c = Context(0)
    yield c
    c.close()


def tie_free_matrix(rows, cols, seed):
    """N(0,1) in float32, rows holding two equal values drawn again."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((rows, cols)).astype(np.float32)
    while True:
        bad = (np.diff(np.sort(X, axis=1), axis=1) == 0).any(axis=1)
        if not bad.any():
            return X
        X[bad] = rng.standard_normal((int(bad.sum()), cols)).astype(np.float32)


def repeated_first(rng, cols, n):
    """c, c, b, ... (lengths 3..30), c, c, c, b, ..., c, c and a few plain ones."""
    inds = []
    for i in range(n):
        k = int(rng.integers(2, 29))
        base = [int(c) for c in rng.permutation(cols)[:k]]
        kind = i % 5
        if kind in (0, 1):
            ind = [base[0]] + base                 # length k + 1: 3..30
        elif kind == 2:
            ind = [base[0]] * 3 + base[1:]
        elif kind == 3:
            ind = [base[0], base[0]]
        else:
            ind = base
        inds.append(np.asarray(ind, np.int32))
    return gen.csr(inds)


CASES = [  # columns, staging, tiles per wave (one or two lane words per row)
    (64, 3, 4), (64, 3, 8), (128, 3, 4), (128, 3, 8),
    (200, 4, 2), (200, 4, 4), (310, 4, 2), (310, 4, 4),
    (200, 5, 3), (310, 5, 3), (512, 5, 3),  # 10-bit codes
]


@pytest.fixture(scope="module")
def matrices(ctx):
    out = {}
    for cols in sorted({c for c, _, _ in CASES}):
        X = tie_free_matrix(ROWS, cols, 7000 + cols)
        m = ctx.upload(X)
        st = ctx.stats(m)
        # every chunk of the SWAR codes is tie-free, and nothing is missing
        assert st["swar_chunks"] == ((ROWS + 511) // 512 if cols <= 128 else (ROWS + 191) // 192), st
        assert st["swar_tie_chunks"] == 0, st
        assert st["has_missing"] == 0, st
        out[cols] = (X, m)
    yield out
    for _, m in out.values():
        ctx.release(m)


@pytest.mark.parametrize("cols,staging,tiles", CASES, ids=lambda v: str(v))
def test_repeated_first_column_plain(ctx, matrices, cols, staging, tiles):
    from paper_1807_09932_amd import ebic
    X, m = matrices[cols]
    rng = np.random.default_rng(cols * 10 + tiles)
    offs, cc = repeated_first(rng, cols, 150)
    ctx.set_launch_shape(tiles, 8, 64, staging, 0)
    try:
        plan = ebic.ebic_plan_shape(ctx.handle, m, offs.size - 1)
        assert plan[3] == staging, plan
        for negative in (True, False):
            announce("repeated first column plain", cols, staging, plan[0], negative)
            got = gpu_eval(ctx, m, offs, cc, negative=negative, masks=True)
            want = oracle_eval(X, offs, cc, negative=negative, masks=True)
            assert_same(got, want, f"cols={cols} staging={staging} L={plan[0]} neg={negative}")
            if negative:
                # the case is reached: repeated-first individuals with rows
                # on the negative trend only
                firsts = cc[offs[:-1]]
                seconds = cc[np.minimum(offs[:-1] + 1, offs[1:] - 1)]
                dup = (firsts == seconds) & (np.diff(offs) >= 3)
                assert (want[1][dup] > 0).sum() > 10
    finally:
        ctx.set_launch_shape()


@pytest.mark.parametrize("cols,staging,tiles", [(64, 3, 4), (128, 3, 4), (200, 4, 2), (310, 4, 2),
                                                (200, 5, 2), (310, 5, 2)],
                         ids=lambda v: str(v))
def test_repeated_first_column_batched(ctx, matrices, cols, staging, tiles):
    import torch
    X, m = matrices[cols]
    rng = np.random.default_rng(cols * 10 + 99)
    pops = [repeated_first(rng, cols, int(rng.integers(40, 160))) for _ in range(5)]
    ctx.set_launch_shape(tiles, 8, 64, staging, 0)
    try:
        from paper_1807_09932_amd import ebic
        for negative in (True, False):
            reqs, outs, held = [], [], []  # (requests hold raw pointers: keep the tensors alive)
            for offs, cc in pops:
                p = ctx.population(offsets=offs, cols=cc)
                o = ctx.outputs(m, p.n, masks=True, negative=negative)
                held.append(p)
                outs.append(o)
                reqs.append(ctx.request(m, p, o, negative=negative))
            shape = ebic.ebic_plan_batch_shape(ctx.handle, reqs)
            assert all(s == staging for s in shape[3]), shape
            announce("repeated first column batched", cols, staging, negative)
            ctx.eval_batch(reqs)
            torch.cuda.synchronize()
            for (offs, cc), o in zip(pops, outs):
                got = tuple(to_np(t) for t in o)
                want = oracle_eval(X, offs, cc, negative=negative, masks=True)
                assert_same(got, want, f"batched cols={cols} neg={negative}")
    finally:
        ctx.set_launch_shape()
