"""Byte codes four lane words per row group (1024-row chunks; counts only)
against the oracle, bit-exact: tie-free matrices (the four-word sequences),
sparse ties (tied and tie-free chunks side by side), tie-heavy and
missing-valued ones (each pair of words on its own),
ragged row counts, several launch shapes, and the planner's fallback to
two words when masks are asked for."""
import numpy as np
import pytest

from paper_1807_09932_amd import gen
from tests.gpu_common import announce, assert_same, gpu_eval, oracle_eval

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1807_09932_amd.ebic import Context
    c = Context(0)
    yield c
    c.close()


def _tie_free(rows, cols, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((rows, cols)).astype(np.float32)
    while True:
        bad = (np.diff(np.sort(X, axis=1), axis=1) == 0).any(axis=1)
        if not bad.any():
            return X
        X[bad] = rng.standard_normal((int(bad.sum()), cols)).astype(np.float32)


def _pop(rng, cols, n):
    inds = []
    for i in range(n):
        k = int(rng.integers(1, 31))
        ind = [int(c) for c in rng.permutation(cols)[:k]]
        if i % 7 == 0:
            ind = [ind[0]] + ind  # a repeated first column
        if i % 13 == 0:
            ind = ind + [cols + 2]  # invalid
        inds.append(np.asarray(ind, np.int32))
    return gen.csr(inds)


def _counts(got):
    return (got[0], got[1], None, None)


SHAPES = [(16, 16, 200, 3, 0), (16, 8, 64, 3, 0), (16, 5, 33, 3, 7), (16, 16, 400, 3, 8)]


@pytest.mark.parametrize("kind", ["tiefree", "ties", "missing"])
@pytest.mark.parametrize("cols", [64, 128])
def test_four_words(ctx, kind, cols):
    from paper_1807_09932_amd import ebic
    rows = 9_037 if kind == "tiefree" else 5_101
    if kind == "tiefree":
        X = _tie_free(rows, cols, cols)
    else:
        rng = np.random.default_rng(cols + 1)
        X = rng.integers(0, 9, size=(rows, cols)).astype(np.float32)
        if kind == "missing":
            X[rng.random(X.shape) < 0.03] = np.float32(np.nan)
    rng = np.random.default_rng(cols * 3)
    offs, cc = _pop(rng, cols, 260)
    mat = ctx.upload(X, fill=2.5)
    try:
        for shape in SHAPES:
            ctx.set_launch_shape(*shape)
            for include in ((True,) if kind == "missing" else (False, True)):
                plan = ebic.ebic_plan_shape(ctx.handle, mat, offs.size - 1)
                for negative in (True, False):
                    announce("four words", kind, cols, shape, include, negative)
                    got = gpu_eval(ctx, mat, offs, cc, include=include, negative=negative, masks=False)
                    want = oracle_eval(X, offs, cc, include=include, negative=negative, masks=False, fill=2.5)
                    assert_same(_counts(got), want, f"{kind} cols={cols} {shape} include={include} neg={negative}")
            if kind == "tiefree" and cols == 64:
                assert tuple(plan[:2]) == (16, shape[1]), plan
                assert ctx.stats(mat)["swar_tie_chunks"] == 0
    finally:
        ctx.set_launch_shape()
        ctx.release(mat)


def test_sparse_ties(ctx):
    """A tie-free matrix with a few rows holding two equal cells: their
    chunks run the two-word sequences with the tie chain, the others the
    four-word ones; some individuals start with exactly an equal pair."""
    from paper_1807_09932_amd import ebic
    rows, cols = 20_011, 64
    X = _tie_free(rows, cols, 21)
    rng = np.random.default_rng(21)
    tied_rows = rng.choice(rows, size=60, replace=False)
    pairs = []
    for r in tied_rows:
        a, b = (int(v) for v in rng.choice(cols, size=2, replace=False))
        X[r, b] = X[r, a]
        pairs.append((a, b))
    offs0, cc0 = _pop(rng, cols, 300)
    inds = [cc0[offs0[i]:offs0[i + 1]] for i in range(offs0.size - 1)]
    for a, b in pairs[:40]:  # first pair equal in one row
        rest = [int(c) for c in rng.permutation(cols) if c not in (a, b)][: int(rng.integers(0, 6))]
        inds.append(np.asarray([a, b] + rest, np.int32))
        inds.append(np.asarray([b, a] + rest, np.int32))
    offs, cc = gen.csr(inds)
    mat = ctx.upload(X)
    try:
        st = ctx.stats(mat)
        assert 0 < st["swar_tie_chunks"] < st["swar_chunks"], st
        for shape in SHAPES:
            ctx.set_launch_shape(*shape)
            assert ebic.ebic_plan_shape(ctx.handle, mat, offs.size - 1)[0] == 16
            for include in (False, True):
                for negative in (True, False):
                    announce("sparse ties", shape, include, negative)
                    got = gpu_eval(ctx, mat, offs, cc, include=include, negative=negative, masks=False)
                    want = oracle_eval(X, offs, cc, include=include, negative=negative, masks=False)
                    assert_same(_counts(got), want, f"sparse ties {shape} include={include} neg={negative}")
    finally:
        ctx.set_launch_shape()
        ctx.release(mat)


def test_masks_take_two_words(ctx):
    """A call with masks is planned at eight sub-tiles (two words); the
    masks and counts are exact."""
    from paper_1807_09932_amd import ebic
    X = _tie_free(3_001, 64, 5)
    rng = np.random.default_rng(5)
    offs, cc = _pop(rng, 64, 100)
    mat = ctx.upload(X)
    try:
        ctx.set_launch_shape(16, 16, 200, ebic.STAGE_BYTES, 0)
        got = gpu_eval(ctx, mat, offs, cc, negative=True, masks=True)
        assert_same(got, oracle_eval(X, offs, cc, negative=True, masks=True), "masks at L=16 request")
    finally:
        ctx.set_launch_shape()
        ctx.release(mat)


def test_methylation_full_four_words(ctx):
    from paper_1807_09932_amd import ebic
    w, pop = gen.methylation_436444x64()
    offs, cols = gen.csr(pop)
    mat = ctx.upload(w.X)
    try:
        for shape in ((16, 16, 200, 3, 0), (16, 16, 400, 3, 0)):
            ctx.set_launch_shape(*shape)
            assert ebic.ebic_plan_shape(ctx.handle, mat, offs.size - 1)[0] == 16
            announce("methylation four words", shape)
            got = gpu_eval(ctx, mat, offs, cols, negative=True, masks=False)
            assert_same(_counts(got), oracle_eval(w.X, offs, cols, negative=True, masks=False),
                        f"methylation {shape}")
    finally:
        ctx.set_launch_shape()
        ctx.release(mat)


@pytest.mark.parametrize("rows", [1, 63, 64, 65, 511, 512, 513, 1023, 1024, 1025, 1537, 2049])
@pytest.mark.parametrize("blocks", [0, 1, 3])
def test_edge_rows_four_words(ctx, rows, blocks):
    """Row counts around the 64-row sub-tiles, 512-row units and 1024-row
    chunks, with ranges of one, three or as many blocks as the planner
    picks (half chunks at range ends, a last chunk past the matrix)."""
    from paper_1807_09932_amd import ebic
    rng = np.random.default_rng(rows * 7 + blocks)
    X = rng.integers(0, 6, size=(rows, 64)).astype(np.float32)  # tie-heavy: both paths
    X[: rows // 2] = _tie_free(rows // 2, 64, rows) if rows >= 2 else X[: rows // 2]
    offs, cc = _pop(rng, 64, 90)
    mat = ctx.upload(X)
    try:
        ctx.set_launch_shape(16, 8, 32, ebic.STAGE_BYTES, blocks)
        assert ebic.ebic_plan_shape(ctx.handle, mat, offs.size - 1)[0] == 16
        for negative in (True, False):
            announce("four words rows", rows, blocks, negative)
            got = gpu_eval(ctx, mat, offs, cc, negative=negative, masks=False)
            assert_same(_counts(got), oracle_eval(X, offs, cc, negative=negative, masks=False),
                        f"rows={rows} blocks={blocks} negative={negative}")
    finally:
        ctx.set_launch_shape()
        ctx.release(mat)
