"""The pairwise order bitmaps (one bit per row for every ordered pair of
columns, built on first use) against the oracle, bit-exact, through the C
ABI: special values (signed zeros, infinities, NaN, ties), both missing-value
modes with and without negative trends and masks, one-column, repeated-column
and invalid individuals, individuals longer than the header's window, row
counts around the 32-row words and 2,048-row chunks, widths around the
bitmap build's column blocking and past the codes' limits, several launch
shapes, the methylation workloads at full size, the
fallbacks (too many columns, the allocation-free entry point before the
bitmaps exist), and batches: requests on several matrices and in both modes
on the batched pairs kernel beside requests on the tiled one."""
import numpy as np
import pytest

from paper_1807_09932_amd import gen
from tests.gpu_common import announce, assert_same, gpu_eval, oracle_eval

pytestmark = pytest.mark.gpu

# (tiles_per_wave, waves_per_block, individuals_per_group, chunks per wave
# run: 0 = the planner's)
SHAPES = [(1, 16, 200, 0), (1, 8, 64, 0), (1, 5, 33, 0), (1, 1, 7, 0), (1, 16, 800, 0),
          (1, 2, 128, 2), (1, 4, 9, 1), (1, 8, 8, 5), (1, 4, 4, 0)]


@pytest.fixture(scope="module")
def ctx():
    from paper_1807_09932_amd.ebic import Context
    c = Context(0)
    yield c
    c.close()


def _special(rows, cols, seed):
    rng = np.random.default_rng(seed)
    X = np.round(rng.standard_normal((rows, cols)), 1).astype(np.float32)
    pick = rng.random(X.shape)
    X[pick < 0.02] = np.float32(0.0)
    X[(pick >= 0.02) & (pick < 0.04)] = np.float32(-0.0)
    X[(pick >= 0.04) & (pick < 0.05)] = np.float32(np.inf)
    X[(pick >= 0.05) & (pick < 0.06)] = np.float32(-np.inf)
    X[(pick >= 0.06) & (pick < 0.09)] = np.float32(np.nan)
    return X


def _pop(rng, cols, n, kmax=30):
    inds = []
    for i in range(n):
        k = int(rng.integers(1, kmax + 1))
        ind = [int(c) for c in rng.permutation(cols)[:k]]
        if i % 9 == 0:
            ind = [ind[0], ind[0]] + ind  # leading repeats
        if i % 11 == 0 and k > 2:
            ind = ind[:2] + [ind[1]] + ind[2:]  # an inner repeat
        if i % 17 == 0:
            ind = ind + [cols + 1]  # invalid
        if i % 23 == 0:
            ind = [ind[0]]  # one column
        inds.append(np.asarray(ind, np.int32))
    inds.append(np.asarray([], np.int32))  # empty: invalid
    return gen.csr(inds)


def _check(ctx, mat, X, offs, cc, what, *, fill=0.0, masks=True, modes=(False, True)):
    from paper_1807_09932_amd import ebic
    for shape in SHAPES:
        ctx.set_launch_shape(shape[0], shape[1], shape[2], ebic.STAGE_PAIRS, shape[3])
        for include in modes:
            for negative in (True, False):
                announce("pairs", what, shape, include, negative)
                got = gpu_eval(ctx, mat, offs, cc, include=include, negative=negative, masks=masks)
                want = oracle_eval(X, offs, cc, include=include, negative=negative, masks=masks, fill=fill)
                if not masks:
                    got = (got[0], got[1], None, None)
                assert_same(got, want, f"{what} {shape} include={include} negative={negative}")


@pytest.mark.parametrize("cols", [5, 64, 200, 600])
def test_pairs_special_values(ctx, cols):
    from paper_1807_09932_amd import ebic
    rows = 4_133
    X = _special(rows, cols, cols)
    rng = np.random.default_rng(cols + 3)
    offs, cc = _pop(rng, cols, 150, kmax=min(30, 2 * cols))
    mat = ctx.upload(X, fill=-0.0)
    try:
        _check(ctx, mat, X, offs, cc, f"special cols={cols}", fill=-0.0)
        st = ctx.stats(mat)
        assert st["code_sets"] & ebic.SET_PAIRS and st["code_sets"] & ebic.SET_PAIRS_FILL, st
        assert ebic.ebic_plan_shape(ctx.handle, mat, offs.size - 1)[3] == ebic.STAGE_PAIRS
    finally:
        ctx.set_launch_shape()
        ctx.release(mat)


def test_pairs_no_missing_share_one_set(ctx):
    """Without missing cells include mode reads the bitmaps of X itself: one
    set is built."""
    from paper_1807_09932_amd import ebic
    rng = np.random.default_rng(8)
    X = rng.integers(0, 7, size=(3_001, 40)).astype(np.float32)
    offs, cc = _pop(rng, 40, 120)
    mat = ctx.upload(X)
    try:
        _check(ctx, mat, X, offs, cc, "no missing")
        st = ctx.stats(mat)
        assert st["code_sets"] & ebic.SET_PAIRS and not st["code_sets"] & ebic.SET_PAIRS_FILL, st
    finally:
        ctx.set_launch_shape()
        ctx.release(mat)


def test_pairs_long_individuals(ctx):
    """Individuals of up to 200 columns (past the eight-column window, with
    the exit checks along the tail) on a matrix where long chains survive:
    rows sorted along a random column order."""
    rng = np.random.default_rng(12)
    rows, cols = 6_000, 256
    X = rng.standard_normal((rows, cols)).astype(np.float32)
    order = rng.permutation(cols)
    keep = rows // 3
    X[:keep, order] = np.sort(X[:keep], axis=1)          # rising along `order`
    X[keep:2 * keep, order] = -np.sort(X[keep:2 * keep], axis=1)  # falling
    inds = []
    for _ in range(90):
        k = int(rng.integers(9, 201))
        start = int(rng.integers(0, cols - k + 1))
        inds.append(order[start:start + k].astype(np.int32))
        inds.append(order[np.sort(rng.choice(cols, size=k, replace=False))].astype(np.int32))
    offs, cc = gen.csr(inds)
    mat = ctx.upload(X)
    try:
        _check(ctx, mat, X, offs, cc, "long", modes=(False,))
    finally:
        ctx.set_launch_shape()
        ctx.release(mat)


@pytest.mark.parametrize("rows", [1, 31, 32, 33, 2047, 2048, 2049, 4096, 6145])
def test_pairs_edge_rows(ctx, rows):
    from paper_1807_09932_amd import ebic
    rng = np.random.default_rng(rows)
    X = rng.integers(0, 4, size=(rows, 24)).astype(np.float32)
    X[rng.random(X.shape) < 0.02] = np.float32(np.nan)
    offs, cc = _pop(rng, 24, 70, kmax=12)
    mat = ctx.upload(X, fill=1.5)
    try:
        ctx.set_launch_shape(1, 4, 16, ebic.STAGE_PAIRS, 0)
        for include in (False, True):
            for negative in (True, False):
                announce("pairs rows", rows, include, negative)
                got = gpu_eval(ctx, mat, offs, cc, include=include, negative=negative, masks=True)
                want = oracle_eval(X, offs, cc, include=include, negative=negative, masks=True, fill=1.5)
                assert_same(got, want, f"rows={rows} include={include} negative={negative}")
    finally:
        ctx.set_launch_shape()
        ctx.release(mat)


@pytest.mark.parametrize("cols", [1, 2, 3, 129, 131])
def test_pairs_build_widths(ctx, cols):
    """Widths around the bitmap build's column blocking (two columns of a
    chunk per block up to 128 columns, four past that): the last block of
    a chunk holds fewer columns. The rows span nine chunks, one past a
    multiple of eight, so most of the build grid's second row of blocks has
    no chunk."""
    from paper_1807_09932_amd import ebic
    rows = 8 * 2048 + 77
    X = _special(rows, cols, 1000 + cols)
    rng = np.random.default_rng(cols + 11)
    offs, cc = _pop(rng, cols, 60, kmax=min(30, 2 * cols))
    mat = ctx.upload(X, fill=0.5)
    try:
        ctx.set_launch_shape(1, 4, 16, ebic.STAGE_PAIRS, 0)
        for include in (False, True):
            for negative in (True, False):
                announce("pairs build widths", cols, include, negative)
                got = gpu_eval(ctx, mat, offs, cc, include=include, negative=negative, masks=True)
                want = oracle_eval(X, offs, cc, include=include, negative=negative, masks=True, fill=0.5)
                assert_same(got, want, f"build widths cols={cols} include={include} negative={negative}")
        st = ctx.stats(mat)
        assert st["code_sets"] & ebic.SET_PAIRS and st["code_sets"] & ebic.SET_PAIRS_FILL, st
    finally:
        ctx.set_launch_shape()
        ctx.release(mat)


@pytest.mark.parametrize("which", ["m64", "wide"])
def test_pairs_methylation_full(ctx, which):
    """The methylation workloads at full size (436,444 rows; 64 and 310
    columns), counts and a sample of masks."""
    from paper_1807_09932_amd import ebic
    w, pop = gen.methylation_436444x64() if which == "m64" else gen.methylation_wide()
    offs, cols = gen.csr(pop)
    mat = ctx.upload(w.X)
    try:
        ctx.set_launch_shape(1, 16, 200, ebic.STAGE_PAIRS, 0)
        assert ebic.ebic_plan_shape(ctx.handle, mat, offs.size - 1)[3] == ebic.STAGE_PAIRS
        announce("pairs methylation", which)
        got = gpu_eval(ctx, mat, offs, cols, negative=True, masks=False)
        want = oracle_eval(w.X, offs, cols, negative=True, masks=False)
        assert_same((got[0], got[1], None, None), want, f"methylation {which}")
        sample = np.arange(0, offs.size - 1, 37)
        so, sc = gen.csr([cols[offs[i]:offs[i + 1]] for i in sample])
        announce("pairs methylation masks", which)
        got = gpu_eval(ctx, mat, so, sc, negative=True, masks=True)
        assert_same(got, oracle_eval(w.X, so, sc, negative=True, masks=True), f"methylation {which} masks")
    finally:
        ctx.set_launch_shape()
        ctx.release(mat)


def test_pairs_fallbacks(ctx):
    """Past 1,024 columns the shape falls back to another staging; the
    allocation-free entry point uses the bitmaps only once they exist;
    a batch never stages them; results are exact throughout."""
    import torch
    from paper_1807_09932_amd import ebic
    rng = np.random.default_rng(4)
    X = rng.integers(0, 5, size=(700, 1100)).astype(np.float32)
    offs, cc = _pop(rng, 1100, 40, kmax=10)
    mat = ctx.upload(X)
    try:
        ctx.set_launch_shape(1, 8, 64, ebic.STAGE_PAIRS, 0)
        assert ebic.ebic_plan_shape(ctx.handle, mat, offs.size - 1)[3] != ebic.STAGE_PAIRS
        announce("pairs fallback wide")
        got = gpu_eval(ctx, mat, offs, cc, negative=True, masks=True)
        assert_same(got, oracle_eval(X, offs, cc, negative=True, masks=True), "1100 columns")
        assert not ctx.stats(mat)["code_sets"] & ebic.SET_PAIRS
    finally:
        ctx.set_launch_shape()
        ctx.release(mat)

    X = rng.integers(0, 5, size=(3_000, 50)).astype(np.float32)
    offs, cc = _pop(rng, 50, 60, kmax=10)
    mat = ctx.upload(X)
    try:
        ctx.set_launch_shape(1, 8, 64, ebic.STAGE_PAIRS, 0)
        pop = ctx.population(offsets=offs, cols=cc)
        want = oracle_eval(X, offs, cc, negative=True, masks=False)
        n = offs.size - 1
        m = torch.empty(n, dtype=torch.int32, device=ctx.device)
        g = torch.empty(n, dtype=torch.int32, device=ctx.device)
        flags = ctx.flags(include=False, negative=True)

        def noalloc():
            ebic.ebic_eval_population_noalloc(ctx.handle, mat, n, pop.offsets.data_ptr(), pop.cols.data_ptr(),
                                              flags, m.data_ptr(), g.data_ptr(), 0, 0, 0)
            torch.cuda.synchronize()

        announce("pairs noalloc before build")
        noalloc()
        assert not ctx.stats(mat)["code_sets"] & ebic.SET_PAIRS
        assert_same((m.cpu().numpy(), g.cpu().numpy(), None, None), want, "noalloc before the build")
        gpu_eval(ctx, mat, offs, cc, negative=True, masks=False)  # builds them
        assert ctx.stats(mat)["code_sets"] & ebic.SET_PAIRS
        announce("pairs noalloc after build")
        noalloc()
        assert_same((m.cpu().numpy(), g.cpu().numpy(), None, None), want, "noalloc after the build")
        outs = [ctx.outputs(mat, n) for _ in range(2)]
        reqs = [ctx.request(mat, pop, o) for o in outs]
        announce("pairs batch")
        ctx.eval_batch(reqs)
        torch.cuda.synchronize()
        for out in outs:
            assert_same((out[0].cpu().numpy(), out[1].cpu().numpy(), None, None), want, "batch")
        assert ebic.ebic_plan_batch_shape(ctx.handle, reqs)[3] == [ebic.STAGE_PAIRS] * 2
    finally:
        ctx.set_launch_shape()
        ctx.release(mat)


def _tie_free(rows, cols, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((rows, cols)).astype(np.float32)
    while True:
        bad = (np.diff(np.sort(X, axis=1), axis=1) == 0).any(axis=1)
        if not bad.any():
            return X
        X[bad] = rng.standard_normal((int(bad.sum()), cols)).astype(np.float32)


@pytest.mark.parametrize("cols", [64, 310])
def test_pairs_sparse_ties(ctx, cols):
    """A tie-free matrix with equal pairs planted on a few rows (some as
    +0 / -0): chunks without ties, chunks listing a few tied pairs, and one
    chunk with more tied pairs than its list holds. Individuals start with a
    tied pair, hold one inside the window, or reach one past the window."""
    from paper_1807_09932_amd import ebic
    rows = 20_011
    X = _tie_free(rows, cols, cols + 7)
    rng = np.random.default_rng(cols + 8)
    pairs = []
    for r in rng.choice(np.arange(8192, rows), size=50, replace=False):  # chunks 4 .. 9
        a, b = (int(v) for v in rng.choice(cols, size=2, replace=False))
        if len(pairs) % 5 == 0:
            X[r, a], X[r, b] = np.float32(0.0), np.float32(-0.0)
        else:
            X[r, b] = X[r, a]
        pairs.append((a, b))
    for r in range(4096, 4096 + 45):  # chunk 2: 45 tied pairs, past the list
        a, b = (int(v) for v in rng.choice(cols, size=2, replace=False))
        X[r, b] = X[r, a]
    # a run of rows rising along one order, so that chains reach the tail
    order = rng.permutation(cols)
    X[10_000:10_600, order] = np.sort(X[10_000:10_600], axis=1)
    inds = [np.asarray(rng.permutation(cols)[: int(rng.integers(2, 31))], np.int32) for _ in range(200)]
    for a, b in pairs[:30]:
        rest = [int(c) for c in order if c not in (a, b)]
        inds.append(np.asarray([a, b] + rest[:5], np.int32))           # first pair tied
        inds.append(np.asarray(rest[:3] + [b, a] + rest[3:12], np.int32))  # inside the window
        inds.append(np.asarray(rest[:10] + [a, b] + rest[10:14], np.int32))  # past the window
    offs, cc = gen.csr(inds)
    mat = ctx.upload(X)
    try:
        for shape in ((1, 4, 13, 0), (1, 8, 25, 0), (1, 16, 200, 0)):
            ctx.set_launch_shape(shape[0], shape[1], shape[2], ebic.STAGE_PAIRS, shape[3])
            for include in (False, True):
                for negative in (True, False):
                    announce("pairs sparse ties", cols, shape, include, negative)
                    got = gpu_eval(ctx, mat, offs, cc, include=include, negative=negative, masks=True)
                    want = oracle_eval(X, offs, cc, include=include, negative=negative, masks=True)
                    assert_same(got, want, f"sparse ties cols={cols} {shape} include={include} neg={negative}")
    finally:
        ctx.set_launch_shape()
        ctx.release(mat)


def test_pairs_batched_mixed(ctx):
    """One batch: requests on two matrices (64 columns with ties and NaN, 300
    tie-free columns) in both modes, with and without negative trends and
    masks, an empty population, invalid individuals, and requests on a
    600-column matrix (past the default width: the tiled kernel) in the same
    launch; then a smaller batch on the same stream (the captured graph
    again). Each result equals the oracle's."""
    import torch
    from paper_1807_09932_amd import ebic
    rng = np.random.default_rng(77)
    Xa = rng.integers(0, 9, size=(9_001, 64)).astype(np.float32)
    Xa[rng.random(Xa.shape) < 0.02] = np.float32(np.nan)
    Xb = _tie_free(15_000, 300, 78)
    Xc = rng.standard_normal((3_000, 600)).astype(np.float32)
    mats = {k: ctx.upload(X, fill=0.75) for k, X in (("a", Xa), ("b", Xb), ("c", Xc))}
    Xs = {"a": Xa, "b": Xb, "c": Xc}
    jobs = []
    for q in range(14):
        key = "abc"[q % 3]
        cols = Xs[key].shape[1]
        n = 0 if q == 5 else int(rng.integers(20, 300))
        offs, cc = _pop(rng, cols, n, kmax=24) if n else gen.csr([])
        jobs.append((key, offs, cc, q % 2 == 1, q % 4 != 3, q % 5 == 0))
    s = torch.cuda.Stream()
    try:
        for rnd, sub in enumerate((jobs, jobs[:6])):
            reqs, outs, held = [], [], []
            for key, offs, cc, include, negative, masks in sub:
                pop = ctx.population(offsets=offs, cols=cc)
                o = ctx.outputs(mats[key], pop.n, masks=masks, negative=True)
                held.append(pop)
                outs.append(o)
                reqs.append(ctx.request(mats[key], pop, o, include=include, negative=negative))
            stg = ebic.ebic_plan_batch_shape(ctx.handle, reqs)[3]
            for (key, offs, *_), st in zip(sub, stg):
                if offs.size > 1:
                    assert (st == ebic.STAGE_PAIRS) == (key != "c"), (key, st)
            announce("pairs batched mixed", rnd, len(sub))
            ctx.eval_batch(reqs, stream=s)
            s.synchronize()
            for (key, offs, cc, include, negative, masks), o in zip(sub, outs):
                got = tuple(t.cpu().numpy() if t is not None else None for t in o)
                got = tuple(g.view(np.uint64) if g is not None and g.dtype == np.int64 else g for g in got)
                want = oracle_eval(Xs[key], offs, cc, include=include, negative=negative, masks=masks, fill=0.75)
                if not negative:
                    got = (got[0], None, got[2], got[3])
                if not masks:
                    got = (got[0], got[1], None, None)
                assert_same(got, want, f"round {rnd} matrix {key} include={include} negative={negative}")
    finally:
        for m in mats.values():
            ctx.release(m)


def test_pairs_allocation_failure_falls_back():
    """A failed allocation of the bitmaps (injected with EBIC_FAULT at each
    allocation in turn) leaves the matrix on its rank codes: the call that
    would have built them evaluates on the codes, later plans do not offer
    the bitmaps again, and the counts are exact throughout."""
    import os
    import torch
    from paper_1807_09932_amd import ebic
    from paper_1807_09932_amd.ebic import Context
    rng = np.random.default_rng(55)
    X = rng.standard_normal((5_000, 48)).astype(np.float32)
    offs, cc = _pop(rng, 48, 80, kmax=16)
    want = oracle_eval(X, offs, cc, negative=True, masks=False)
    fell_back = 0
    for after in range(0, 8):
        old = os.environ.pop("EBIC_FAULT", None)
        os.environ["EBIC_FAULT"] = f"alloc:{after}"
        try:
            ctx = Context(0)
        finally:
            os.environ.pop("EBIC_FAULT", None)
            if old is not None:
                os.environ["EBIC_FAULT"] = old
        try:
            announce("pairs alloc fault", after)
            try:
                mat = ctx.upload(X)
            except ebic.EbicError as e:
                assert e.status == ebic.EBIC_ENOMEM
                mat = ctx.upload(X)
            for _ in range(2):
                try:
                    got = gpu_eval(ctx, mat, offs, cc, negative=True, masks=False)
                except ebic.EbicError as e:  # (a failure of another allocation: the call fails whole)
                    assert e.status == ebic.EBIC_ENOMEM
                    got = gpu_eval(ctx, mat, offs, cc, negative=True, masks=False)
                assert_same((got[0], got[1], None, None), want, f"alloc fault {after}")
            if not ctx.stats(mat)["code_sets"] & ebic.SET_PAIRS:
                fell_back += 1
                assert ebic.ebic_plan_shape(ctx.handle, mat, offs.size - 1)[3] != ebic.STAGE_PAIRS
            torch.cuda.synchronize()
            ctx.release(mat)
        finally:
            ctx.close()
    assert fell_back >= 1, "no injected failure reached the bitmap allocation"
