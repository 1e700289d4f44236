"""The batched path (one persistent launch replayed from a HIP graph) against
the CPU oracle, per request, bit-exact; and against the plain path."""
import numpy as np
import pytest

from paper_1807_09932_amd import gen
from tests.gpu_common import announce, assert_same, oracle_eval, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1807_09932_amd.ebic import Context
    c = Context(0)
    yield c
    c.close()


def _pops(seed, ncols, n_pops, n_range, length_fn):
    rng = np.random.default_rng(seed)
    pops = []
    for _ in range(n_pops):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        inds = [rng.choice(ncols, max(1, min(ncols, length_fn(rng))), replace=False).astype(np.int32)
                for _ in range(n)]
        pops.append(gen.csr(inds))
    return pops


def _run_batch(ctx, jobs, stream=None, plan=None):
    """jobs: list of (matrix handle, (offs, cols), include, negative, masks).
    If `plan` is a list, the batch's planned launch shape is appended to it."""
    import torch
    from paper_1807_09932_amd import ebic
    reqs, outs = [], []
    for mat, (offs, cols), include, negative, masks in jobs:
        pop = ctx.population(offsets=offs, cols=cols)
        out = ctx.outputs(mat, pop.n, masks=masks, negative=True)
        outs.append((pop, out))
        reqs.append(ctx.request(mat, pop, out, include=include, negative=negative))
    if plan is not None:
        plan.append(ebic.ebic_plan_batch_shape(ctx.handle, reqs))
    ctx.eval_batch(reqs, stream=stream)
    torch.cuda.synchronize()
    return [tuple(to_np(t) for t in out) for _, out in outs]


def test_batched_skewed_populations(ctx):
    """The batched 100,000 x 256 workload, reduced: uneven population sizes, lengths 2..40
    skewed toward short, one N(0,1) matrix with planted trends."""
    w = gen.make_matrix(4, 20000, 256, "normal", 8, (100, 1000), (4, 12))
    pops = _pops(41, 256, 24, (5, 400), gen.skewed_length)
    mat = ctx.upload(w.X)
    jobs = [(mat, p, False, True, i % 3 == 0) for i, p in enumerate(pops)]
    announce("batch skewed")
    got = _run_batch(ctx, jobs)
    for i, (p, g) in enumerate(zip(pops, got)):
        want = oracle_eval(w.X, *p, negative=True, masks=jobs[i][4])
        assert_same(g, want, f"request {i}")
    # the plain path gives the same numbers
    for i in (0, 5, 17):
        pop = ctx.population(offsets=pops[i][0], cols=pops[i][1])
        out = ctx.eval(mat, pop, negative=True, masks=jobs[i][4])
        import torch
        torch.cuda.synchronize()
        assert_same(tuple(to_np(t) for t in out), got[i], f"plain vs batch {i}")
    ctx.release(mat)


def test_batched_many_matrices_and_modes(ctx):
    rng = np.random.default_rng(42)
    mats, Xs = [], []
    for rows, ncols in [(3000, 40), (700, 310), (1500, 700), (64, 5)]:
        X = rng.standard_normal((rows, ncols)).astype(np.float32)
        X[:, ::4] = np.round(X[:, ::4])
        X[rng.random(X.shape) < 0.03] = np.float32(np.nan)
        Xs.append(X)
        mats.append(ctx.upload(X, fill=0.5))
    jobs, want = [], []
    for q in range(20):
        m = q % len(mats)
        ncols = Xs[m].shape[1]
        (offs, cols), = _pops(100 + q, ncols, 1, (0 if q == 7 else 3, 150),
                              lambda r: int(r.integers(1, 26)))
        include, negative, masks = bool(q & 1), bool(q & 2), bool(q & 4)
        jobs.append((mats[m], (offs, cols), include, negative, masks))
        want.append(oracle_eval(Xs[m], offs, cols, include=include, negative=negative,
                                masks=masks, fill=0.5))
    announce("batch many matrices")
    got = _run_batch(ctx, jobs)
    for q in range(len(jobs)):
        assert_same(got[q], want[q], f"request {q}")
    # the same batch in another order gives the same per-request results
    order = np.random.default_rng(5).permutation(len(jobs))
    announce("batch shuffled")
    got2 = _run_batch(ctx, [jobs[i] for i in order])
    for k, i in enumerate(order):
        assert np.array_equal(got2[k][0], got[i][0])
        assert np.array_equal(got2[k][1], got[i][1])
    for m in mats:
        ctx.release(m)


@pytest.mark.parametrize("tiles", [4, 2])
def test_batch_byte_codes(ctx, tiles):
    """The batched kernel with the SWAR codes forced: requests on a matrix
    without missing cells (byte codes in both modes), on one with them (byte
    codes in include mode only) and on a 230-column one (16-bit codes),
    masks on and off. Batches stage byte codes at four tiles per wave and
    16-bit codes at two; other requests take the FP16 codes, the FP32 tile
    or direct reads."""
    from paper_1807_09932_amd import ebic
    rng = np.random.default_rng(44)
    Xa = rng.integers(0, 7, size=(4099, 64)).astype(np.float32)
    Xb = rng.standard_normal((1030, 100)).astype(np.float32)
    Xb[rng.random(Xb.shape) < 0.03] = np.float32(np.nan)
    Xc = np.round(rng.standard_normal((2050, 230)), 1).astype(np.float32)  # 16-bit codes, ties
    mats = [ctx.upload(Xa), ctx.upload(Xb, fill=0.25), ctx.upload(Xc)]
    Xs = [Xa, Xb, Xc]
    jobs, want = [], []
    for q in range(18):
        m = q % 3
        (offs, cols), = _pops(300 + q, Xs[m].shape[1], 1, (1, 220), lambda r: int(r.integers(1, 31)))
        include, negative, masks = bool(q & 2), bool(q & 4), bool(q & 1)
        jobs.append((mats[m], (offs, cols), include, negative, masks))
        want.append(oracle_eval(Xs[m], offs, cols, include=include, negative=negative, masks=masks,
                                fill=0.25))
    try:
        ctx.set_launch_shape(tiles, 8, 128, ebic.STAGE_BYTES, 0)
        announce("batch byte codes", tiles)
        plan = []
        got = _run_batch(ctx, jobs, plan=plan)
        for q in range(len(jobs)):
            assert_same(got[q], want[q], f"request {q}")
        L, W, P, stagings, _ = plan[0]
        assert (L, W, P) == (tiles, 8, 128)
        for q, (m, _, include, _, _) in enumerate(jobs):
            k = mats.index(m)
            # SWAR codes take their own number of sub-tiles whatever the
            # batch's: byte codes on the 64- and 100-column matrices (the
            # latter has missing cells, so exclude mode takes its FP16 codes
            # there, at the batch's tiles); 10-bit codes on the 230-column one
            if k == 2:
                expect = ebic.STAGE_T10
            elif k == 0 or include:
                expect = ebic.STAGE_BYTES
            else:
                expect = ebic.STAGE_CODES
            assert stagings[q] == expect, (q, k, include, stagings[q])
    finally:
        ctx.set_launch_shape()
        for m in mats:
            ctx.release(m)


def test_batch_graph_replays_with_eager_work_between(ctx):
    """One captured graph replayed for batches of different contents, with
    plain evaluations and synchronisations between the replays; every
    replay is checked against the oracle."""
    import torch
    rng = np.random.default_rng(43)
    X = rng.random((5000, 64)).astype(np.float32)
    mat = ctx.upload(X)
    for rep in range(4):
        pops = _pops(200 + rep, 64, 6 + rep, (20, 200), lambda r: int(r.integers(2, 31)))
        jobs = [(mat, p, False, True, rep % 2 == 0) for p in pops]
        announce("graph replay", rep)
        got = _run_batch(ctx, jobs)
        for i, p in enumerate(pops):
            assert_same(got[i], oracle_eval(X, *p, masks=rep % 2 == 0), f"replay {rep} req {i}")
        # eager work between replays
        pop = ctx.population(offsets=pops[0][0], cols=pops[0][1])
        out = ctx.eval(mat, pop)
        torch.cuda.synchronize()
        assert np.array_equal(to_np(out[0]), got[0][0])
    ctx.release(mat)


def test_batch_invalid_and_empty(ctx):
    X = np.arange(600, dtype=np.float32).reshape(100, 6)[::-1].copy()
    mat = ctx.upload(X)
    p1 = gen.csr([[0, 1], [], [0, 6], [5, 4, 3], [2]])
    p2 = gen.csr([])
    p3 = gen.csr([[3, 3], [-2]])
    jobs = [(mat, p1, False, True, True), (mat, p2, False, True, True), (mat, p3, True, True, True)]
    announce("batch invalid/empty")
    got = _run_batch(ctx, jobs)
    assert_same(got[0], oracle_eval(X, *p1), "p1")
    assert got[1][0].size == 0
    assert_same(got[2], oracle_eval(X, *p3, include=True), "p3")
    ctx.release(mat)


def test_batch_matches_plain_on_batched_100000x256_sample(ctx):
    """Three populations of the full batched workload (100,000 x 256)."""
    w, pops = gen.batched_100000x256(n_pops=3)
    mat = ctx.upload(w.X)
    packed = [gen.csr(p) for p in pops]
    jobs = [(mat, p, False, True, False) for p in packed]
    announce("batched_100000x256 sample batch")
    got = _run_batch(ctx, jobs)
    for i, p in enumerate(packed):
        assert_same(got[i], oracle_eval(w.X, *p, masks=False), f"batched_100000x256 pop {i}")
    ctx.release(mat)


def test_plan_batch_shape_reports_and_rejects(ctx):
    """ebic_plan_batch_shape: the planned shape of a valid batch, and the
    same validation errors as ebic_eval_batch, with nothing launched."""
    from paper_1807_09932_amd import ebic
    rng = np.random.default_rng(45)
    X = rng.standard_normal((3000, 64)).astype(np.float32)
    mat = ctx.upload(X)
    try:
        (offs, cols), = _pops(450, 64, 1, (10, 40), lambda r: int(r.integers(2, 20)))
        pop = ctx.population(offsets=offs, cols=cols)
        out = ctx.outputs(mat, pop.n)
        req = ctx.request(mat, pop, out)
        ctx.set_launch_shape(4, 8, 128, ebic.STAGE_BYTES, 0)
        L, W, P, stagings, blocks = ebic.ebic_plan_batch_shape(ctx.handle, [req, req])
        assert (L, W, P) == (4, 8, 128) and stagings == [ebic.STAGE_BYTES] * 2 and blocks >= 1
        with pytest.raises(ebic.EbicError):
            ebic.ebic_plan_batch_shape(ctx.handle, [])
        bad = ctx.request(mat, pop, out)
        bad.flags = 1 << 7  # not a defined flag
        with pytest.raises(ebic.EbicError):
            ebic.ebic_plan_batch_shape(ctx.handle, [req, bad])
        bad = ctx.request(mat, pop, out)
        bad.matrix = 987654  # no such matrix
        with pytest.raises(ebic.EbicError):
            ebic.ebic_plan_batch_shape(ctx.handle, [bad])
    finally:
        ctx.set_launch_shape()
        ctx.release(mat)
