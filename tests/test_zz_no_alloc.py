"""ebic_eval_population_noalloc (the entry point for callers that cannot
allocate device memory) against ebic_eval_population on the same inputs,
bit-exact, through the C ABI: two calls in a row on one stream, the second
with a smaller population, and the size limit."""
import numpy as np
import pytest

from tests.gpu_common import announce, assert_same, oracle_eval, to_np

pytestmark = pytest.mark.gpu


def _outputs(torch, n, words, dev):
    return (torch.full((n,), 7, dtype=torch.int32, device=dev),
            torch.full((n,), 7, dtype=torch.int32, device=dev),
            torch.full((n, words), 7, dtype=torch.int64, device=dev),
            torch.full((n, words), 7, dtype=torch.int64, device=dev))


def _call(ebic, fn, ctx, mat, pop, flags, out, stream):
    m, g, mm, nm = out
    fn(ctx.handle, mat, pop.n, pop.offsets.data_ptr(), pop.cols.data_ptr(), flags, m.data_ptr(),
       g.data_ptr(), mm.data_ptr(), nm.data_ptr(), stream)


def test_noalloc_equals_eval_population():
    import torch
    from paper_1807_09932_amd import ebic, gen
    dev = torch.device("cuda", 0)
    with ebic.Context(0) as ctx:
        # a methylation-shaped matrix (byte codes) with 800 individuals, then
        # a smaller population on a wider matrix with missing cells
        w1 = gen.make_matrix(11, 30_000, 64, "beta", 6, (500, 3000), (4, 12), directions="alternate")
        p1 = gen.make_population(11, 1, 64, 800, (2, 30), w1.plants)
        w2 = gen.make_matrix(12, 5_003, 200, "normal", 3, (100, 400), (5, 10))
        X2 = w2.X.copy()
        X2[np.random.default_rng(12).random(X2.shape) < 0.02] = np.float32(np.nan)
        p2 = gen.make_population(12, 1, 200, 150, (1, 20), w2.plants)
        cases = [(w1.X, p1, ctx.flags(include=False, negative=True)),
                 (X2, p2, ctx.flags(include=True, negative=True))]
        mats, pops, outs_na, outs_ref = [], [], [], []
        for X, inds, flags in cases:
            offs, cols = gen.csr(inds)
            mat = ctx.upload(X, fill=0.5)
            pop = ctx.population(offsets=offs, cols=cols)
            words = ebic.ebic_mask_words(X.shape[0])
            mats.append(mat)
            pops.append((pop, offs, cols))
            outs_na.append(_outputs(torch, pop.n, words, dev))
            outs_ref.append(_outputs(torch, pop.n, words, dev))
        stream = torch.cuda.Stream()
        sh = stream.cuda_stream
        torch.cuda.synchronize()
        before = torch.cuda.memory_stats(dev).get("allocation.all.allocated", 0)
        # two calls in a row on one stream, the second smaller
        for (X, _, flags), mat, (pop, _, _), out in zip(cases, mats, pops, outs_na):
            announce("noalloc", X.shape, pop.n)
            _call(ebic, ebic.ebic_eval_population_noalloc, ctx, mat, pop, flags, out, sh)
        stream.synchronize()
        after = torch.cuda.memory_stats(dev).get("allocation.all.allocated", 0)
        assert after == before, "the no-allocation entry point allocated device memory"
        for (X, _, flags), mat, (pop, offs, cols), out_na, out_ref in zip(cases, mats, pops, outs_na,
                                                                         outs_ref):
            announce("eval_population", X.shape, pop.n)
            _call(ebic, ebic.ebic_eval_population, ctx, mat, pop, flags, out_ref, sh)
            stream.synchronize()
            got = tuple(to_np(t) for t in out_na)
            ref = tuple(to_np(t) for t in out_ref)
            assert_same(got, ref, f"noalloc vs eval_population {X.shape}")
            include = bool(flags & ebic.EBIC_NAN_INCLUDE)
            assert_same(got, oracle_eval(X, offs, cols, include=include, fill=0.5),
                        f"noalloc vs oracle {X.shape}")
        # above the limit: refused before anything is enqueued
        big = 65_537
        offs = np.arange(big + 1, dtype=np.int32)
        cols = np.zeros(big, np.int32)
        pop = ctx.population(offsets=offs, cols=cols)
        m = torch.full((big,), 7, dtype=torch.int32, device=dev)
        with pytest.raises(ebic.EbicError) as e:
            ebic.ebic_eval_population_noalloc(ctx.handle, mats[0], big, pop.offsets.data_ptr(),
                                              pop.cols.data_ptr(), 0, m.data_ptr(), None, None, None, sh)
        assert e.value.status == ebic.EBIC_EINVAL and "65536" in str(e.value)
        torch.cuda.synchronize()
        assert int(m.min()) == 7 and int(m.max()) == 7
        for mat in mats:
            ctx.release(mat)
