"""Breeding on the device (ebic_ea_breed) against the host driver
(ebic_ea_step): from the same population and the same counts, every
generation bred on the device equals the host's column for column, and
the counts of the evolving population equal the oracle's. Also a loop that
alternates evaluation and breeding on one stream with no host round trip,
parameter corners (no elites, no crossover, always crossover, fixed
length, k_max = n_cols, two individuals; populations bred by one
workgroup and, above 1,024 individuals, by the five-kernel path, with
children built in LDS or, for k_max above 64, in global memory), caller-made populations with
invalid and over-long individuals, and argument errors."""
import numpy as np
import pytest

from paper_1807_09932_amd import ebic, gen
from tests.gpu_common import announce, oracle_eval, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1807_09932_amd.ebic import Context
    c = Context(0)
    yield c
    c.close()


def _host_pop(ea):
    offs, cols, g = ea.population()
    return offs, cols, g


def _device_pop(pop):
    offs = to_np(pop.offsets)
    return offs, to_np(pop.cols)[: int(offs[-1])]


def _same(host, dev, what):
    ho, hc = host[0], host[1]
    do, dc = dev
    assert np.array_equal(ho, do), f"{what}: offsets differ"
    assert np.array_equal(hc, dc), f"{what}: columns differ"


@pytest.mark.parametrize("workload,include", [("methylation", False), ("missing", True)])
def test_device_breeding_equals_host(ctx, workload, include):
    import torch
    w = (gen.methylation_436444x64()[0] if workload == "methylation"
         else gen.normal_missing_20000x200()[0])
    rows, n_cols = w.X.shape
    mat = ctx.upload(w.X)
    ea = ebic.EA(n_cols, 400, 2, 30, seed=77 + len(workload))
    try:
        host = _host_pop(ea)
        pop = ctx.population(offsets=host[0], cols=host[1])
        for g in range(1, 7):
            announce("breed", workload, g)
            m, neg, _, _ = ctx.eval(mat, pop, include=include, negative=True)
            torch.cuda.synchronize()
            om, on, _, _ = oracle_eval(w.X, host[0], host[1], include=include, negative=True, masks=False)
            assert np.array_equal(to_np(m), om), f"generation {g - 1}: matched differs from the oracle"
            assert np.array_equal(to_np(neg), on), f"generation {g - 1}: negative differs from the oracle"
            best_h, _ = ea.step(to_np(m))
            pop, best = ctx.breed(ea.params, g, pop, m)
            torch.cuda.synchronize()
            assert int(best.cpu()[0]) == best_h
            host = _host_pop(ea)
            assert host[2] == g
            _same(host, _device_pop(pop), f"generation {g}")
    finally:
        ea.close()
        ctx.release(mat)


def test_on_device_loop_matches_host_loop(ctx):
    """Ten generations alternating evaluation and breeding on one stream,
    synchronised only at the end, against the host-driven run."""
    import torch
    w, _ = gen.methylation_436444x64()
    X = w.X[:50_000]
    mat = ctx.upload(X)
    ea = ebic.EA(64, 800, 2, 30, seed=5)
    try:
        offs, cols, _ = ea.population()
        pop = ctx.population(offsets=offs, cols=cols)
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            bufs = [ctx.outputs(mat, 800, negative=False)[0] for _ in range(2)]
            for g in range(1, 11):
                m = bufs[g & 1]
                ctx.eval(mat, pop, negative=True, out=(m, None, None, None), stream=s)
                pop, _ = ctx.breed(ea.params, g, pop, m, stream=s)
        s.synchronize()
        announce("device loop done")
        for g in range(1, 11):
            ho, hc, _ = ea.population()
            hp = ctx.population(offsets=ho, cols=hc)
            m, _, _, _ = ctx.eval(mat, hp, negative=True)
            ea.step(to_np(m))
        _same(ea.population(), _device_pop(pop), "generation 10")
    finally:
        ea.close()
        ctx.release(mat)


@pytest.mark.parametrize("n_cols,pop,k_min,k_max,elite,pc,pm", [
    (24, 64, 2, 8, 0, 0.5, 0.9),
    (24, 64, 2, 8, 3, 0.0, 1.0),
    (24, 64, 2, 8, 3, 1.0, 0.0),
    (24, 64, 5, 5, 1, 0.7, 1.0),
    (6, 33, 1, 6, 2, 0.8, 1.0),
    (10, 2, 1, 10, 1, 1.0, 1.0),
    (300, 1500, 2, 40, 20, 0.5, 0.9),
    (100, 200, 2, 80, 5, 0.6, 0.9),
    (120, 1100, 2, 80, 10, 0.6, 0.9),  # over 1,024 and k_max above 64: children in global memory
])
def test_parameter_corners(ctx, n_cols, pop, k_min, k_max, elite, pc, pm):
    import torch
    rng = np.random.default_rng(n_cols * 7 + pop)
    X = rng.integers(0, 5, size=(700, n_cols)).astype(np.float32)
    mat = ctx.upload(X)
    ea = ebic.EA(n_cols, pop, k_min, k_max, elite=elite, p_crossover=pc, p_mutation=pm, seed=pop + elite)
    try:
        ho, hc, _ = ea.population()
        p = ctx.population(offsets=ho, cols=hc)
        for g in range(1, 6):
            announce("corner", n_cols, pop, k_min, k_max, elite, pc, pm, g)
            m, _, _, _ = ctx.eval(mat, p, negative=True)
            ea.step(to_np(m))
            p, _ = ctx.breed(ea.params, g, p, m)
            torch.cuda.synchronize()
            host = ea.population()
            _same(host, _device_pop(p), f"generation {g}")
            lens = np.diff(host[0])
            assert lens.min() >= k_min and lens.max() <= k_max
    finally:
        ea.close()
        ctx.release(mat)


def test_caller_made_population(ctx):
    """Invalid individuals (matched -1), empty and over-long ones, columns
    out of range: breeding is deterministic, the elites are the best
    parents cut to k_max columns, every other child is 1..k_max long, and
    the reported best is the rank order's first."""
    import torch
    n_cols, n = 20, 50
    params = ebic.ebic_ea_params(n_cols, n, 2, 6, 4, 0.6, 0.8, 12345)
    rng = np.random.default_rng(3)
    inds = []
    for i in range(n):
        k = int(rng.integers(0, 10))  # 0 (no columns) .. 9 (> k_max)
        ind = rng.integers(0, n_cols + 3, size=k).astype(np.int32)  # some out of range
        inds.append(ind)
    offs, cols = gen.csr(inds)
    matched = rng.integers(-1, 400, size=n).astype(np.int32)
    matched[::7] = -1
    pop = ctx.population(offsets=offs, cols=cols)
    mt = torch.from_numpy(matched).to(ctx.device)
    for g in (1, 2, 9):
        nxt, best = ctx.breed(params, g, pop, mt)
        torch.cuda.synchronize()
        # (the host driver cannot be given a caller-made population: a
        # second call and the rules' invariants stand in for it)
        again, _ = ctx.breed(params, g, pop, mt)
        torch.cuda.synchronize()
        _same(_device_pop(nxt), _device_pop(again), f"repeat of generation {g}")
        do, dc = _device_pop(nxt)
        lens = np.diff(do)
        # elites keep their (at most k_max) columns, even none; every other
        # child has at least one and at most k_max
        assert lens.max() <= 6 and lens[4:].min() >= 1
        f = np.where(matched < 0, -np.inf, matched * np.ldexp(1.0, np.diff(offs) - 2))
        f[matched == 0] = 0.0
        order = sorted(range(n), key=lambda i: (-f[i], i))
        assert int(best.cpu()[0]) == order[0]
        for e in range(4):  # elites: the best parents' first k_max columns
            src = cols[offs[order[e]]:offs[order[e] + 1]][:6]
            assert np.array_equal(dc[do[e]:do[e + 1]], src), f"elite {e}"


def test_breed_argument_errors(ctx):
    import torch
    params = ebic.ebic_ea_params(10, 4, 1, 3, 1, 0.5, 0.5, 1)
    offs, cols = gen.csr([[1, 2], [3], [4, 5, 6], [7]])
    pop = ctx.population(offsets=offs, cols=cols)
    m = torch.zeros(4, dtype=torch.int32, device=ctx.device)
    with pytest.raises(ebic.EbicError) as e:
        ctx.breed(params, 0, pop, m)  # generation 0 is the random first one
    assert e.value.status == ebic.EBIC_EINVAL
    bad = ebic.ebic_ea_params(10, 4, 3, 2, 1, 0.5, 0.5, 1)  # k_min > k_max
    with pytest.raises(ebic.EbicError):
        ctx.breed(bad, 1, pop, m)
    other = ebic.ebic_ea_params(10, 5, 1, 3, 1, 0.5, 0.5, 1)  # n_ind != pop_size
    with pytest.raises(ebic.EbicError):
        ctx.breed(other, 1, pop, m)
