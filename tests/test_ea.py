"""The stand-in evolutionary driver (host code in libebic.so): validity of
every generation, determinism, elitism. Counts come from the CPU oracle, so
these run without a GPU."""
import numpy as np
import pytest

import oracle
from paper_1807_09932_amd import ebic, gen


def _check_population(offs, cols, n, n_cols, k_min, k_max):
    assert offs.size == n + 1 and offs[0] == 0
    lens = np.diff(offs)
    assert lens.min() >= k_min and lens.max() <= k_max
    assert cols.size == offs[-1]
    assert cols.min() >= 0 and cols.max() < n_cols
    for i in range(n):
        ind = cols[offs[i]:offs[i + 1]]
        assert np.unique(ind).size == ind.size, f"individual {i} repeats a column"


def _counts(X, offs, cols):
    m, _, _, _ = oracle.eval_population(X, offs, cols, negative=True, threads=4)
    return m


@pytest.fixture(scope="module")
def small():
    w = gen.make_matrix(60, 2000, 24, "uniform", 2, (200, 200), (6, 6))
    return w


def test_generations_stay_valid(small):
    ea = ebic.EA(24, 64, 2, 8, seed=11)
    for g in range(15):
        offs, cols, gen_no = ea.population()
        assert gen_no == g
        _check_population(offs, cols, 64, 24, 2, 8)
        ea.step(_counts(small.X, offs, cols))


def test_same_seed_same_run_and_other_seed_differs(small):
    def run(seed):
        ea = ebic.EA(24, 48, 3, 10, seed=seed)
        hist = []
        for _ in range(6):
            offs, cols, _ = ea.population()
            hist.append((offs.copy(), cols.copy()))
            ea.step(_counts(small.X, offs, cols))
        return hist
    a, b, c = run(5), run(5), run(6)
    for (o1, c1), (o2, c2) in zip(a, b):
        assert np.array_equal(o1, o2) and np.array_equal(c1, c2)
    assert any(not np.array_equal(x[1], y[1]) or not np.array_equal(x[0], y[0])
               for x, y in zip(a, c))


def test_elitism_keeps_the_best(small):
    ea = ebic.EA(24, 64, 2, 8, elite=2, seed=3)
    best = []
    for _ in range(12):
        offs, cols, _ = ea.population()
        bi, bf = ea.step(_counts(small.X, offs, cols))
        best.append(bf)
        # the best individual of this generation is the first of the next
        nxt, ncols, _ = ea.population()
        assert np.array_equal(ncols[nxt[0]:nxt[1]], cols[offs[bi]:offs[bi + 1]])
    assert all(b2 >= b1 for b1, b2 in zip(best, best[1:]))


def test_invalid_individuals_rank_last(small):
    ea = ebic.EA(24, 16, 2, 4, elite=1, seed=9)
    offs, cols, _ = ea.population()
    m = np.full(16, -1, np.int32)
    m[7] = 0  # the only valid one, with no matched row
    bi, bf = ea.step(m)
    assert bi == 7 and bf == 0.0


def test_rejects_bad_parameters():
    with pytest.raises(ebic.EbicError):
        ebic.EA(10, 10, 5, 3)         # k_min > k_max
    with pytest.raises(ebic.EbicError):
        ebic.EA(10, 1, 2, 4)          # population of one
    ea = ebic.EA(10, 8, 2, 4, seed=1)
    with pytest.raises(ValueError):
        ea.step(np.zeros(7, np.int32))
