"""The CPU oracle against facts the paper and mathematics fix (no GPU)."""
import numpy as np
import pytest

import oracle
from tests import oracle_pins as pins


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda f: f.__name__)
def test_oracle_pin(pin):
    pin(oracle.eval_population)


def test_oracle_threads_agree():
    from paper_1807_09932_amd import gen
    w, pop = gen.uniform_1000x50()
    offs, cols = gen.csr(pop)
    a = oracle.eval_population(w.X, offs, cols, masks=True, threads=1)
    b = oracle.eval_population(w.X, offs, cols, masks=True, threads=4)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_oracle_rejects_bad_args():
    X = np.zeros((4, 3), np.float32)
    offs = np.array([0, 2], np.int32)
    cols = np.array([0, 1], np.int32)
    with pytest.raises(ValueError):
        oracle.eval_population(X, offs, cols, include=True, fill=float("nan"))


def test_statistical_one_over_k_factorial():
    """iid continuous rows: the fraction on the positive trend is 1/k!."""
    import math
    rng = np.random.default_rng(16)
    rows = 200_000
    X = rng.random((rows, 6)).astype(np.float32)
    for k in (2, 3, 4, 5):
        m, n, _, _ = oracle.eval_population(X, np.array([0, k], np.int32),
                                            np.arange(k, dtype=np.int32), negative=False)
        p = 1 / math.factorial(k)
        sd = math.sqrt(rows * p * (1 - p))
        assert abs(m[0] - rows * p) < 6 * sd, (k, m[0], rows * p)
