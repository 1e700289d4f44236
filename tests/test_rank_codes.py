"""The rank codes used to stage wide matrices at half the bytes: a cell's
code is the number of cells of its row that are strictly smaller (IEEE <).
For every pair of non-missing values, a >= b exactly when code(a) >=
code(b), so the row-trend predicate on codes selects the same rows. Checked
here with numpy on special values (ties, +-0, +-inf, denormals) and on
random rows; codes are exact FP16 integers for up to 2048 columns."""
import numpy as np


def codes(row):
    r = row.astype(np.float32)
    return np.array([np.sum(r < v) for v in r], dtype=np.int64)


def test_order_is_preserved_on_special_values():
    vals = np.array([-np.inf, -3.0, -1.0, -0.0, 0.0, 1.4e-45, 2.8e-45, 1.0, 1.0, 7.5, np.inf],
                    dtype=np.float32)
    rng = np.random.default_rng(1)
    for _ in range(200):
        row = rng.choice(vals, size=12)
        c = codes(row)
        for i in range(row.size):
            for j in range(row.size):
                assert (row[i] >= row[j]) == (c[i] >= c[j])
                assert (row[i] == row[j]) == (c[i] == c[j])


def test_random_rows_and_fp16_exactness():
    rng = np.random.default_rng(2)
    for ncols in (2, 64, 310, 384):
        row = rng.standard_normal(ncols).astype(np.float32)
        row[:: 7] = np.round(row[:: 7])
        c = codes(row)
        assert c.max() <= ncols - 1
        assert np.array_equal(c.astype(np.float16).astype(np.int64), c)  # exact in FP16
        ge = row[:, None] >= row[None, :]
        assert np.array_equal(ge, c[:, None] >= c[None, :])
    assert np.float16(2047) == 2047 and np.float16(2048) == 2048
