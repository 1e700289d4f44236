"""A CPU model of the SWAR rank-code arithmetic that the byte, 10-bit and
16-bit evaluation sequences run, checked against the oracle (no GPU).

The model restates, word by word in uint32 arithmetic, what the sequences
compute on rank codes (per row, the number of cells of the row that are
strictly smaller; codes below 2^(BITS-1), 32 // BITS rows per 32-bit word,
the 10-bit fields leaving bits 30-31 unused):

* the first pair: D = (t1 | H) - t0 and E = (t0 | H) - t1, whose part top
  bits say t1 >= t0 and t0 >= t1 (no borrow crosses a part);
* the tied variant: rows with both bits are tied and also run the <= chain;
  a falling row (E without D) mirrors its codes;
* the tie-free variant (for chunks in which no row holds two equal values):
  a row that does not rise falls, and no row is tied;
* every later column: alive &= (x_j | H) - x_{j-1} on the oriented codes.

The counts it gives are compared with the oracle's on the same matrix. This
pins the case where the tie-free variant alone is wrong: an individual whose
first two columns are the same column compares a cell with itself, so its
first pair is tied in every row, whatever the matrix holds. The evaluation
drops such a leading run in its prep step (c, c, ..., c, rest selects the
rows of c, rest), and the model shows that this makes the tie-free variant
exact again.
"""
import numpy as np
import pytest

import oracle

M32 = np.uint64(0xFFFFFFFF)


def _consts(bits):
    parts = 32 // bits
    H = sum(1 << (bits * p + bits - 1) for p in range(parts))
    return parts, np.uint64(H), bits - 1


def rank_codes(X):
    """Per cell, the number of cells of its row that are strictly smaller."""
    s = np.sort(X, axis=1)
    return np.stack([np.searchsorted(s[r], X[r], side="left") for r in range(X.shape[0])]).astype(np.uint64)


def pack(codes_col, bits):
    """One column of codes -> uint32 words (rows w*parts + p in part p)."""
    parts = 32 // bits
    n = codes_col.size
    pad = (-n) % parts
    c = np.concatenate([codes_col, np.zeros(pad, np.uint64)]).reshape(-1, parts)
    w = np.zeros(c.shape[0], np.uint64)
    for p in range(parts):
        w |= c[:, p] << np.uint64(bits * p)
    return w, n


def sub(a, b):
    """32-bit wrap-around a - b."""
    return (a + (M32 + np.uint64(1)) - b) & M32


def swar_eval(codes, ind, bits, ties):
    """(matched, negative) of one individual, NEG on, all rows in range."""
    parts, H, shf = _consts(bits)
    words = [pack(codes[:, c], bits)[0] for c in ind]
    rows = codes.shape[0]
    hv = np.full(words[0].shape, H, np.uint64)
    pad_rows = words[0].size * parts - rows
    if pad_rows:  # parts past the last row are out of range
        keep = np.uint64(sum(1 << (bits * p + bits - 1) for p in range(parts - pad_rows)))
        hv[-1] = keep
    if len(ind) == 1:
        mw, gw = hv, np.zeros_like(hv)
    else:
        t0, t1 = words[0], words[1]
        D = sub(t1 | H, t0)
        E = sub(t0 | H, t1)
        if ties:
            tied = D & E & hv
            fall = E & ~D & hv & M32
        else:
            tied = np.zeros_like(hv)
            fall = ~D & hv & M32
        fm = sub(fall, fall >> np.uint64(shf))
        alive = hv.copy()
        prev = t1 ^ fm
        for t in words[2:]:
            x = t ^ fm
            alive &= sub(x | H, prev)
            prev = x
        if len(ind) >= 3:
            tp = t1
            for t in words[2:]:  # the <= chain of the tied rows: t_{j-1} >= t_j
                tied &= sub(tp | H, t)
                tp = t
        else:  # two columns: a tied row is on the >= chain already
            tied = np.zeros_like(hv)
        alive &= hv
        tied &= hv
        mw = (alive | tied) & H
        gw = ((alive & fall) | (tied & ~alive & M32)) & H
    popc = lambda w: int(sum(bin(int(v)).count("1") for v in w))
    return popc(mw), popc(gw)


def strip_leading_repeats(ind):
    """What the prep step keeps: the last entry of the leading run of ind[0]."""
    s = 0
    while s + 1 < len(ind) and ind[s + 1] == ind[0]:
        s += 1
    return ind[s:]


def _tie_free_matrix(rows, cols, seed):
    """N(0,1) in float32, rows with two equal values drawn again."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((rows, cols)).astype(np.float32)
    while True:
        bad = (np.diff(np.sort(X, axis=1), axis=1) == 0).any(axis=1)
        if not bad.any():
            return X
        X[bad] = rng.standard_normal((int(bad.sum()), cols)).astype(np.float32)


def _individuals(rng, cols, n):
    inds = []
    for i in range(n):
        k = int(rng.integers(3, 12))
        ind = list(rng.permutation(cols)[:k])
        kind = i % 4
        if kind == 0:
            ind = [ind[0]] + ind              # a, a, b, ...
        elif kind == 1:
            ind = [ind[0]] * 3 + ind[1:]      # a, a, a, b, ...
        elif kind == 2:
            ind = [ind[0], ind[0]]            # a, a
        inds.append([int(c) for c in ind])
    return inds


@pytest.mark.parametrize("bits,cols", [(8, 64), (8, 128), (16, 200), (16, 310), (10, 200), (10, 310),
                                       (10, 512)])
def test_tie_free_variant_needs_the_leading_run_dropped(bits, cols):
    rows = 700 if bits == 8 else 351
    X = _tie_free_matrix(rows, cols, 40 + cols)
    codes = rank_codes(X)
    assert int(codes.max()) < 2 ** (bits - 1)
    rng = np.random.default_rng(cols)
    inds = _individuals(rng, cols, 40)
    from paper_1807_09932_amd import gen
    offs, cc = gen.csr([np.asarray(i, np.int32) for i in inds])
    om, on, _, _ = oracle.eval_population(X, offs, cc, negative=True)
    wrong = 0
    for i, ind in enumerate(inds):
        want = (int(om[i]), int(on[i]))
        assert swar_eval(codes, ind, bits, ties=True) == want, ind
        assert swar_eval(codes, strip_leading_repeats(ind), bits, ties=False) == want, ind
        if swar_eval(codes, ind, bits, ties=False) != want:
            wrong += 1
            assert ind[0] == ind[1], "only a repeated first column may break the tie-free variant"
    # the case is reached: the tie-free variant without the prep step is wrong
    assert wrong > 0


def test_model_agrees_on_ties():
    """On a tie-heavy matrix (integers) the tied variant is exact for every
    individual, repeated columns included."""
    rng = np.random.default_rng(3)
    X = rng.integers(0, 5, size=(300, 20)).astype(np.float32)
    codes = rank_codes(X)
    inds = [[int(c) for c in rng.integers(0, 20, size=int(rng.integers(1, 9)))] for _ in range(60)]
    from paper_1807_09932_amd import gen
    offs, cc = gen.csr([np.asarray(i, np.int32) for i in inds])
    om, on, _, _ = oracle.eval_population(X, offs, cc, negative=True)
    for bits in (8, 10, 16):
        for i, ind in enumerate(inds):
            assert swar_eval(codes, ind, bits, ties=True) == (int(om[i]), int(on[i])), (bits, ind)
