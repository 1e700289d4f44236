"""Pins of the CPU oracle to facts outside its own code.

Each pin takes ``ev``, a function with the signature of
``oracle.eval_population``, so the same pins can be run against deliberately
broken copies of the oracle (see test_oracle_mutants.py). A pin raises
AssertionError when ``ev`` disagrees with what it pins.

What pins what (Methods, "Handling missing values": rows are counted when
the values in the individual's columns stand in a greater-or-equal relation;
missing values are either excluded or take part through a fill value):

* pin_multiset_count   -- combinatorics: over an alphabet of a values, the
  number of length-k sequences that are non-decreasing is C(a+k-1, k);
  exactly a of them are constant. Fixes ">=" (not ">"), the tie rule and
  every pair of the chain.
* pin_permutation_count -- over all k! orderings of k columns, a row whose
  values have multiplicities m_1..m_t is non-decreasing in prod(m_v!)
  orderings, and constant in all k! only if t == 1.
* pin_sort_reduction   -- a row follows an individual's positive trend iff
  its values along the individual equal Python's sorted() of them (and the
  negative trend iff they equal sorted(reverse=True)).
* pin_closed_forms     -- k = 1 and k = 2 in both missing-value modes, with
  NaN and with a sentinel.
* pin_constant_and_sorted_rows, pin_planted -- whole-matrix special cases.
* pin_invariants       -- bounds, prefix nesting, reversal, mode nesting,
  exact scaling, negation, row and column permutations.
* pin_invalid          -- the -1 convention for invalid individuals.
* pin_repeated_columns -- reflexivity of the relation (x >= x and x <= x
  for every present value): repeating a column in place, at the start or
  anywhere inside an individual, changes no count and no mask bit, in
  both missing-value modes.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from paper_1807_09932_amd import gen

NAN = np.float32(np.nan)


def _bits(mask_row: np.ndarray, rows: int) -> np.ndarray:
    """uint64 mask words -> bool per row."""
    b = np.unpackbits(mask_row.view(np.uint8), bitorder="little").astype(bool)
    return b[:rows]


def _csr(inds):
    return gen.csr(inds)


def _run(ev, X, inds, **kw):
    offs, cols = _csr(inds)
    return ev(X, offs, cols, masks=True, **kw)


def _pn_bits(m, n, i, rows):
    """(P, negative) bool vectors of individual i; P = matched & ~negative."""
    mb = _bits(m[i], rows)
    nb = _bits(n[i], rows)
    return mb & ~nb, nb, mb


# ---------------------------------------------------------------------------
def pin_multiset_count(ev):
    for a, k in [(2, 2), (3, 3), (4, 3), (3, 4), (2, 5), (5, 2)]:
        rows = np.array(list(itertools.product(range(a), repeat=k)), dtype=np.float32)
        X = rows  # column j holds the j-th element of every sequence
        ind = list(range(k))
        nondec = math.comb(a + k - 1, k)
        for include in (False, True):
            m, n, _, _ = _run(ev, X, [ind], include=include, negative=True)
            assert m[0] == 2 * nondec - a, (a, k, m[0])
            assert n[0] == nondec - a, (a, k, n[0])
            m, n, _, _ = _run(ev, X, [ind], include=include, negative=False)
            assert m[0] == nondec and n[0] == 0, (a, k, m[0], n[0])
        # the reversed column order sees the same multiset counts
        m, n, _, _ = _run(ev, X, [ind[::-1]], negative=True)
        assert m[0] == 2 * nondec - a and n[0] == nondec - a


def pin_permutation_count(ev):
    rng = np.random.default_rng(11)
    for k in (2, 3, 4, 5):
        X = rng.integers(0, 3, size=(60, 6)).astype(np.float32)
        X[:3] = 1.0  # a few constant rows
        S = [5, 0, 3, 1, 4][:k]
        perms = [list(p) for p in itertools.permutations(S)]
        m, n, mm, nm = _run(ev, X, perms, negative=True)
        P_sum = np.zeros(X.shape[0], np.int64)
        neg_sum = np.zeros(X.shape[0], np.int64)
        mat_sum = np.zeros(X.shape[0], np.int64)
        for i in range(len(perms)):
            P, nb, mb = _pn_bits(mm, nm, i, X.shape[0])
            P_sum += P
            neg_sum += nb
            mat_sum += mb
        for r in range(X.shape[0]):
            vals = X[r, S]
            mult = np.unique(vals, return_counts=True)[1]
            nondec = int(np.prod([math.factorial(int(c)) for c in mult]))
            const = math.factorial(k) if mult.size == 1 else 0
            assert P_sum[r] == nondec, (k, r, P_sum[r], nondec)
            assert neg_sum[r] == nondec - const, (k, r)
            assert mat_sum[r] == 2 * nondec - const, (k, r)
        assert int(m.sum()) == int(mat_sum.sum()) and int(n.sum()) == int(neg_sum.sum())


def _special_alphabet():
    return np.array([-np.inf, -1.0, -0.0, 0.0, 1.4e-45, 2.8e-45, 1.0, 2.0, np.inf],
                    dtype=np.float32)


def pin_sort_reduction(ev):
    rng = np.random.default_rng(12)
    alpha = _special_alphabet()
    for trial in range(4):
        rows, ncols = 200, 6
        if trial % 2 == 0:
            X = alpha[rng.integers(0, alpha.size, size=(rows, ncols))]
        else:
            X = rng.integers(0, 4, size=(rows, ncols)).astype(np.float32)
        inds = []
        for _ in range(40):
            k = int(rng.integers(1, 7))
            dup = rng.random() < 0.2
            inds.append(rng.integers(0, ncols, size=k) if dup else rng.permutation(ncols)[:k])
        for negative in (True, False):
            m, n, mm, nm = _run(ev, X, inds, negative=negative)
            for i, ind in enumerate(inds):
                mb = _bits(mm[i], rows)
                nb = _bits(nm[i], rows)
                for r in range(rows):
                    vals = [float(x) for x in X[r, ind]]
                    P = vals == sorted(vals)
                    N = negative and vals == sorted(vals, reverse=True)
                    assert mb[r] == (P or N), (trial, i, r, vals)
                    assert nb[r] == (N and not P), (trial, i, r, vals)
                assert m[i] == mb.sum() and n[i] == nb.sum()


def pin_closed_forms(ev):
    rng = np.random.default_rng(13)
    rows = 500
    X = rng.standard_normal((rows, 7)).astype(np.float32)
    X[rng.random((rows, 7)) < 0.15] = NAN
    X[rng.random((rows, 7)) < 0.05] = np.float32(999.0)
    X[:20, 2] = X[:20, 5]  # ties
    for sentinel in (float("nan"), 999.0):
        miss = np.isnan(X) | (X == np.float32(sentinel))
        for fill in (0.0, 999.0, -2.5):
            Xf = np.where(miss, np.float32(fill), X)
            for a in range(7):
                # k = 1
                m, n, _, _ = _run(ev, X, [[a]], include=False, sentinel=sentinel)
                assert m[0] == int((~miss[:, a]).sum()) and n[0] == 0
                m, n, _, _ = _run(ev, X, [[a]], include=True, sentinel=sentinel, fill=fill)
                assert m[0] == rows and n[0] == 0
                for b in range(7):
                    if b == a:
                        continue
                    ok = ~miss[:, a] & ~miss[:, b]
                    # k = 2, exclude: any two present values are ordered one way or the other
                    m, n, _, _ = _run(ev, X, [[a, b]], include=False, sentinel=sentinel)
                    assert m[0] == int(ok.sum()), (sentinel, a, b)
                    assert n[0] == int((ok & (X[:, b] < X[:, a])).sum())
                    m, n, _, _ = _run(ev, X, [[a, b]], include=False, sentinel=sentinel,
                                      negative=False)
                    assert m[0] == int((ok & (X[:, b] >= X[:, a])).sum()) and n[0] == 0
                    # k = 2, include: the fill value takes part in the comparison
                    m, n, _, _ = _run(ev, X, [[a, b]], include=True, sentinel=sentinel, fill=fill)
                    assert m[0] == rows
                    assert n[0] == int((Xf[:, b] < Xf[:, a]).sum())


def pin_constant_and_sorted_rows(ev):
    rng = np.random.default_rng(14)
    rows, ncols = 300, 12
    inds = [rng.permutation(ncols)[: int(rng.integers(1, 9))] for _ in range(30)]
    inds += [sorted(x) for x in inds[:10]] + [sorted(x, reverse=True) for x in inds[10:20]]
    for c in (0.0, -3.5, 7.0):
        X = np.full((rows, ncols), c, np.float32)
        for include in (False, True):
            m, n, _, _ = _run(ev, X, inds, include=include)
            assert np.all(m == rows) and np.all(n == 0)
    # every row strictly increasing along the column index
    X = np.cumsum(rng.random((rows, ncols)) + 0.1, axis=1).astype(np.float32)
    assert np.all(np.diff(X, axis=1) > 0)
    m, n, _, _ = _run(ev, X, inds)
    for i, ind in enumerate(inds):
        ind = list(ind)
        if len(ind) == 1:
            assert m[i] == rows and n[i] == 0
        elif ind == sorted(ind):
            assert m[i] == rows and n[i] == 0, i
        elif ind == sorted(ind, reverse=True):
            assert m[i] == rows and n[i] == rows, i
        else:
            assert m[i] == 0 and n[i] == 0, i


def pin_planted(ev):
    w = gen.make_matrix(901, 3000, 40, "uniform", 6, (50, 200), (3, 9), directions="alternate")
    inds = [p.cols for p in w.plants]
    m, n, mm, nm = _run(ev, w.X, inds)
    for i, p in enumerate(w.plants):
        mb = _bits(mm[i], w.X.shape[0])
        nb = _bits(nm[i], w.X.shape[0])
        assert mb[p.rows].all(), i
        if p.increasing:
            assert not nb[p.rows].any(), i
        else:
            assert nb[p.rows].all(), i
        assert m[i] >= p.rows.size


def pin_invariants(ev):
    rng = np.random.default_rng(15)
    rows, ncols = 700, 16
    X = rng.standard_normal((rows, ncols)).astype(np.float32)
    miss = rng.random((rows, ncols)) < 0.03
    Xn = X.copy()
    Xn[miss] = NAN
    inds = [rng.permutation(ncols)[: int(rng.integers(1, 12))] for _ in range(40)]
    m, n, mm, nm = _run(ev, Xn, inds)
    assert np.all(n >= 0) and np.all(n <= m) and np.all(m <= rows)
    # prefix: matched and |P| never decrease when the individual is cut short,
    # and the masks of the whole are contained in those of the prefix
    for i, ind in enumerate(inds):
        for include in (False, True):
            mw, nw, mmw, nmw = _run(ev, Xn, [ind], include=include)
            Pw = _bits(mmw[0], rows) & ~_bits(nmw[0], rows)
            for L in range(1, len(ind)):
                mp, np_, mmp, nmp = _run(ev, Xn, [ind[:L]], include=include)
                Pp = _bits(mmp[0], rows) & ~_bits(nmp[0], rows)
                assert mp[0] >= mw[0] and mp[0] - np_[0] >= mw[0] - nw[0]
                assert not (_bits(mmw[0], rows) & ~_bits(mmp[0], rows)).any()
                assert not (Pw & ~Pp).any()
    # reversal keeps matched and the matched mask
    mr, nr, mmr, _ = _run(ev, Xn, [ind[::-1] for ind in inds])
    assert np.array_equal(mr, m) and np.array_equal(mmr, mm)
    # exclude-mode mask = include-mode mask restricted to rows with no missing cell
    mi, ni, mmi, nmi = _run(ev, Xn, inds, include=True, fill=0.0)
    for i, ind in enumerate(inds):
        ex = _bits(mm[i], rows)
        inc = _bits(mmi[i], rows)
        clean = ~miss[:, ind].any(axis=1)
        assert np.array_equal(ex, inc & clean), i
    mc, _, mmc, _ = _run(ev, X, inds)
    mic, _, mmic, _ = _run(ev, X, inds, include=True, fill=5.0)
    assert np.array_equal(mmc, mmic) and np.array_equal(mc, mic)
    # exact scaling by 2 changes nothing
    m2, n2, mm2, nm2 = _run(ev, Xn * np.float32(2), inds)
    assert np.array_equal(m2, m) and np.array_equal(n2, n) and np.array_equal(mm2, mm)
    # negation swaps the trends: matched and its mask stay, negative becomes |P|
    mg, ng, mmg, nmg = _run(ev, -Xn, inds)
    assert np.array_equal(mg, m) and np.array_equal(mmg, mm)
    for i, ind in enumerate(inds):
        if len(ind) >= 2:  # distinct continuous values: no row is on both trends
            assert np.array_equal(_bits(nmg[i], rows),
                                  _bits(mm[i], rows) & ~_bits(nm[i], rows)), i
    # row permutation permutes the mask bits
    perm = rng.permutation(rows)
    mp, npm, mmp, nmp = _run(ev, Xn[perm], inds)
    assert np.array_equal(mp, m) and np.array_equal(npm, n)
    for i in range(len(inds)):
        assert np.array_equal(_bits(mmp[i], rows), _bits(mm[i], rows)[perm])
        assert np.array_equal(_bits(nmp[i], rows), _bits(nm[i], rows)[perm])
    # consistent column relabelling changes nothing
    cperm = rng.permutation(ncols)          # new column q holds old column cperm[q]
    inv = np.argsort(cperm)
    mq, nq, mmq, nmq = _run(ev, Xn[:, cperm], [inv[np.asarray(ind)] for ind in inds])
    assert np.array_equal(mq, m) and np.array_equal(nq, n) and np.array_equal(mmq, mm)


def pin_invalid(ev):
    X = np.arange(40, dtype=np.float32).reshape(10, 4)
    inds = [[0, 1], [], [0, 4], [-1, 2], [3], [2, 2, 2]]
    m, n, mm, nm = _run(ev, X, inds)
    assert list(m) == [10, -1, -1, -1, 10, 10]
    assert list(n) == [0, -1, -1, -1, 0, 0]
    for i in (1, 2, 3):
        assert not mm[i].any() and not nm[i].any()
    # bits past the last row are zero
    assert int(mm[0][0]) == (1 << 10) - 1


def pin_repeated_columns(ev):
    rng = np.random.default_rng(17)
    rows, ncols = 600, 12
    X = rng.standard_normal((rows, ncols)).astype(np.float32)
    X[rng.random((rows, ncols)) < 0.04] = NAN
    X[:50, 3] = X[:50, 5]  # some ties between different columns too
    base = [rng.permutation(ncols)[: int(rng.integers(1, 9))] for _ in range(30)]
    rep = []
    for ind in base:
        ind = list(ind)
        at = int(rng.integers(0, len(ind)))
        times = int(rng.integers(1, 4))
        rep.append(ind[: at + 1] + [ind[at]] * times + ind[at + 1:])
    lead = [[ind[0]] * int(rng.integers(2, 5)) + list(ind[1:]) for ind in base]
    for include in (False, True):
        want = _run(ev, X, base, include=include, fill=0.25)
        for other in (rep, lead):
            got = _run(ev, X, other, include=include, fill=0.25)
            for a, b in zip(got, want):
                assert np.array_equal(a, b), include
    # a column repeated throughout: every row with the value present, none negative
    m, n, _, _ = _run(ev, X, [[4, 4, 4]])
    assert m[0] == int((~np.isnan(X[:, 4])).sum()) and n[0] == 0


ALL_PINS = [pin_multiset_count, pin_permutation_count, pin_sort_reduction,
            pin_closed_forms, pin_constant_and_sorted_rows, pin_planted,
            pin_invariants, pin_invalid, pin_repeated_columns]
