"""Seeded synthetic inputs for the EBIC fitness evaluation.

This module only draws data: expression- or methylation-shaped matrices,
planted monotone (trend) biclusters, missing cells and CSR populations of
ordered column lists. It contains no part of the row-trend predicate, so both
the CPU oracle and the HIP path can take their inputs from it without sharing
any of the method's arithmetic.

Every draw goes through ``numpy.random.default_rng`` (PCG64) seeded with
``SEED_BASE + stream`` (``+ 1000 * sub_stream`` for populations and
request streams). Values are drawn in float64 and rounded to float32 (round
to nearest even).

The five workload shapes stand in for the paper's GEO datasets (Results,
Table 1: 12,483 x 150, 54,675 x 178 and 436,444 x 310), which are not
available here; the population sizes follow the Methods ("Support for Big
Data": converged populations of 1,600 or fewer individuals).
"""
from __future__ import annotations

import dataclasses
from typing import List, Sequence, Tuple

import numpy as np

SEED_BASE = 180709932


def rng_for(stream: int, sub: int = 0) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + int(stream) + 1000 * int(sub))


def draw_values(rng: np.random.Generator, dist: str, shape) -> np.ndarray:
    """float64 draws from ``dist`` rounded to float32."""
    if dist == "uniform":
        v = rng.random(shape)
    elif dist == "normal":
        v = rng.standard_normal(shape)
    elif dist == "beta":
        v = rng.beta(0.5, 0.5, shape)
    else:
        raise ValueError(f"unknown distribution {dist!r}")
    return v.astype(np.float32)


@dataclasses.dataclass
class Plant:
    rows: np.ndarray          # int64 row indices (sorted)
    cols: np.ndarray          # int32 column order of the planted trend
    increasing: bool


@dataclasses.dataclass
class Workload:
    X: np.ndarray             # float32, row-major (rows x cols), C-contiguous
    plants: List[Plant]
    dist: str


def _distinct_sorted_rows(rng, dist, m, k, increasing):
    """m rows of k float32 values, strictly monotone (ties redrawn)."""
    out = np.empty((m, k), dtype=np.float32)
    todo = np.arange(m)
    while todo.size:
        v = np.sort(draw_values(rng, dist, (todo.size, k)), axis=1)
        ok = np.all(np.diff(v, axis=1) > 0, axis=1) if k > 1 else np.ones(todo.size, bool)
        out[todo[ok]] = v[ok]
        todo = todo[~ok]
    if not increasing:
        out = out[:, ::-1]
    return out


def make_matrix(stream: int, rows: int, cols: int, dist: str,
                n_plants: int, plant_rows: Tuple[int, int], plant_cols: Tuple[int, int],
                directions: str = "increasing", nan_fraction: float = 0.0) -> Workload:
    """Matrix + planted trend biclusters (+ missing cells after planting).

    Planted row sets are disjoint, drawn without replacement; each plant's
    columns are a random ordered subset; along that order every planted row
    holds sorted, tie-free draws of the matrix's own distribution.
    ``directions``: "increasing", or "alternate" (even plants increasing,
    odd plants decreasing).
    """
    rng = rng_for(stream)
    X = draw_values(rng, dist, (rows, cols))
    plants: List[Plant] = []
    sizes = [int(rng.integers(plant_rows[0], plant_rows[1] + 1)) for _ in range(n_plants)]
    widths = [int(rng.integers(plant_cols[0], min(plant_cols[1], cols) + 1)) for _ in range(n_plants)]
    if sum(sizes) > rows:
        raise ValueError("planted rows exceed the matrix")
    perm = rng.permutation(rows)
    start = 0
    for p in range(n_plants):
        prow = np.sort(perm[start:start + sizes[p]]).astype(np.int64)
        start += sizes[p]
        pcol = rng.choice(cols, widths[p], replace=False).astype(np.int32)
        inc = True if directions == "increasing" else (p % 2 == 0)
        vals = _distinct_sorted_rows(rng, dist, prow.size, pcol.size, inc)
        X[prow[:, None], pcol[None, :]] = vals
        plants.append(Plant(prow, pcol, inc))
    if nan_fraction > 0:
        n_nan = int(round(nan_fraction * rows * cols))
        flat = rng.choice(rows * cols, n_nan, replace=False)
        X.reshape(-1)[flat] = np.float32(np.nan)
    return Workload(np.ascontiguousarray(X), plants, dist)


def csr(individuals: Sequence[Sequence[int]]) -> Tuple[np.ndarray, np.ndarray]:
    """(offsets int32[n+1], cols int32[nnz]) of a list of column lists."""
    offs = np.zeros(len(individuals) + 1, dtype=np.int64)
    for i, ind in enumerate(individuals):
        offs[i + 1] = offs[i] + len(ind)
    cols = np.zeros(int(offs[-1]), dtype=np.int32)
    for i, ind in enumerate(individuals):
        cols[offs[i]:offs[i + 1]] = np.asarray(ind, dtype=np.int32)
    return offs.astype(np.int32), cols


def make_population(stream: int, sub: int, cols: int, n: int,
                    lengths, plants: Sequence[Plant] = ()) -> List[np.ndarray]:
    """Planted orders first, then random individuals.

    ``lengths`` is (lo, hi) for a uniform integer length, or a callable
    ``f(rng) -> int``. Columns are distinct, ``choice(cols, k)`` in draw order.
    """
    rng = rng_for(stream, sub + 1)
    inds: List[np.ndarray] = [p.cols.copy() for p in plants][:n]
    while len(inds) < n:
        k = int(lengths(rng)) if callable(lengths) else int(rng.integers(lengths[0], lengths[1] + 1))
        k = max(1, min(k, cols))
        inds.append(rng.choice(cols, k, replace=False).astype(np.int32))
    return inds


def skewed_length(rng: np.random.Generator) -> int:
    """2 + min(38, floor(Exp(mean 5))): lengths 2..40 skewed toward short."""
    return 2 + min(38, int(np.floor(rng.exponential(5.0))))


# --------------------------------------------------------------------------
# The five workloads. ``scale`` < 1 shrinks the row count (tests only).
# --------------------------------------------------------------------------

def uniform_1000x50():
    w = make_matrix(1, 1000, 50, "uniform", 3, (50, 50), (8, 8))
    pop = make_population(1, 0, 50, 100, (3, 8), w.plants)
    return w, pop


def normal_missing_20000x200():
    w = make_matrix(2, 20000, 200, "normal", 8, (200, 1000), (5, 15), nan_fraction=0.05)
    pop = make_population(2, 0, 200, 800, (3, 20), w.plants)
    return w, pop


def methylation_436444x64(rows: int = 436444):
    lo, hi = (1000, 20000) if rows >= 436444 else (max(1, rows // 400), max(1, rows // 25))
    w = make_matrix(3, rows, 64, "beta", 10, (lo, hi), (4, 12), directions="alternate")
    pop = make_population(3, 0, 64, 800, (2, 30), w.plants)
    return w, pop


def methylation_wide(rows: int = 436444, cols: int = 310):
    """The methylation workload at the paper's own dataset width (Results,
    Table 1: 436,444 x 310, 541 MB): Beta(0.5,0.5), 10 planted trends,
    800 individuals of 2-30 columns."""
    lo, hi = (1000, 20000) if rows >= 436444 else (max(1, rows // 400), max(1, rows // 25))
    w = make_matrix(30, rows, cols, "beta", 10, (lo, hi), (4, 12), directions="alternate")
    pop = make_population(30, 0, cols, 800, (2, 30), w.plants)
    return w, pop


def batched_100000x256(rows: int = 100000, n_pops: int = 64):
    lo, hi = (500, 5000) if rows >= 100000 else (max(1, rows // 200), max(1, rows // 20))
    w = make_matrix(4, rows, 256, "normal", 8, (lo, hi), (4, 12))
    rng = rng_for(4, 999)
    sizes = [int(rng.integers(100, 1601)) for _ in range(n_pops)]
    pops = [make_population(4, p, 256, sizes[p], skewed_length, w.plants) for p in range(n_pops)]
    return w, pops


SERVED_SHAPES = [(10000, 100, "normal"), (50000, 200, "normal"),
                  (200000, 64, "beta"), (436444, 64, "beta")]


def served_matrices(scale: float = 1.0):
    out = []
    for m, (r, c, dist) in enumerate(SERVED_SHAPES):
        rr = max(64, int(r * scale))
        out.append(make_matrix(50 + m, rr, c, dist, 4,
                               (max(1, rr // 200), max(1, rr // 50)), (4, 12)))
    return out


def population_fast(rng: np.random.Generator, ncols: int, n: int, k_range=(2, 30)):
    """CSR population of n individuals, lengths uniform in k_range, distinct
    columns per individual (vectorised: the first k entries of a random
    permutation per row)."""
    kmax = min(k_range[1], ncols)
    k = rng.integers(k_range[0], kmax + 1, size=n)
    perm = np.argsort(rng.random((n, ncols)), axis=1)[:, :kmax].astype(np.int32)
    offs = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(k, out=offs[1:])
    take = np.arange(kmax)[None, :] < k[:, None]
    return offs.astype(np.int32), perm[take]


@dataclasses.dataclass
class Request:
    t_arrival: float          # seconds from the start of the stream
    run: int                  # EBIC run id (0..n_runs-1)
    matrix: int               # resident matrix index (run mod 4)
    pool_index: int           # population in that matrix's pool


def served_pools(pool_size: int = 32, n_range=(100, 800), k_range=(2, 30)):
    """Per resident matrix, `pool_size` seeded populations (CSR): the
    generations the served runs submit are drawn from these."""
    pools = []
    for m, (_, c, _) in enumerate(SERVED_SHAPES):
        rng = rng_for(5, 100 + m)
        pools.append([population_fast(rng, c, int(rng.integers(n_range[0], n_range[1] + 1)), k_range)
                      for _ in range(pool_size)])
    return pools


def served_requests(duration_s: float, rate_hz: float = 2000.0, n_runs: int = 16,
                     pool_size: int = 32):
    """Poisson arrivals (mean rate_hz) from n_runs concurrent runs; run j
    uses matrix j mod 4 and submits populations from that matrix's pool."""
    rng = rng_for(5, 7)
    n = int(rng.poisson(rate_hz * duration_s * 1.2)) + 16
    gaps = rng.exponential(1.0 / rate_hz, size=n)
    t = np.cumsum(gaps)
    t = t[t < duration_s]
    runs = rng.integers(0, n_runs, size=t.size)
    picks = rng.integers(0, pool_size, size=t.size)
    return [Request(float(t[i]), int(runs[i]), int(runs[i]) % len(SERVED_SHAPES), int(picks[i]))
            for i in range(t.size)]


def nominal_checks(rows: int, offsets: np.ndarray) -> int:
    """rows x sum of individual lengths (the metric's unit of work)."""
    return int(rows) * int(offsets[-1])
