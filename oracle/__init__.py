"""CPU oracle of EBIC's row-counting fitness evaluation (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the benchmark's CPU-baseline leg, never by the product path. The C source
(``ebic_oracle.c``) states the definition it follows and its citations.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ebic_oracle.c")
LIB = os.path.join(HERE, "libebic_oracle.so")

NAN_EXCLUDE = 0
NAN_INCLUDE = 1
NEG_TRENDS = 2

# Plain C, no fast-math: IEEE ordered compares, NaN unordered, denormals kept.
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
          "-ffp-contract=off", "-Wall", "-Wextra"]


def build(src: str = SRC, out: str = LIB, extra=()) -> str:
    """Compile the oracle with gcc; returns the library path."""
    cmd = ["gcc", *CFLAGS, *extra, src, "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


_lib_cache = {}


def load(path: str = LIB):
    """Load (building first if absent) an oracle library."""
    if path in _lib_cache:
        return _lib_cache[path]
    if not os.path.exists(path):
        if path != LIB:
            raise FileNotFoundError(path)
        build()
    lib = ctypes.CDLL(path)
    lib.ebic_oracle_eval.restype = ctypes.c_int
    lib.ebic_oracle_eval.argtypes = [
        ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
        ctypes.c_uint32, ctypes.c_float, ctypes.c_float,
        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
        ctypes.c_int32]
    lib.ebic_oracle_mask_words.restype = ctypes.c_int64
    lib.ebic_oracle_mask_words.argtypes = [ctypes.c_int64]
    _lib_cache[path] = lib
    return lib


def mask_words(rows: int) -> int:
    return (int(rows) + 63) // 64


def eval_population(X, offsets, cols, *, include=False, negative=True,
                    sentinel=float("nan"), fill=0.0, masks=False, threads=1,
                    lib_path: str = LIB):
    """Counts (and optionally masks) for every individual.

    X: float32 (rows x ncols) row-major. offsets/cols: CSR int32.
    Returns (matched, negative, matched_mask, negative_mask); the masks are
    None unless ``masks``.
    """
    lib = load(lib_path)
    X = np.ascontiguousarray(X, dtype=np.float32)
    if X.ndim != 2:
        raise ValueError("X must be 2-D")
    rows, ncols = X.shape
    offsets = np.ascontiguousarray(offsets, dtype=np.int32)
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    n = offsets.size - 1
    matched = np.zeros(n, np.int32)
    neg = np.zeros(n, np.int32)
    w = mask_words(rows)
    mm = np.zeros((n, w), np.uint64) if masks else None
    nm = np.zeros((n, w), np.uint64) if masks else None
    flags = (NAN_INCLUDE if include else 0) | (NEG_TRENDS if negative else 0)
    ptr = lambda a: None if a is None else a.ctypes.data
    cols_p = cols.ctypes.data if cols.size else None
    rc = lib.ebic_oracle_eval(X.ctypes.data, rows, ncols, ncols, offsets.ctypes.data,
                              cols_p, n, flags, float(sentinel), float(fill),
                              matched.ctypes.data, neg.ctypes.data, ptr(mm), ptr(nm),
                              int(threads))
    if rc != 0:
        raise ValueError(f"oracle rejected its arguments (status {rc})")
    return matched, neg, mm, nm
