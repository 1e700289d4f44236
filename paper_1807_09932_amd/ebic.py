"""Python binding of libebic.so (include/ebic.h), argument marshalling only.

The ``ebic_*`` functions mirror the C ABI one to one (ctypes). ``Context``
adds tensor handling on top: PyTorch supplies the device memory (its caching
allocator is installed as the library's allocator) and the HIP streams;
every step of the evaluation runs in the library's HIP kernels. There is no
CPU fallback: without the built library (or without a GPU) every call
raises.

torch is imported before the library is loaded so that both use the same
HIP runtime instance.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libebic.so")

EBIC_OK = 0
EBIC_EINVAL = -1
EBIC_ENOMEM = -2
EBIC_EHIP = -3
EBIC_ENOENT = -4
EBIC_EBUSY = -5
EBIC_EBUDGET = -6
EBIC_ECANCELED = -7

EBIC_NAN_EXCLUDE = 0
EBIC_NAN_INCLUDE = 1
EBIC_NEG_TRENDS = 2
EBIC_SRC_DEVICE = 4
EBIC_SRC_COL_MAJOR = 8
EBIC_KEEP_FILL_COPY = 16

STAGE_LDS = 0
STAGE_DIRECT = 1
STAGE_CODES = 2   # FP16 rank codes staged in LDS (matrices of <= 384 columns)
STAGE_BYTES = 3   # byte rank codes, four rows per lane word (<= 128 columns; 4 or 8 tiles per wave)
STAGE_HALVES = 4  # 16-bit rank codes, two rows per lane word (129..384 columns; 2 or 4 tiles per wave)
STAGE_T10 = 5     # 10-bit rank codes, three rows per lane word (129..512 columns; 3 tiles per wave)
STAGE_PAIRS = 6   # pairwise order bitmaps, 32 rows per lane word (<= 1,024 columns; built on first use)

EXPORTED = ["ebic_create", "ebic_destroy", "ebic_set_allocator", "ebic_last_error",
            "ebic_upload_matrix", "ebic_matrix_info", "ebic_matrix_get_stats", "ebic_release_matrix",
            "ebic_mask_words", "ebic_eval_population", "ebic_eval_population_noalloc", "ebic_eval_batch", "ebic_autotune",
            "ebic_set_launch_shape", "ebic_set_profiling", "ebic_read_profile",
            "ebic_plan_shape", "ebic_plan_batch_shape", "ebic_server_request_bytes", "ebic_server_create",
            "ebic_server_destroy", "ebic_server_submit", "ebic_server_poll",
            "ebic_server_get_stats", "ebic_server_cancel", "ebic_server_set_paused", "ebic_ea_create", "ebic_ea_destroy", "ebic_ea_population",
            "ebic_ea_step", "ebic_ea_breed", "ebic_read_delimited", "ebic_free_text_matrix",
            "ebic_write_biclusters"]


class EbicError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"ebic status {status}: {message}")
        self.status = status


class ebic_request(ctypes.Structure):
    _fields_ = [("matrix", ctypes.c_int32), ("n_ind", ctypes.c_int32),
                ("d_offsets", ctypes.c_void_p), ("d_cols", ctypes.c_void_p),
                ("flags", ctypes.c_uint32),
                ("d_matched", ctypes.c_void_p), ("d_negative", ctypes.c_void_p),
                ("d_matched_mask", ctypes.c_void_p), ("d_negative_mask", ctypes.c_void_p)]


class ebic_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("batches", ctypes.c_int64), ("pending", ctypes.c_int64),
                ("reserved_bytes", ctypes.c_int64), ("high_water_bytes", ctypes.c_int64),
                ("budget_bytes", ctypes.c_int64), ("nominal_checks", ctypes.c_int64),
                ("latency_p50_ms", ctypes.c_double), ("latency_p99_ms", ctypes.c_double),
                ("mean_batch", ctypes.c_double), ("latency_max_ms", ctypes.c_double),
                ("graph_captures", ctypes.c_int64), ("staging_grows", ctypes.c_int64),
                ("queue_p99_ms", ctypes.c_double), ("cancelled", ctypes.c_int64)]


class ebic_matrix_stats(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int64), ("cols", ctypes.c_int32), ("code_sets", ctypes.c_uint32),
                ("value_bytes", ctypes.c_int64), ("code_bytes", ctypes.c_int64),
                ("swar_chunks", ctypes.c_int64), ("swar_tie_chunks", ctypes.c_int64),
                ("has_missing", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("upload_ms", ctypes.c_double)]


SET_FILL_COPY, SET_FP16, SET_FP16_FILL, SET_U8, SET_U16, SET_U10 = 1, 2, 4, 8, 16, 32
SET_PAIRS, SET_PAIRS_FILL = 64, 128


class ebic_ea_params(ctypes.Structure):
    _fields_ = [("n_cols", ctypes.c_int32), ("pop_size", ctypes.c_int32),
                ("k_min", ctypes.c_int32), ("k_max", ctypes.c_int32), ("elite", ctypes.c_int32),
                ("p_crossover", ctypes.c_double), ("p_mutation", ctypes.c_double),
                ("seed", ctypes.c_uint64)]


class ebic_text_matrix(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int64), ("cols", ctypes.c_int32), ("delimiter", ctypes.c_char),
                ("values", ctypes.POINTER(ctypes.c_float)),
                ("row_names", ctypes.POINTER(ctypes.c_char_p)),
                ("col_names", ctypes.POINTER(ctypes.c_char_p))]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
RELEASE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libebic.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1807_09932_amd.build`")
    lib = ctypes.CDLL(path)
    P, I32, I64, U32, F = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_float
    sig = {
        "ebic_create": (I32, [I32, ctypes.POINTER(P)]),
        "ebic_destroy": (I32, [P]),
        "ebic_set_allocator": (I32, [P, ALLOC_FN, RELEASE_FN, P]),
        "ebic_last_error": (ctypes.c_char_p, []),
        "ebic_upload_matrix": (I32, [P, P, I64, I32, I64, U32, F, F, P, ctypes.POINTER(I32)]),
        "ebic_matrix_info": (I32, [P, I32, ctypes.POINTER(I64), ctypes.POINTER(I32),
                                   ctypes.POINTER(I64)]),
        "ebic_matrix_get_stats": (I32, [P, I32, ctypes.POINTER(ebic_matrix_stats)]),
        "ebic_release_matrix": (I32, [P, I32]),
        "ebic_mask_words": (I64, [I64]),
        "ebic_eval_population": (I32, [P, I32, I32, P, P, U32, P, P, P, P, P]),
        "ebic_eval_population_noalloc": (I32, [P, I32, I32, P, P, U32, P, P, P, P, P]),
        "ebic_eval_batch": (I32, [P, ctypes.POINTER(ebic_request), I32, P]),
        "ebic_autotune": (I32, [P, ctypes.POINTER(ebic_request), I32, ctypes.c_char_p]),
        "ebic_set_launch_shape": (I32, [P, I32, I32, I32, I32, I32]),
        "ebic_set_profiling": (I32, [P, I32]),
        "ebic_plan_shape": (I32, [P, I32, I32, I64] + [ctypes.POINTER(I32)] * 5),
        "ebic_plan_batch_shape": (I32, [P, ctypes.POINTER(ebic_request), I32]
                                  + [ctypes.POINTER(I32)] * 5),
        "ebic_read_profile": (I32, [P, ctypes.POINTER(I64), ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(I64)]),
        "ebic_server_request_bytes": (I32, [P, I32, I32, I64, U32, I32, ctypes.POINTER(I64)]),
        "ebic_server_create": (I32, [P, I64, I32, I32, ctypes.POINTER(P)]),
        "ebic_server_destroy": (I32, [P]),
        "ebic_server_submit": (I32, [P, I32, I32, P, P, U32, P, P, P, P, ctypes.c_uint64]),
        "ebic_server_poll": (I32, [P, P, P, I32, I32, ctypes.POINTER(I32)]),
        "ebic_server_get_stats": (I32, [P, ctypes.POINTER(ebic_server_stats), I32]),
        "ebic_server_cancel": (I32, [P, ctypes.c_uint64]),
        "ebic_server_set_paused": (I32, [P, I32]),
        "ebic_ea_create": (I32, [ctypes.POINTER(ebic_ea_params), ctypes.POINTER(P)]),
        "ebic_ea_destroy": (I32, [P]),
        "ebic_ea_population": (I32, [P, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(I32),
                                     ctypes.POINTER(I64)]),
        "ebic_ea_step": (I32, [P, P, ctypes.POINTER(I32), ctypes.POINTER(ctypes.c_double)]),
        "ebic_ea_breed": (I32, [P, ctypes.POINTER(ebic_ea_params), ctypes.c_int64, I32, P, P, P, P, P, P, P]),
        "ebic_read_delimited": (I32, [ctypes.c_char_p, ctypes.c_char, I32, I32, I32,
                                      ctypes.POINTER(ebic_text_matrix)]),
        "ebic_free_text_matrix": (I32, [ctypes.POINTER(ebic_text_matrix)]),
        "ebic_write_biclusters": (I32, [ctypes.c_char_p, I64, I32, P, P, P, I32, P,
                                        ctypes.POINTER(ctypes.c_char_p),
                                        ctypes.POINTER(ctypes.c_char_p)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int):
    if status != EBIC_OK:
        raise EbicError(status, ebic_last_error())


# ---------------------------------------------------------------------------
# One-to-one wrappers of the C ABI (raise EbicError on a non-zero status).
# ---------------------------------------------------------------------------

def ebic_last_error() -> str:
    return (load_library().ebic_last_error() or b"").decode()


def ebic_create(hip_device: int) -> int:
    h = ctypes.c_void_p()
    _check(load_library().ebic_create(int(hip_device), ctypes.byref(h)))
    return h.value


def ebic_destroy(ctx: int) -> None:
    _check(load_library().ebic_destroy(ctx))


def ebic_set_allocator(ctx: int, alloc, release, user=None) -> None:
    _check(load_library().ebic_set_allocator(ctx, alloc, release, user))


def ebic_upload_matrix(ctx: int, src: int, rows: int, cols: int, ld_src: int, flags: int,
                       missing_sentinel: float, missing_fill: float, hip_stream: int) -> int:
    out = ctypes.c_int32()
    _check(load_library().ebic_upload_matrix(ctx, src, rows, cols, ld_src, flags,
                                             missing_sentinel, missing_fill, hip_stream,
                                             ctypes.byref(out)))
    return out.value


def ebic_matrix_info(ctx: int, matrix: int) -> Tuple[int, int, int]:
    r, c, b = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64()
    _check(load_library().ebic_matrix_info(ctx, matrix, ctypes.byref(r), ctypes.byref(c),
                                           ctypes.byref(b)))
    return r.value, c.value, b.value


def ebic_matrix_get_stats(ctx: int, matrix: int) -> dict:
    st = ebic_matrix_stats()
    _check(load_library().ebic_matrix_get_stats(ctx, matrix, ctypes.byref(st)))
    return {name: getattr(st, name) for name, _ in st._fields_ if name != "reserved"}


def ebic_release_matrix(ctx: int, matrix: int) -> None:
    _check(load_library().ebic_release_matrix(ctx, matrix))


def ebic_mask_words(rows: int) -> int:
    return int(load_library().ebic_mask_words(rows))


def ebic_eval_population(ctx: int, matrix: int, n_ind: int, d_offsets: int, d_cols: int,
                         flags: int, d_matched: int, d_negative: Optional[int],
                         d_matched_mask: Optional[int], d_negative_mask: Optional[int],
                         hip_stream: int) -> None:
    _check(load_library().ebic_eval_population(ctx, matrix, n_ind, d_offsets, d_cols, flags,
                                               d_matched, d_negative, d_matched_mask,
                                               d_negative_mask, hip_stream))


def ebic_eval_population_noalloc(ctx: int, matrix: int, n_ind: int, d_offsets: int, d_cols: int,
                                 flags: int, d_matched: int, d_negative: Optional[int],
                                 d_matched_mask: Optional[int], d_negative_mask: Optional[int],
                                 hip_stream: int) -> None:
    _check(load_library().ebic_eval_population_noalloc(ctx, matrix, n_ind, d_offsets, d_cols, flags,
                                                       d_matched, d_negative, d_matched_mask,
                                                       d_negative_mask, hip_stream))


def ebic_eval_batch(ctx: int, reqs: Sequence[ebic_request], hip_stream: int) -> None:
    arr = (ebic_request * len(reqs))(*reqs)
    _check(load_library().ebic_eval_batch(ctx, arr, len(reqs), hip_stream))


def ebic_autotune(ctx: int, reqs: Sequence[ebic_request], cache_path: Optional[str]) -> None:
    arr = (ebic_request * len(reqs))(*reqs)
    _check(load_library().ebic_autotune(ctx, arr, len(reqs),
                                        cache_path.encode() if cache_path else None))


def ebic_set_launch_shape(ctx: int, tiles_per_wave: int, waves_per_block: int,
                          individuals_per_group: int, staging: int, blocks: int) -> None:
    _check(load_library().ebic_set_launch_shape(ctx, tiles_per_wave, waves_per_block,
                                                individuals_per_group, staging, blocks))


def ebic_plan_shape(ctx: int, matrix: int, n_ind: int, nnz: int = -1) -> Tuple[int, int, int, int, int]:
    """(tiles_per_wave, waves_per_block, individuals_per_group, staging, blocks)."""
    v = [ctypes.c_int32() for _ in range(5)]
    _check(load_library().ebic_plan_shape(ctx, matrix, n_ind, nnz, *[ctypes.byref(x) for x in v]))
    return tuple(x.value for x in v)


def ebic_plan_batch_shape(ctx: int, reqs: Sequence[ebic_request]) -> Tuple[int, int, int, List[int], int]:
    """(tiles_per_wave, waves_per_block, individuals_per_group, per-request
    stagings, blocks) of the batched launch for `reqs`."""
    arr = (ebic_request * len(reqs))(*reqs)
    v = [ctypes.c_int32() for _ in range(4)]
    st = (ctypes.c_int32 * len(reqs))()
    _check(load_library().ebic_plan_batch_shape(ctx, arr, len(reqs), ctypes.byref(v[0]),
                                                ctypes.byref(v[1]), ctypes.byref(v[2]), st,
                                                ctypes.byref(v[3])))
    return v[0].value, v[1].value, v[2].value, list(st), v[3].value


def ebic_set_profiling(ctx: int, mode: int) -> None:
    _check(load_library().ebic_set_profiling(ctx, mode))


def ebic_read_profile(ctx: int) -> Tuple[int, float, int]:
    """(kernels timed, their summed duration in ms, executed predicate steps)."""
    n, ms, steps = ctypes.c_int64(), ctypes.c_double(), ctypes.c_int64()
    _check(load_library().ebic_read_profile(ctx, ctypes.byref(n), ctypes.byref(ms),
                                            ctypes.byref(steps)))
    return n.value, ms.value, steps.value


def ebic_server_request_bytes(ctx: int, matrix: int, n_ind: int, nnz: int, flags: int,
                              masks: bool) -> int:
    out = ctypes.c_int64()
    _check(load_library().ebic_server_request_bytes(ctx, matrix, n_ind, nnz, flags, int(masks),
                                                    ctypes.byref(out)))
    return out.value


def ebic_server_create(ctx: int, hbm_budget_bytes: int, slots: int, max_batch: int) -> int:
    h = ctypes.c_void_p()
    _check(load_library().ebic_server_create(ctx, int(hbm_budget_bytes), slots, max_batch,
                                             ctypes.byref(h)))
    return h.value


def ebic_server_destroy(srv: int) -> None:
    _check(load_library().ebic_server_destroy(srv))


def ebic_server_submit(srv: int, matrix: int, n_ind: int, offsets: int, cols: Optional[int],
                       flags: int, matched: int, negative: Optional[int],
                       matched_mask: Optional[int], negative_mask: Optional[int], tag: int) -> None:
    """Host pointers; the output buffers must stay alive until `tag` is polled."""
    _check(load_library().ebic_server_submit(srv, matrix, n_ind, offsets, cols, flags, matched,
                                             negative, matched_mask, negative_mask, tag))


def ebic_server_poll(srv: int, tags: np.ndarray, statuses: np.ndarray, timeout_us: int) -> int:
    """Fill tags (uint64) / statuses (int32) with completed requests; returns their number."""
    n = ctypes.c_int32()
    _check(load_library().ebic_server_poll(srv, tags.ctypes.data, statuses.ctypes.data,
                                           min(tags.size, statuses.size), int(timeout_us),
                                           ctypes.byref(n)))
    return n.value


def ebic_server_get_stats(srv: int, reset: bool = False) -> ebic_server_stats:
    st = ebic_server_stats()
    _check(load_library().ebic_server_get_stats(srv, ctypes.byref(st), int(reset)))
    return st


def ebic_server_cancel(srv: int, tag: int) -> None:
    _check(load_library().ebic_server_cancel(srv, tag))


def ebic_server_set_paused(srv: int, paused: bool) -> None:
    _check(load_library().ebic_server_set_paused(srv, 1 if paused else 0))


def ebic_ea_create(params: "ebic_ea_params") -> int:
    h = ctypes.c_void_p()
    _check(load_library().ebic_ea_create(ctypes.byref(params), ctypes.byref(h)))
    return h.value


def ebic_ea_destroy(ea: int) -> None:
    _check(load_library().ebic_ea_destroy(ea))


def ebic_ea_population(ea: int) -> Tuple[int, int, int, int]:
    """(offsets pointer, cols pointer, n_ind, generation) of the driver's host CSR."""
    o, c, n, g = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_int32(), ctypes.c_int64()
    _check(load_library().ebic_ea_population(ea, ctypes.byref(o), ctypes.byref(c),
                                             ctypes.byref(n), ctypes.byref(g)))
    return o.value, c.value, n.value, g.value


def ebic_ea_breed(ctx: int, params: "ebic_ea_params", generation: int, n_ind: int, d_offsets: int,
                  d_cols: int, d_matched: int, d_next_offsets: int, d_next_cols: int,
                  d_best: Optional[int] = None, stream: Optional[int] = None) -> None:
    _check(load_library().ebic_ea_breed(ctx, ctypes.byref(params), generation, n_ind, d_offsets, d_cols,
                                        d_matched, d_next_offsets, d_next_cols, d_best, stream))


def ebic_ea_step(ea: int, matched: int) -> Tuple[int, float]:
    """`matched`: host pointer to pop_size int32 counts; returns (best index, fitness)."""
    bi, bf = ctypes.c_int32(), ctypes.c_double()
    _check(load_library().ebic_ea_step(ea, matched, ctypes.byref(bi), ctypes.byref(bf)))
    return bi.value, bf.value


def ebic_read_delimited(path: str, delimiter: bytes, header: int, row_names: int,
                        threads: int) -> "ebic_text_matrix":
    m = ebic_text_matrix()
    _check(load_library().ebic_read_delimited(os.fsencode(path), delimiter, header, row_names,
                                              threads, ctypes.byref(m)))
    return m


def ebic_free_text_matrix(m: "ebic_text_matrix") -> None:
    _check(load_library().ebic_free_text_matrix(ctypes.byref(m)))


def ebic_write_biclusters(path: str, rows: int, n_ind: int, offsets: int, cols: Optional[int],
                          matched_mask: int, n_out: int, which: Optional[int],
                          row_names, col_names) -> None:
    _check(load_library().ebic_write_biclusters(os.fsencode(path), rows, n_ind, offsets, cols,
                                                matched_mask, n_out, which, row_names, col_names))


def read_delimited(path: str, delimiter: str = "", header: int = -1, row_names: int = -1,
                   threads: int = 8):
    """Parse a delimited text matrix with the library's reader.

    Returns (X, row_names, col_names): X is a float32 (rows x cols) array in
    column-major (Fortran) order, ready for Context.upload; the name lists
    are None when the file has none."""
    d = delimiter.encode()[:1] if delimiter else b"\0"
    m = ebic_read_delimited(path, d, header, row_names, max(1, threads))
    try:
        n = m.rows * m.cols
        flat = np.ctypeslib.as_array(m.values, shape=(n,)).copy() if n else np.zeros(0, np.float32)
        X = flat.reshape(m.cols, m.rows).T  # column-major view of (rows, cols)
        # (names are bytes as written in the file; bytes that are not UTF-8
        # are kept as escapes, so writing the names back gives the same bytes)
        rn = ([m.row_names[i].decode("utf-8", "surrogateescape") for i in range(m.rows)]
              if m.row_names else None)
        cn = ([m.col_names[i].decode("utf-8", "surrogateescape") for i in range(m.cols)]
              if m.col_names else None)
    finally:
        ebic_free_text_matrix(m)
    return X, rn, cn


def write_biclusters(path: str, rows: int, offsets: np.ndarray, cols: np.ndarray,
                     matched_mask: np.ndarray, which: Sequence[int],
                     row_names: Optional[Sequence[str]] = None,
                     col_names: Optional[Sequence[str]] = None) -> None:
    """Write the biclusters of individuals `which` (text, see include/ebic.h)."""
    offsets = np.ascontiguousarray(offsets, dtype=np.int32)
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    mask = np.ascontiguousarray(matched_mask).view(np.uint64)
    n = offsets.size - 1
    if mask.size != n * ebic_mask_words(rows):
        raise ValueError("matched_mask must hold n x ebic_mask_words(rows) words")
    w = np.ascontiguousarray(which, dtype=np.int32)

    def names(v):
        if v is None:
            return None
        arr = (ctypes.c_char_p * len(v))(*[str(x).encode("utf-8", "surrogateescape") for x in v])
        return ctypes.cast(arr, ctypes.POINTER(ctypes.c_char_p)), arr
    rn, cn = names(row_names), names(col_names)
    ebic_write_biclusters(path, rows, n, offsets.ctypes.data, cols.ctypes.data if cols.size else None,
                          mask.ctypes.data, w.size, w.ctypes.data if w.size else None,
                          rn[0] if rn else None, cn[0] if cn else None)


class EA:
    """The library's stand-in evolutionary driver (host code, include/ebic.h):
    ``population()`` gives the current generation as CSR, ``step(matched)``
    scores it from its matched counts and breeds the next one."""

    def __init__(self, n_cols: int, pop_size: int, k_min: int = 2, k_max: int = 30,
                 elite: int = -1, p_crossover: float = 0.5, p_mutation: float = 0.9,
                 seed: int = 0):
        if elite < 0:
            elite = max(1, pop_size // 20)
        self.params = ebic_ea_params(n_cols, pop_size, k_min, min(k_max, n_cols), elite,
                                     p_crossover, p_mutation, seed & (2**64 - 1))
        self.handle = ebic_ea_create(self.params)

    def population(self) -> Tuple[np.ndarray, np.ndarray, int]:
        """(offsets, cols, generation): copies of the current generation's CSR."""
        o, c, n, g = ebic_ea_population(self.handle)
        offs = np.ctypeslib.as_array(ctypes.cast(o, ctypes.POINTER(ctypes.c_int32)),
                                     shape=(n + 1,)).copy()
        nnz = int(offs[-1])
        cols = (np.ctypeslib.as_array(ctypes.cast(c, ctypes.POINTER(ctypes.c_int32)),
                                      shape=(nnz,)).copy() if nnz else np.zeros(0, np.int32))
        return offs, cols, g

    def step(self, matched: np.ndarray) -> Tuple[int, float]:
        """Score the current generation; returns (best index, best fitness)."""
        m = np.ascontiguousarray(matched, dtype=np.int32)
        if m.size != self.params.pop_size:
            raise ValueError("one matched count per individual is required")
        return ebic_ea_step(self.handle, m.ctypes.data)

    def close(self):
        if self.handle:
            ebic_ea_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Tensor-level API
# ---------------------------------------------------------------------------

def pack(individuals: Sequence[Sequence[int]]) -> Tuple[np.ndarray, np.ndarray]:
    """CSR of a list of column lists: (offsets int32[n+1], cols int32[nnz])."""
    lens = np.fromiter((len(x) for x in individuals), dtype=np.int64, count=len(individuals))
    offs = np.zeros(len(individuals) + 1, dtype=np.int64)
    np.cumsum(lens, out=offs[1:])
    if offs[-1] > np.iinfo(np.int32).max:
        raise ValueError("population too large for int32 offsets")
    cols = (np.concatenate([np.asarray(x, dtype=np.int32) for x in individuals])
            if len(individuals) and offs[-1] else np.zeros(0, np.int32))
    return offs.astype(np.int32), cols.astype(np.int32)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


class Population:
    """A CSR population resident on the device (int32 offsets and columns)."""

    def __init__(self, offsets: torch.Tensor, cols: torch.Tensor):
        self.offsets = offsets
        self.cols = cols
        self.n = offsets.numel() - 1
        self.nnz = cols.numel()


class Context:
    """One library context on one HIP device, with torch as the allocator."""

    def __init__(self, device: int = 0, torch_allocator: bool = True):
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: the EBIC library runs only on the GPU")
        load_library()
        self.device = torch.device("cuda", device)
        self.handle = ebic_create(device)
        self._blocks = {}
        self._alloc_cb = self._release_cb = None
        if torch_allocator:
            def _alloc(nbytes, _user):
                try:
                    t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
                except Exception:
                    return None
                self._blocks[t.data_ptr()] = t
                return t.data_ptr()

            def _release(ptr, _user):
                self._blocks.pop(ptr, None)

            self._alloc_cb = ALLOC_FN(_alloc)
            self._release_cb = RELEASE_FN(_release)
            ebic_set_allocator(self.handle, self._alloc_cb, self._release_cb)
        self.matrices = {}

    def close(self):
        if self.handle:
            ebic_destroy(self.handle)
            self.handle = None
            self._blocks.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stream_handle(self, stream: Optional[torch.cuda.Stream] = None) -> int:
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        return s.cuda_stream

    # -- matrices -----------------------------------------------------------
    def upload(self, X, sentinel: Optional[float] = None, fill: float = 0.0,
               keep_fill_copy: bool = False, stream=None) -> int:
        """Make a (rows x cols) float32 matrix resident; returns its handle.

        X: numpy array or torch tensor (host or this device), row-major or
        column-major (a transposed view of a row-major array).
        """
        if isinstance(X, np.ndarray):
            X = torch.from_numpy(np.asarray(X))
        if X.dtype != torch.float32 or X.dim() != 2:
            raise ValueError("X must be a 2-D float32 array")
        rows, cols = X.shape
        flags = EBIC_KEEP_FILL_COPY if keep_fill_copy else 0
        if X.is_cuda:
            if X.device != self.device:
                raise ValueError("X is on another device")
            flags |= EBIC_SRC_DEVICE
        if X.stride(1) == 1 and X.stride(0) >= cols:
            ld = X.stride(0)
        elif X.stride(0) == 1 and X.stride(1) >= rows:
            flags |= EBIC_SRC_COL_MAJOR
            ld = X.stride(1)
        else:
            X = X.contiguous()
            ld = cols
        sent = float("nan") if sentinel is None else float(sentinel)
        h = ebic_upload_matrix(self.handle, X.data_ptr(), rows, cols, ld, flags, sent, float(fill),
                               self.stream_handle(stream))
        self.matrices[h] = (rows, cols)
        return h

    def release(self, matrix: int) -> None:
        ebic_release_matrix(self.handle, matrix)
        self.matrices.pop(matrix, None)

    def info(self, matrix: int):
        return ebic_matrix_info(self.handle, matrix)

    def stats(self, matrix: int) -> dict:
        return ebic_matrix_get_stats(self.handle, matrix)

    # -- populations --------------------------------------------------------
    def population(self, individuals=None, offsets=None, cols=None) -> Population:
        """Device CSR from a list of column lists or from (offsets, cols).

        Host inputs are checked here (non-decreasing offsets starting at 0 and
        a column array long enough) before they are copied to the device.
        """
        if individuals is not None:
            offsets, cols = pack(individuals)
        if isinstance(offsets, np.ndarray):
            offsets = torch.from_numpy(np.ascontiguousarray(offsets, dtype=np.int32))
        if isinstance(cols, np.ndarray):
            cols = torch.from_numpy(np.ascontiguousarray(cols, dtype=np.int32))
        if offsets.dtype != torch.int32 or cols.dtype != torch.int32:
            raise ValueError("offsets and cols must be int32")
        if offsets.dim() != 1 or offsets.numel() < 1:
            raise ValueError("offsets must be 1-D with n + 1 entries")
        # Every offset must lie in [0, len(cols)]: the kernels read
        # cols[offsets[i] .. offsets[i+1]) of each individual whose offsets
        # increase. Decreasing offsets are allowed and mark an invalid
        # individual (-1), as the C ABI specifies.
        o = offsets if not offsets.is_cuda else offsets.cpu()
        if int(o.min()) < 0 or int(o.max()) > cols.numel():
            raise ValueError("offsets reach outside the column array")
        offsets = offsets.to(self.device, non_blocking=False).contiguous()
        cols = cols.to(self.device, non_blocking=False).contiguous()
        if cols.numel() == 0:
            cols = torch.zeros(1, dtype=torch.int32, device=self.device)
        return Population(offsets, cols)

    def breed(self, params: "ebic_ea_params", generation: int, pop: Population, matched: torch.Tensor,
              stream=None, out=None):
        """The next generation bred on the device (ebic_ea_breed) from `pop`
        and its matched counts: returns (Population, best) where best is a
        one-element device tensor holding the current generation's best
        index. `out` = (offsets, cols, best) tensors to reuse (n + 1,
        n * k_max, 1). Asynchronous on the stream."""
        n = pop.n
        if out is None:
            out = (torch.empty(n + 1, dtype=torch.int32, device=self.device),
                   torch.empty(max(1, n * params.k_max), dtype=torch.int32, device=self.device),
                   torch.empty(1, dtype=torch.int32, device=self.device))
        o, c, b = out
        ebic_ea_breed(self.handle, params, generation, n, pop.offsets.data_ptr(), pop.cols.data_ptr(),
                      matched.data_ptr(), o.data_ptr(), c.data_ptr(), b.data_ptr(), self.stream_handle(stream))
        return Population(o, c), b

    def outputs(self, matrix: int, n: int, masks: bool = False, negative: bool = True):
        rows, _ = self.matrices[matrix]
        words = ebic_mask_words(rows)
        m = torch.empty(n, dtype=torch.int32, device=self.device)
        g = torch.empty(n, dtype=torch.int32, device=self.device) if negative else None
        mm = torch.empty((n, words), dtype=torch.int64, device=self.device) if masks else None
        nm = torch.empty((n, words), dtype=torch.int64, device=self.device) if masks else None
        return m, g, mm, nm

    @staticmethod
    def flags(include: bool = False, negative: bool = True) -> int:
        return (EBIC_NAN_INCLUDE if include else EBIC_NAN_EXCLUDE) | (EBIC_NEG_TRENDS if negative else 0)

    def eval(self, matrix: int, pop: Population, include: bool = False, negative: bool = True,
             masks: bool = False, out=None, stream=None):
        """Evaluate a population; returns (matched, negative, matched_mask,
        negative_mask) device tensors (masks are int64 views of uint64 words;
        None when not requested). Asynchronous on the stream."""
        if out is None:
            out = self.outputs(matrix, pop.n, masks)
        m, g, mm, nm = out
        ebic_eval_population(self.handle, matrix, pop.n, pop.offsets.data_ptr(),
                             pop.cols.data_ptr(), self.flags(include, negative), m.data_ptr(),
                             _ptr(g), _ptr(mm), _ptr(nm), self.stream_handle(stream))
        return m, g, mm, nm

    def request(self, matrix: int, pop: Population, out, include=False, negative=True) -> ebic_request:
        m, g, mm, nm = out
        return ebic_request(matrix, pop.n, pop.offsets.data_ptr(), pop.cols.data_ptr(),
                            self.flags(include, negative), m.data_ptr(), _ptr(g), _ptr(mm), _ptr(nm))

    def eval_batch(self, reqs: Sequence[ebic_request], stream=None) -> None:
        ebic_eval_batch(self.handle, reqs, self.stream_handle(stream))

    def autotune(self, reqs: Sequence[ebic_request], cache_path: Optional[str] = None) -> None:
        ebic_autotune(self.handle, reqs, cache_path)

    def set_launch_shape(self, tiles_per_wave=0, waves_per_block=0, individuals_per_group=1,
                         staging=STAGE_LDS, blocks=0) -> None:
        ebic_set_launch_shape(self.handle, tiles_per_wave, waves_per_block, individuals_per_group,
                              staging, blocks)
