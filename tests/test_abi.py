"""The C-ABI library loads and exports every entry point of include/ebic.h
(no GPU needed; nothing here launches a kernel)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ebic.h")
LIB = os.path.join(ROOT, "paper_1807_09932_amd", "libebic.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:ebic_status|int64_t|const char \*)\s*(ebic_\w+)\s*\(",
                                 src, flags=re.M)))


def _lib():
    if not os.path.exists(LIB):
        pytest.skip("libebic.so not built")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["ebic_create", "ebic_destroy", "ebic_upload_matrix", "ebic_eval_population",
              "ebic_eval_batch", "ebic_autotune", "ebic_release_matrix", "ebic_mask_words"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = _lib()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_mirrors_the_header():
    from paper_1807_09932_amd import ebic
    assert sorted(ebic.EXPORTED) == declared_functions()
    for name in declared_functions():
        assert callable(getattr(ebic, name))


def test_mask_words_host_arithmetic():
    lib = _lib()
    lib.ebic_mask_words.restype = ctypes.c_int64
    lib.ebic_mask_words.argtypes = [ctypes.c_int64]
    assert [lib.ebic_mask_words(r) for r in (0, 1, 63, 64, 65, 436444, 2**31 - 1)] == \
        [0, 1, 1, 1, 2, 6820, 33554432]


def test_host_errors_without_device():
    """Null pointers are rejected before any device work."""
    lib = _lib()
    lib.ebic_create.restype = ctypes.c_int32
    lib.ebic_create.argtypes = [ctypes.c_int32, ctypes.c_void_p]
    lib.ebic_last_error.restype = ctypes.c_char_p
    assert lib.ebic_create(0, None) == -1
    assert b"NULL" in lib.ebic_last_error()
    lib.ebic_eval_population.restype = ctypes.c_int32
    lib.ebic_eval_population.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32] + \
        [ctypes.c_void_p] * 2 + [ctypes.c_uint32] + [ctypes.c_void_p] * 5
    assert lib.ebic_eval_population(None, 0, 1, None, None, 0, None, None, None, None, None) == -1
