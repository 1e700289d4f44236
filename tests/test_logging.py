"""EBIC_LOG: errors returned by the ABI are reported on stderr at level 1 and
above, and nothing is printed at level 0 (no GPU: the calls fail on their
arguments before touching a device)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1807_09932_amd", "libebic.so")

PROG = r"""
import ctypes, sys
lib = ctypes.CDLL(sys.argv[1])
lib.ebic_create.restype = ctypes.c_int32
lib.ebic_create.argtypes = [ctypes.c_int32, ctypes.c_void_p]
assert lib.ebic_create(0, None) == -1
lib.ebic_server_cancel.restype = ctypes.c_int32
lib.ebic_server_cancel.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
assert lib.ebic_server_cancel(None, 5) == -1
"""


def _run(level):
    if not os.path.exists(LIB):
        pytest.skip("libebic.so not built")
    env = dict(os.environ)
    env.pop("EBIC_LOG", None)
    if level is not None:
        env["EBIC_LOG"] = str(level)
    r = subprocess.run([sys.executable, "-c", PROG, LIB], env=env, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    return r.stderr


def test_errors_logged_at_level_1():
    err = _run(1)
    assert "[ebic] error: out is NULL" in err
    assert "[ebic] error: server is NULL" in err


@pytest.mark.parametrize("level", [None, 0])
def test_silent_by_default(level):
    assert "[ebic]" not in _run(level)
