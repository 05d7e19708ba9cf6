"""C-ABI contract checks that need no GPU: the library loads, exports every
symbol the header declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "messi.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(messi_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2009_00786_amd import messi
    if not os.path.exists(messi.LIB_PATH):
        pytest.skip("libmessi.so not built")
    return messi


def test_header_declares_the_boundary():
    names = _declared_functions()
    for f in ["messi_build", "messi_knn", "messi_free", "messi_last_error"]:
        assert f in names


def test_library_exports_every_declared_symbol(lib):
    raw = ctypes.CDLL(lib.LIB_PATH)
    missing = [f for f in _declared_functions() if not hasattr(raw, f)]
    assert not missing, missing
    assert sorted(lib.EXPORTED) == _declared_functions()


def test_breakpoints_host_only_match_oracle(lib, oracle_mod):
    # two independent methods (AS241 in the library, bisection in the oracle)
    for b in range(1, 9):
        np.testing.assert_array_equal(lib.breakpoints(b), oracle_mod.breakpoints(b))


def test_breakpoints_bad_bits(lib):
    m = lib.load()
    out = np.zeros(255, dtype=np.float32)
    assert m.messi_breakpoints(0, out.ctypes.data) == lib.MESSI_EINVAL
    assert m.messi_breakpoints(9, out.ctypes.data) == lib.MESSI_EINVAL
    assert m.messi_breakpoints(8, None) == lib.MESSI_EINVAL
    code, msg = lib.last_error()
    assert code == lib.MESSI_EINVAL and "null" in msg


def test_server_stats_rejects_null(lib):
    m = lib.load()
    st = lib.ServerStats()
    assert m.messi_server_stats(None, ctypes.byref(st)) == lib.MESSI_EINVAL
    assert m.messi_server_stats(None, None) == lib.MESSI_EINVAL


def test_argument_validation_without_device(lib):
    m = lib.load()
    # null series / bad sizes are rejected before any device call
    assert m.messi_build(None, 10, 256, 16, 8, 2000) is None
    assert lib.last_error()[0] == lib.MESSI_EINVAL
    assert m.messi_build(ctypes.c_void_p(16), 0, 256, 16, 8, 2000) is None
    assert lib.last_error()[0] == lib.MESSI_EINVAL
    assert m.messi_build(ctypes.c_void_p(16), 10, 2048, 16, 8, 2000) is None
    assert lib.last_error()[0] == lib.MESSI_EINVAL
    assert m.messi_knn(None, None, 1, 1, None, None) == lib.MESSI_EINVAL
    assert m.messi_index_info(None, None) == lib.MESSI_EINVAL
    m.messi_free(None)  # NULL-safe


def test_no_device_reports_enodev(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    m = lib.load()
    host = np.zeros((4, 16), dtype=np.float32)
    assert m.messi_build(ctypes.c_void_p(host.ctypes.data), 4, 16, 4, 8, 10) is None
    assert lib.last_error()[0] == lib.MESSI_ENODEV
    assert m.messi_znorm(ctypes.c_void_p(host.ctypes.data), 4, 16, None) == lib.MESSI_ENODEV
