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


def _struct_fields(name):
    """Field names of a typedef'd struct of the header, in order."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct \{([^}]*)\}\s*" + name + r"\s*;", text, flags=re.S).group(1)
    names = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        for part in decl.split(","):
            names.append(re.findall(r"\**(\w+)\s*(?:\[\w+\])?\s*$", part.strip())[0])
    return names


@pytest.mark.parametrize("cname,pyname", [("messi_opts", "Opts"), ("messi_info", "Info"),
                                          ("messi_knn_stats", "KnnStats"), ("messi_leaf", "Leaf"),
                                          ("messi_server_counters", "ServerStats")])
def test_binding_structs_match_the_header(lib, cname, pyname):
    assert [f for f, _ in getattr(lib, pyname)._fields_] == _struct_fields(cname)


def test_knn_ex_takes_k_per_query_and_k_max():
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    sig = re.search(r"int messi_knn_ex\(([^)]*)\)", text, flags=re.S).group(1)
    params = [p.strip() for p in sig.split(",")]
    assert params[3] == "const int32_t* k_per_query" and params[4] == "int32_t k_max"


def test_options_checked_before_any_device_call(lib):
    m = lib.load()
    ptr = ctypes.c_void_p(16)  # never dereferenced: the options are rejected first
    for bad in (dict(mode=7), dict(mode=lib.MODE_BF16), dict(scan_chunk=300), dict(max_slots=-1),
                dict(znorm=2)):
        o = lib.Opts()
        for key, v in bad.items():
            setattr(o, key, v)
        assert m.messi_build_ex(ptr, 10, 256, 16, 8, 2000, ctypes.byref(o)) is None, bad
        code, msg = lib.last_error()
        assert code == lib.MESSI_EINVAL and "opts." in msg, (bad, msg)
