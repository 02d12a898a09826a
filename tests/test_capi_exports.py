"""The C ABI library loads on the CPU and exports every symbol include/ahpp.h declares.

No compute call is made here (no GPU): only symbol lookup and argument
checks that return before any device work.
"""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "ahpp.h")).read()
    return sorted(set(re.findall(r"\b(ahpp_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2512_11606_amd import ahpp
    if not os.path.exists(ahpp.LIB_PATH):
        from paper_2512_11606_amd import build
        build.build()
    return ahpp.load_library()


def test_every_declared_symbol_is_exported(lib):
    from paper_2512_11606_amd import ahpp
    names = declared_functions()
    assert set(names) == set(ahpp.EXPORTED)
    bound_by_methods = {"ahpp_graph_free": ahpp.Graph.free, "ahpp_last_error": ahpp._check,
                        "ahpp_server_create": ahpp.Server.__init__, "ahpp_server_free": ahpp.Server.close,
                        "ahpp_server_submit": ahpp.Server.submit, "ahpp_server_step": ahpp.Server.step,
                        "ahpp_server_results": ahpp.Server.results, "ahpp_server_info": ahpp.Server.info,
                        "ahpp_server_set_solo": ahpp.Server.set_solo}
    for n in names:
        assert hasattr(lib, n), n
        assert getattr(ahpp, n, None) is not None or n in bound_by_methods, n


def test_argument_errors_need_no_device(lib):
    from paper_2512_11606_amd import ahpp
    h = ctypes.c_void_p()
    assert lib.ahpp_graph_load(None, ctypes.byref(h)) == ahpp.ERR_INVALID_ARG
    assert b"NULL" in lib.ahpp_last_error()
    d = ahpp.GraphDesc(10, 5, 2, 0, None, None, None, 0, None, None, None, 1.5, 0.35, 0.0, 0, 0)
    assert lib.ahpp_graph_load(ctypes.byref(d), ctypes.byref(h)) == ahpp.ERR_INVALID_ARG
    assert b"alpha" in lib.ahpp_last_error()
    d = ahpp.GraphDesc(10, 5, 2, 0, None, None, None, 0, None, None, None, 0.15, 1.5, 0.0, 0, 0)
    assert lib.ahpp_graph_load(ctypes.byref(d), ctypes.byref(h)) == ahpp.ERR_INVALID_ARG
    d = ahpp.GraphDesc(0, 5, 2, 0, None, None, None, 0, None, None, None, 0.15, 0.35, 0.0, 0, 0)
    assert lib.ahpp_graph_load(ctypes.byref(d), ctypes.byref(h)) == ahpp.ERR_INVALID_ARG
    assert lib.ahpp_query(None, 0, 1e-6, 0, None, None, 0, None, None, None, None, None) == ahpp.ERR_INVALID_ARG
    assert lib.ahpp_topk(None, None, 5, -1, None, None, None, None) == ahpp.ERR_INVALID_ARG
    assert lib.ahpp_graph_tune(None, 0, None, None) == ahpp.ERR_INVALID_ARG
    assert lib.ahpp_query_schedule(None, 0, 1e-6, 1, 0, None, None, 0, None, None, None, None,
                                   None) == ahpp.ERR_INVALID_ARG
    assert lib.ahpp_query_mc(None, 0, 10, 1, None, 0, None, None, None, None, None) == ahpp.ERR_INVALID_ARG
    lib.ahpp_graph_free(None)


def test_header_documents_each_entry_point():
    text = open(os.path.join(ROOT, "include", "ahpp.h")).read()
    for n in ("ahpp_graph_load", "ahpp_query", "ahpp_query_batch", "ahpp_topk"):
        i = text.index(n + "(")
        block = text[max(0, i - 1500): i]
        assert "/*" in block, n


def test_binding_refuses_ids_that_would_wrap():
    """Ids given in a wider integer type must fit int32: a wrapped id could be
    a valid node.  Checked before any call into the library."""
    import numpy as np
    from paper_2512_11606_amd import ahpp
    big = np.array([0, 2 ** 32 + 1], np.int64)
    ok = np.array([0, 1], np.int64)
    with pytest.raises(ValueError, match="int32 range"):
        ahpp.ahpp_graph_load(2, 2, 1, big, ok, None, ok, np.zeros(2, np.int64), None)
    with pytest.raises(ValueError, match="integers"):
        ahpp.ahpp_graph_load(2, 2, 1, ok.astype(np.float64), ok, None, ok, np.zeros(2, np.int64), None)
    assert ahpp._as_i32([3, 4], "x").dtype == np.int32
    assert ahpp._as_i32(np.arange(3, dtype=np.int32), "x").flags["C_CONTIGUOUS"]
