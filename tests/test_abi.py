"""The C-ABI library loads and exports every entry point of include/bhpp.h
(CPU only: no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "bhpp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bhpp_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("bhpp_build_graph", "bhpp_query", "bhpp_query_batch", "bhpp_topk"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_2312_06724_amd as bh
    if not os.path.exists(bh.LIB_PATH):
        pytest.skip("libbhpp.so not built")
    lib = ctypes.CDLL(bh.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(bh.EXPORTED) == declared_functions()
    # a call that touches no device: status strings
    lib.bhpp_status_string.restype = ctypes.c_char_p
    assert lib.bhpp_status_string(0) == b"ok"
    assert lib.bhpp_status_string(-3) == b"source node has no edge"


def test_argument_errors_need_no_device():
    """Invalid arguments are rejected before any HIP call."""
    import paper_2312_06724_amd as bh
    if not os.path.exists(bh.LIB_PATH):
        pytest.skip("libbhpp.so not built")
    L = bh.load_library()
    h = ctypes.c_void_p()
    opts = bh.GraphOpts(1.5, -1, 0, 0)   # alpha outside (0,1)
    assert L.bhpp_build_graph(10, 10, 0, None, None, None, ctypes.byref(opts), None, ctypes.byref(h)) == -1
    opts = bh.GraphOpts(0.15, -1, 7, 0)  # unknown dtype
    assert L.bhpp_build_graph(10, 10, 0, None, None, None, ctypes.byref(opts), None, ctypes.byref(h)) == -7
    assert L.bhpp_build_graph(0, 10, 0, None, None, None, None, None, ctypes.byref(h)) == -1
    assert L.bhpp_topk(None, 1, 10, 0, None, 0, None, None, None) == -1       # k < 1
    assert L.bhpp_topk(None, 1, 10, 11, None, 0, None, None, None) == -1      # k > n
    assert L.bhpp_query_batch(None, 1, None, None, 0.15, 1e-6, None, 0, 0, None, None, None, None) == -1
    srv = ctypes.c_void_p()
    assert L.bhpp_server_create(None, None, 64, 0.0, 0.15, 100, 1, ctypes.byref(srv)) == -1   # no graph
    assert L.bhpp_server_submit(None, 0, 1e-6, 0) == -1
    n = ctypes.c_int32(5)
    assert L.bhpp_server_poll(None, 64, None, None, None, None, None, ctypes.byref(n)) == -1
    assert L.bhpp_server_info(None, None) == -1
    L.bhpp_server_destroy(None)                                    # ignored
    mdl = ctypes.c_void_p()
    assert L.bhpp_model_create(None, 0, ctypes.byref(mdl)) == -1
    assert L.bhpp_model_params(None, None, None, None, None) == -1
    assert L.bhpp_model_embed(None) == -1
    assert L.bhpp_model_train(None, 1, None, 1, None, None, 1, 1, 1, 1e-3, 0, None) == -1
    assert L.bhpp_query_batch_warm(None, None, 1, None, None, 0.15, 1e-6, None, 0, 0, None, None, None, None,
                                   None) == -1
    assert L.bhpp_gemm_bf16(0, 1, 1, None, 0, None, 0, None, None) == -1
    L.bhpp_model_free(None)
    assert L.bhpp_set_eps_b_ratio(None, 0.3) == -1
    assert L.bhpp_tune_eps_b(None, 1, None, 1e-6, 0.15, 1, None, None, None, None, None, None) == -1
    assert L.bhpp_query_hpp(None, 1, None, None, 0.15, 1e-6, 0, None, None, None) == -1
