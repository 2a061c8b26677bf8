"""The C-ABI library loads and exports every symbol include/steiner.h declares
(no GPU needed: nothing here launches a kernel)."""
import ctypes
import os
import re

import pytest

import paper_2205_14503_amd as st

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "steiner.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(steiner_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(st.LIB_PATH):
        pytest.fail("libsteiner.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(st.LIB_PATH)


def test_exports_every_declared_symbol(lib):
    names = header_functions()
    assert len(names) >= 18
    for name in names:
        assert hasattr(lib, name), f"{name} not exported"


def test_binding_covers_header():
    assert sorted(st.EXPORTS) == header_functions()
    for name in st.EXPORTS:
        assert callable(getattr(st, name))


def test_error_strings_without_gpu():
    st.load()
    assert st.steiner_strerror(st.EDISCONNECTED) == "seeds are not connected"
    assert st.steiner_strerror(st.EOVERFLOW) == "distance overflow"


def test_null_arguments_rejected_without_gpu():
    lib = st.load()
    out = ctypes.c_void_p()
    assert lib.steiner_graph_upload(0, 0, None, None, None, 0, None, 0, ctypes.byref(out)) == st.EINVAL
    assert lib.steiner_solve(None, None, 0, None, ctypes.byref(out)) == st.EINVAL
    assert lib.steiner_result_edges(None, None, None, None, None) == st.EINVAL


def test_options_struct_layout():
    assert ctypes.sizeof(st.steiner_options) == 32
    assert ctypes.sizeof(st.steiner_stats) == 24 + 8 * 8 + 12 * 8
