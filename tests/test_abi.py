"""The C-ABI library: loads on a machine without a GPU, exports every entry
point declared in include/mhr.h, and rejects bad arguments on the host
before touching the device."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mhr.h")
LIB = os.path.join(ROOT, "paper_2406_07727_amd", "libmhr.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mhr_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libmhr.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for fn in ("mhr_graph_create", "mhr_graph_set_embeddings", "mhr_workspace_size", "mhr_topk_paths",
               "mhr_graph_destroy", "mhr_edge_weights", "mhr_status_string", "mhr_last_error"):
        assert fn in names


def test_library_exports_every_declared_symbol(lib):
    missing = [fn for fn in declared_functions() if not hasattr(lib, fn)]
    assert not missing, missing


def test_host_side_validation(lib):
    lib.mhr_graph_create.restype = ctypes.c_int
    lib.mhr_graph_create.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.mhr_graph_create(None, None, None) == 1  # MHR_ERR_INVALID_ARGUMENT
    lib.mhr_last_error.restype = ctypes.c_char_p
    assert b"null" in lib.mhr_last_error()
    lib.mhr_workspace_size.restype = ctypes.c_int
    lib.mhr_workspace_size.argtypes = [ctypes.c_void_p] * 5
    assert lib.mhr_workspace_size(None, None, None, None, None) == 1
    lib.mhr_topk_paths.restype = ctypes.c_int
    assert lib.mhr_topk_paths(*([None] * 14)) == 1
    lib.mhr_status_string.restype = ctypes.c_char_p
    lib.mhr_status_string.argtypes = [ctypes.c_int]
    assert lib.mhr_status_string(2) == b"workspace too small"


def test_binding_record_layout():
    """The binding's record dtype has the field offsets a C compiler gives
    struct mhr_path (laid out here by ctypes from the header's member list)."""
    import numpy as np
    text = open(HEADER).read()
    body = re.search(r"typedef struct mhr_path \{(.*?)\} mhr_path;", text, flags=re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    ctype = {"uint32_t": ctypes.c_uint32, "uint16_t": ctypes.c_uint16, "float": ctypes.c_float}
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        typ, names = decl.split(None, 1)
        fields += [(nm.strip(), ctype[typ]) for nm in names.split(",")]

    class CPath(ctypes.Structure):
        _fields_ = fields
    import paper_2406_07727_amd as mhr
    dt = np.dtype(mhr.PATH_DTYPE)
    assert ctypes.sizeof(CPath) == dt.itemsize == 24
    assert [f for f, _ in fields] == list(dt.names)
    for name, _ in fields:
        assert getattr(CPath, name).offset == dt.fields[name][1], name
    assert dt["score"] == np.float32 and dt["err_bound"] == np.float32
