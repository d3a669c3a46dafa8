"""The C-ABI library loads and exports every entry point its header declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

import paper_2210_07580_amd as G

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gritdbscan.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w \t\*]*?\b([A-Za-z_]\w*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "defined")))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(G.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return G.load_library()


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("gd_create", "gd_destroy", "dbscan", "gd_set_option", "gd_get_stats",
                 "gd_debug_grids", "gd_debug_neighbors", "gd_debug_core", "gd_merge_test",
                 "gd_last_error", "gd_status_string"):
        assert want in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) <= set(G.EXPORTS) | {"gd_status_string"}


def test_null_context_is_rejected(lib):
    assert lib.dbscan(None, None, 0, 2, 1.0, 1, None, None, None) == G.GD_EINVAL
    assert lib.gd_set_option(None, 1, 1) == G.GD_EINVAL
    assert lib.gd_get_stats(None, None) == G.GD_EINVAL
    assert lib.gd_create(None, 0) == G.GD_EINVAL
    lib.gd_destroy(None)
    assert lib.gd_status_string(G.GD_ERANGE) == b"GD_ERANGE"
    assert lib.gd_last_error(None) == b"NULL context"


def test_stats_struct_matches_header():
    # the ctypes mirror of gd_stats must have the header's field count and size
    text = open(HEADER).read()
    body = text[text.index("typedef struct {"):text.index("} gd_stats;")]
    fields = re.findall(r"int(32|64)_t\s+(\w+);", body)
    assert [f for _, f in fields] == [f for f, _ in G.Stats._fields_]
    size = sum(4 if w == "32" else 8 for w, _ in fields)
    assert ctypes.sizeof(G.Stats) == size


def test_no_gpu_means_create_fails_cleanly(lib):
    from conftest import gpu_available
    if gpu_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert lib.gd_create(ctypes.byref(h), 0) == G.GD_EINVAL
