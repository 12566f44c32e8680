"""C ABI checks that need no GPU: the library loads, exports every function
declared in include/bfs.h, and rejects bad arguments before touching the
device."""
import ctypes

import numpy as np
import pytest

from paper_1104_4518_amd import bfs as B


def test_library_exports_every_declared_function():
    lib = B.load()
    names = B.header_functions()
    assert len(names) >= 18
    missing = [n for n in names if not hasattr(lib, n)]
    assert missing == []


def test_version_and_error_strings():
    assert "gfx950" in B.version()
    assert isinstance(B.last_error(), str)


def test_create_csr_argument_errors():
    lib = B.load()
    h = ctypes.c_void_p()
    off = np.array([0, 1, 2], np.int64)
    col = np.array([1, 0], np.int32)
    p_off, p_col = off.ctypes.data, col.ctypes.data
    assert lib.bfs_graph_create_csr(0, 2, p_off, 8, p_col, 0, ctypes.byref(h)) == B.BFS_ERR_ARG
    assert lib.bfs_graph_create_csr(2, -1, p_off, 8, p_col, 0, ctypes.byref(h)) == B.BFS_ERR_ARG
    assert lib.bfs_graph_create_csr(2, 2, p_off, 3, p_col, 0, ctypes.byref(h)) == B.BFS_ERR_ARG
    assert lib.bfs_graph_create_csr(2, 2, None, 8, p_col, 0, ctypes.byref(h)) == B.BFS_ERR_ARG
    assert lib.bfs_graph_create_csr(2, 2, p_off, 8, None, 0, ctypes.byref(h)) == B.BFS_ERR_ARG
    assert lib.bfs_graph_create_csr(2, 2, p_off, 8, p_col, 0, None) == B.BFS_ERR_ARG
    assert lib.bfs_graph_create_csr(1 << 31, 2, p_off, 8, p_col, 0,
                                    ctypes.byref(h)) == B.BFS_ERR_ARG
    assert lib.bfs_graph_create_csr(2, 1 << 31, p_off, 4, p_col, 0,
                                    ctypes.byref(h)) == B.BFS_ERR_ARG
    assert "offset" in B.last_error()


def test_create_dcsc_argument_errors():
    lib = B.load()
    h = ctypes.c_void_p()
    a = np.zeros(4, np.int32)
    p = a.ctypes.data
    assert lib.bfs_graph_create_dcsc(-1, 4, 1, 1, p, p, p, 0, ctypes.byref(h)) == B.BFS_ERR_ARG
    assert lib.bfs_graph_create_dcsc(4, 2, 3, 3, p, p, p, 0,
                                     ctypes.byref(h)) == B.BFS_ERR_FORMAT
    assert lib.bfs_graph_create_dcsc(4, 4, 3, 2, p, p, p, 0,
                                     ctypes.byref(h)) == B.BFS_ERR_FORMAT
    assert lib.bfs_graph_create_dcsc(4, 4, 1, 1, None, p, p, 0,
                                     ctypes.byref(h)) == B.BFS_ERR_ARG


def test_null_handles_rejected():
    lib = B.load()
    assert lib.bfs_graph_destroy(None) == B.BFS_ERR_ARG
    assert lib.bfs_run(None, 0, None, None) == B.BFS_ERR_ARG
    assert lib.bfs_run_async(None, 0, None, None, None) == B.BFS_ERR_ARG
    assert lib.bfs_spmspv(None, None, None, None) == B.BFS_ERR_ARG
    assert lib.bfs_graph_info(None, None, None, None) == B.BFS_ERR_ARG
    assert lib.bfs_last_stats(None, None) == B.BFS_ERR_ARG
    assert lib.bfs_graph_set_options(None, None) == B.BFS_ERR_ARG


def test_binding_errors_are_raised():
    with pytest.raises(B.BfsError) as ei:
        B.Graph.from_csr(0, np.zeros(1, np.int64), np.zeros(0, np.int32))
    assert ei.value.code == B.BFS_ERR_ARG
