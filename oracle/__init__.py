"""CPU oracle for BFS and the local SpMSpV product (TEST INFRASTRUCTURE ONLY).

Only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package. The product library never loads it,
and it shares no code with the GPU path; both read the same seeded inputs
from ``graphgen``.

The arithmetic lives in ``oracle.c`` (plain serial C, compiled with gcc);
this module only marshals numpy arrays into it. See the header of
``oracle.c`` for the passages of the paper each function follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc -O2 (no OpenMP: the oracle is serial)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", _SRC, "-o", tmp],
                       check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_bfs.restype = ctypes.c_int
    lib.oracle_bfs.argtypes = [ctypes.c_int64, _i64p, _i32p, ctypes.c_int32, _i32p, _i32p]
    lib.oracle_reached_degree_sum.restype = ctypes.c_int64
    lib.oracle_reached_degree_sum.argtypes = [ctypes.c_int64, _i64p, _i32p]
    lib.oracle_spmspv.restype = ctypes.c_int64
    lib.oracle_spmspv.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, _i32p, _i32p,
                                  _i32p, ctypes.c_int64, _i32p, _i32p, ctypes.c_int64, _i32p,
                                  _i32p]
    lib.oracle_check_bfs.restype = ctypes.c_int
    lib.oracle_check_bfs.argtypes = [ctypes.c_int64, _i64p, _i32p, ctypes.c_int32, _i32p, _i32p,
                                     _i64p]
    _lib = lib
    return lib


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a, t):
    return a.ctypes.data_as(t)


def bfs(n: int, off, col, root: int):
    """(parent, level) int32 arrays of length n from the serial FIFO BFS."""
    lib = _load()
    off = _c(off, np.int64)
    col = _c(col, np.int32)
    if col.size == 0:
        col = np.zeros(1, np.int32)
    parent = np.empty(n, np.int32)
    level = np.empty(n, np.int32)
    rc = lib.oracle_bfs(n, _ptr(off, _i64p), _ptr(col, _i32p), int(root), _ptr(parent, _i32p),
                        _ptr(level, _i32p))
    if rc != 0:
        raise ValueError(f"oracle_bfs failed with {rc}")
    return parent, level


def bfs_graph(g, root: int):
    return bfs(g.n, g.off, g.col, root)


def reached_edges(g, level) -> int:
    """Undirected edges in the searched component: (sum of reached degrees) / 2."""
    lib = _load()
    off = _c(g.off, np.int64)
    level = _c(level, np.int32)
    return int(lib.oracle_reached_degree_sum(g.n, _ptr(off, _i64p), _ptr(level, _i32p))) // 2


def spmspv(nrows: int, ncols: int, jc, cp, ir, fidx, fval=None):
    """Sorted (idx, val) of out[r] = min{val(k) : k in frontier, A(r, k) != 0}."""
    lib = _load()
    jc = _c(jc, np.int32)
    cp = _c(cp, np.int32)
    ir = _c(ir, np.int32)
    fidx = _c(fidx, np.int32)
    nzc = int(jc.shape[0])
    fz = int(fidx.shape[0])
    fv = _c(fval, np.int32) if fval is not None else None
    # capacity: at most one output per row, and at most one per stored nonzero
    cap = max(1, min(nrows, int(ir.shape[0])))
    out_idx = np.empty(cap, np.int32)
    out_val = np.empty(cap, np.int32)
    keep = [jc, cp, ir, fidx]
    if jc.size == 0:
        jc = np.zeros(1, np.int32)
    if ir.size == 0:
        ir = np.zeros(1, np.int32)
    if fidx.size == 0:
        fidx = np.zeros(1, np.int32)
    cnt = lib.oracle_spmspv(nrows, ncols, nzc, _ptr(jc, _i32p), _ptr(cp, _i32p),
                            _ptr(ir, _i32p), fz, _ptr(fidx, _i32p),
                            _ptr(fv, _i32p) if fv is not None else None, cap,
                            _ptr(out_idx, _i32p), _ptr(out_val, _i32p))
    del keep
    if cnt < 0:
        raise ValueError(f"oracle_spmspv failed with {cnt}")
    return out_idx[:cnt].copy(), out_val[:cnt].copy()


def spmspv_block(block, fidx, fval=None):
    return spmspv(block.nrows, block.ncols, block.jc, block.cp, block.ir, fidx, fval)


def check_bfs(g, root: int, parent, level):
    """(code, vertex): code 0 when (parent, level) satisfies the definition."""
    lib = _load()
    off = _c(g.off, np.int64)
    col = _c(g.col, np.int32)
    if col.size == 0:
        col = np.zeros(1, np.int32)
    parent = _c(parent, np.int32)
    level = _c(level, np.int32)
    bad = ctypes.c_int64(-1)
    rc = lib.oracle_check_bfs(g.n, _ptr(off, _i64p), _ptr(col, _i32p), int(root),
                              _ptr(parent, _i32p), _ptr(level, _i32p), ctypes.byref(bad))
    return int(rc), int(bad.value)


def bfs_2d(n: int, R: int, C: int, pr: int, pc: int, shares, root: int):
    """BFS over a p_r x p_c grid of DCSC shares, step by step as Algorithm 3
    (section 3.2) states it, on one host: per level the frontier f (sorted
    global ids, each carrying its own id as the selected value) is split by
    column block (the vector transpose and column gather); every share
    multiplies its column block's piece (the local SpMSpV, with this
    oracle's own SpMSpV); the pieces of a row block are folded with min (the
    row exchange and merge at the owner); vertices without a parent yet take
    the folded value as parent and form the next frontier (pi <- pi + t,
    f <- t, with the mask of unvisited vertices). Returns (parent, level)."""
    parent = np.full(n, -1, np.int64)
    level = np.full(n, -1, np.int64)
    parent[root] = root
    level[root] = 0
    f = np.array([root], np.int64)
    k = 0
    while f.size:
        k += 1
        t = np.full(n, np.iinfo(np.int64).max, np.int64)
        for j in range(pc):
            fj = f[(f >= j * C) & (f < (j + 1) * C)]
            if not fj.size:
                continue
            local = (fj - j * C).astype(np.int32)
            for i in range(pr):
                oi, ov = spmspv_block(shares[i * pc + j], local, fj.astype(np.int32))
                rows = oi.astype(np.int64) + i * R
                np.minimum.at(t, rows, ov.astype(np.int64))
        new = np.nonzero((t != np.iinfo(np.int64).max) & (parent == -1))[0]
        parent[new] = t[new]
        level[new] = k
        f = new
    return parent.astype(np.int32), level.astype(np.int32)


def bfs_by_rows(n: int, off, col, root: int):
    """Level-synchronous BFS in which every level evaluates the masked
    product of section 3.2 by rows of the mask instead of from the frontier:
    each vertex not yet visited scans its own adjacency list in ascending
    order and takes the first vertex of the current frontier it meets as its
    parent. On an undirected graph with ascending rows that vertex is the
    smallest frontier id adjacent to it, the entry the (select, min) product
    gives, so the result must equal bfs(). Plain Python loops: small graphs.
    Returns (parent, level)."""
    off = np.asarray(off, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    parent = np.full(n, -1, np.int64)
    level = np.full(n, -1, np.int64)
    parent[root] = root
    level[root] = 0
    k = 0
    found = True
    while found:
        k += 1
        found = []
        for v in range(n):
            if level[v] != -1:
                continue
            for u in col[off[v]:off[v + 1]]:
                if level[u] == k - 1:
                    parent[v] = u
                    found.append(v)
                    break
        # the level is assigned after all rows are scanned: a vertex found
        # in this level is not yet a frontier vertex for the others
        for v in found:
            level[v] = k
    return parent.astype(np.int32), level.astype(np.int32)
