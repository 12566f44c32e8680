"""Seeded synthetic inputs shared by the CPU oracle and the GPU library.

This package only builds inputs (graphs in CSR, hypersparse DCSC blocks,
sorted frontier samples, roots). It holds none of the traversal or
sparse-product arithmetic. All randomness is counter based (SplitMix64), so
a (generator, parameters, seed) triple always yields the same bytes.

R-MAT follows Chakrabarti et al. with the parameters of the paper's
experimental section (a, b, c, d; edge factor 16), then a seeded random
relabelling of vertex ids (the paper's load-balancing relabel, section
"Load-balancing traversal"), symmetrisation, self-loop and duplicate
removal, and ascending adjacency lists (section "Graph Representation").
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.cpp")
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None

# Graph 500 R-MAT parameters as bound for this build (a + b + c + d = 1).
RMAT_A, RMAT_B, RMAT_C = 0.57, 0.19, 0.19

_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_u64p = ctypes.POINTER(ctypes.c_uint64)


def build(force: bool = True) -> str:
    """Compile libgraphgen.so with g++ (OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["g++", "-O3", "-std=c++17", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    lib.gg_mix64.restype = ctypes.c_uint64
    lib.gg_mix64.argtypes = [ctypes.c_uint64]
    lib.gg_draw.restype = ctypes.c_uint64
    lib.gg_draw.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    lib.gg_stream_key.restype = ctypes.c_uint64
    lib.gg_stream_key.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    lib.gg_perm.restype = ctypes.c_uint64
    lib.gg_perm.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64]
    spec = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint32,
            ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int]
    lib.gg_edge_list.restype = None
    lib.gg_edge_list.argtypes = spec + [_i64p, _i64p]
    lib.gg_edges_count.restype = ctypes.c_int64
    lib.gg_edges_count.argtypes = spec + [_i64p]
    lib.gg_edges_fill.restype = ctypes.c_int64
    lib.gg_edges_fill.argtypes = spec + [_i64p, _i32p, _i64p]
    lib.gg_compact.restype = None
    lib.gg_compact.argtypes = [ctypes.c_int64, _i64p, _i32p, _i64p, _i64p, _i32p]
    lib.gg_grid_count.restype = ctypes.c_int64
    lib.gg_grid_count.argtypes = [ctypes.c_int64, ctypes.c_int64]
    lib.gg_grid.restype = None
    lib.gg_grid.argtypes = [ctypes.c_int64, ctypes.c_int64, _i64p, _i32p]
    lib.gg_block_keys.restype = ctypes.c_int64
    lib.gg_block_keys.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, _u64p]
    lib.gg_dcsc_from_keys.restype = ctypes.c_int64
    lib.gg_dcsc_from_keys.argtypes = [_u64p, ctypes.c_int64, _i32p, _i32p, _i32p]
    lib.gg_sample.restype = None
    lib.gg_sample.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, _i32p]
    lib.gg_roots.restype = ctypes.c_int64
    lib.gg_roots.argtypes = [ctypes.c_int64, _i64p, ctypes.c_int64, ctypes.c_uint64, _i32p]
    lib.gg_hash_bytes.restype = ctypes.c_uint64
    lib.gg_hash_bytes.argtypes = [ctypes.c_void_p, ctypes.c_int64]
    _lib = lib
    return lib


def _p(a: np.ndarray, t):
    return a.ctypes.data_as(t)


@dataclass
class CSR:
    """Symmetric graph in CSR: row offsets (int64, n + 1) and column ids (int32)."""

    n: int
    off: np.ndarray
    col: np.ndarray
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def degrees(self) -> np.ndarray:
        return np.diff(self.off)

    def hash(self) -> int:
        return csr_hash(self.off, self.col)


@dataclass
class DCSCBlock:
    """Hypersparse block in DCSC: jc (non-empty column ids), cp (nzc + 1), ir (row ids)."""

    nrows: int
    ncols: int
    jc: np.ndarray
    cp: np.ndarray
    ir: np.ndarray

    @property
    def nzc(self) -> int:
        return int(self.jc.shape[0])

    @property
    def nnz(self) -> int:
        return int(self.ir.shape[0])


def thresholds(a: float, b: float, c: float):
    """Cumulative quadrant thresholds as 32-bit integers: floor(p * 2^32)."""
    two32 = float(1 << 32)
    ta = min(int(a * two32), (1 << 32) - 1)
    tab = min(int((a + b) * two32), (1 << 32) - 1)
    tabc = min(int((a + b + c) * two32), (1 << 32) - 1)
    return ta, tab, tabc


def _edges_csr(kind: int, scale: int, m: int, a: float, b: float, c: float, seed: int,
               permute: bool) -> CSR:
    lib = _load()
    n = 1 << scale
    ta, tab, tabc = thresholds(a, b, c)
    spec = (kind, scale, m, ta, tab, tabc, seed, int(permute))
    off_raw = np.empty(n + 1, dtype=np.int64)
    raw = lib.gg_edges_count(*spec, _p(off_raw, _i64p))
    col_raw = np.empty(max(raw, 1), dtype=np.int32)
    deg = np.empty(n, dtype=np.int64)
    total = lib.gg_edges_fill(*spec, _p(off_raw, _i64p), _p(col_raw, _i32p), _p(deg, _i64p))
    off = np.empty(n + 1, dtype=np.int64)
    col = np.empty(total, dtype=np.int32)
    lib.gg_compact(n, _p(off_raw, _i64p), _p(col_raw, _i32p), _p(deg, _i64p), _p(off, _i64p),
                   _p(col, _i32p))
    del col_raw, off_raw, deg
    return CSR(n, off, col)


def rmat_csr(scale: int, edgefactor: int = 16, seed: int = 1, a: float = RMAT_A,
             b: float = RMAT_B, c: float = RMAT_C, permute: bool = True) -> CSR:
    """R-MAT graph with n = 2^scale, edgefactor * n generated edges, symmetrised."""
    g = _edges_csr(0, scale, edgefactor << scale, a, b, c, seed, permute)
    g.name = f"rmat{scale}"
    return g


def er_csr(scale: int, edgefactor: int = 16, seed: int = 1) -> CSR:
    """Erdos-Renyi-style graph: same n and m as R-MAT, uniform endpoints."""
    g = _edges_csr(1, scale, edgefactor << scale, 0.25, 0.25, 0.25, seed, False)
    g.name = f"er{scale}"
    return g


def edge_list(kind: int, scale: int, m: int, seed: int, a: float = RMAT_A, b: float = RMAT_B,
              c: float = RMAT_C, permute: bool = True):
    """Raw generated (u, v) endpoint arrays before symmetrisation (for tests)."""
    lib = _load()
    ta, tab, tabc = thresholds(a, b, c)
    us = np.empty(m, dtype=np.int64)
    vs = np.empty(m, dtype=np.int64)
    lib.gg_edge_list(kind, scale, m, ta, tab, tabc, seed, int(permute), _p(us, _i64p),
                     _p(vs, _i64p))
    return us, vs


def grid_csr(w: int, h: int | None = None) -> CSR:
    """W x H 4-neighbour lattice, row-major ids (not relabelled)."""
    h = w if h is None else h
    lib = _load()
    n = w * h
    off = np.empty(n + 1, dtype=np.int64)
    col = np.empty(max(lib.gg_grid_count(w, h), 0), dtype=np.int32)
    lib.gg_grid(w, h, _p(off, _i64p), _p(col, _i32p))
    return CSR(n, off, col, name=f"grid{w}x{h}")


def from_edges(n: int, edges) -> CSR:
    """Symmetric CSR from an explicit edge list (self-loops dropped, deduplicated)."""
    e = np.asarray(list(edges), dtype=np.int64).reshape(-1, 2)
    if e.size:
        e = e[e[:, 0] != e[:, 1]]
        both = np.concatenate([e, e[:, ::-1]], axis=0)
        both = np.unique(both, axis=0)
    else:
        both = np.zeros((0, 2), dtype=np.int64)
    counts = np.bincount(both[:, 0], minlength=n) if both.size else np.zeros(n, np.int64)
    off = np.zeros(n + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    col = both[:, 1].astype(np.int32) if both.size else np.zeros(0, np.int32)
    return CSR(n, off, col)


def dcsc_block(log_n: int, nnz: int, seed: int) -> DCSCBlock:
    """2^log_n x 2^log_n block with nnz uniform (row, col) draws, deduplicated."""
    lib = _load()
    keys = np.empty(max(nnz, 1), dtype=np.uint64)
    cnt = lib.gg_block_keys(log_n, nnz, seed, _p(keys, _u64p))
    jc = np.empty(cnt + 1, dtype=np.int32)
    cp = np.empty(cnt + 1, dtype=np.int32)
    ir = np.empty(max(cnt, 1), dtype=np.int32)
    nzc = lib.gg_dcsc_from_keys(_p(keys, _u64p), cnt, _p(jc, _i32p), _p(cp, _i32p),
                                _p(ir, _i32p))
    del keys
    return DCSCBlock(1 << log_n, 1 << log_n, jc[:nzc].copy(), cp[:nzc + 1].copy(),
                     ir[:cnt].copy())


def dcsc_from_dense(a: np.ndarray) -> DCSCBlock:
    """DCSC arrays of a small dense boolean matrix (rows x cols)."""
    a = np.asarray(a, dtype=bool)
    nrows, ncols = a.shape
    jc, cp, ir = [], [0], []
    for k in range(ncols):
        rows = np.nonzero(a[:, k])[0]
        if rows.size:
            jc.append(k)
            ir.extend(rows.tolist())
            cp.append(len(ir))
    return DCSCBlock(nrows, ncols, np.array(jc, np.int32), np.array(cp, np.int32),
                     np.array(ir, np.int32))


def frontier_sample(log_n: int, k: int, seed: int) -> np.ndarray:
    """k distinct sorted indices of [0, 2^log_n)."""
    lib = _load()
    out = np.empty(max(k, 1), dtype=np.int32)
    if k:
        lib.gg_sample(log_n, k, seed, _p(out, _i32p))
    return out[:k].copy()


def roots(g: CSR, count: int, seed: int) -> np.ndarray:
    """Distinct seeded roots with degree >= 1."""
    lib = _load()
    out = np.empty(max(count, 1), dtype=np.int32)
    got = lib.gg_roots(g.n, _p(g.off, _i64p), count, seed, _p(out, _i32p))
    return out[:got].copy()


def csr_hash(off: np.ndarray, col: np.ndarray) -> int:
    lib = _load()
    off = np.ascontiguousarray(off)
    col = np.ascontiguousarray(col)
    h1 = lib.gg_hash_bytes(off.ctypes.data, off.nbytes)
    h2 = lib.gg_hash_bytes(col.ctypes.data, col.nbytes)
    return int(lib.gg_mix64(h1 ^ ((h2 << 1) & 0xFFFFFFFFFFFFFFFF)))


def mix64(x: int) -> int:
    return int(_load().gg_mix64(x))


def perm(x: int, bits: int, seed: int) -> int:
    return int(_load().gg_perm(x, bits, seed))


def poisson_arrivals(count: int, qps: float, seed: int) -> np.ndarray:
    """Arrival offsets in seconds of a Poisson process (seeded exponential gaps)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / qps, size=count))


# Seed conventions: graph seed = 1 + config index, root seed = 1000 + index.
CONFIGS = {
    "rmat12": dict(kind="rmat", scale=12, roots=16, graph_seed=1, root_seed=1000),
    "rmat22": dict(kind="rmat", scale=22, roots=64, graph_seed=2, root_seed=1001),
    "rmat26": dict(kind="rmat", scale=26, roots=64, graph_seed=3, root_seed=1002),
    "er26": dict(kind="er", scale=26, roots=64, graph_seed=3, root_seed=1002),
}


def config_graph(name: str) -> CSR:
    c = CONFIGS[name]
    if c["kind"] == "rmat":
        g = rmat_csr(c["scale"], 16, c["graph_seed"])
    else:
        g = er_csr(c["scale"], 16, c["graph_seed"])
    g.name = name
    return g


def config_roots(name: str, g: CSR) -> np.ndarray:
    c = CONFIGS[name]
    return roots(g, c["roots"], c["root_seed"])


def upper_csr(g: CSR) -> CSR:
    """Symmetric storage of an undirected graph (storage only): each edge
    once, in the row of its smaller endpoint, i.e. the entries v > u of every
    row u, kept in ascending order."""
    n = g.n
    goff = np.asarray(g.off, dtype=np.int64)
    cnt = np.zeros(n, np.int64)
    parts = []
    step = 1 << 21   # rows per chunk, so that scale-26 graphs fit in host memory
    for r0 in range(0, n, step):
        r1 = min(n, r0 + step)
        a, b = int(goff[r0]), int(goff[r1])
        src = np.repeat(np.arange(r0, r1, dtype=np.int32), np.diff(goff[r0:r1 + 1]))
        cols = g.col[a:b]
        keep = cols > src
        cnt[r0:r1] = np.bincount(src[keep] - r0, minlength=r1 - r0)
        parts.append(cols[keep])
    off = np.zeros(n + 1, np.int64)
    np.cumsum(cnt, out=off[1:])
    col = np.concatenate(parts) if parts else np.zeros(0, np.int32)
    return CSR(n, off, np.ascontiguousarray(col, dtype=np.int32), name=g.name + "_upper")


def csr_to_2d(g: CSR, pr: int, pc: int):
    """The p_r x p_c decomposition of a graph's adjacency matrix into DCSC
    shares (storage only). A(v, u) = 1 for each stored adjacency u -> v, so
    column u of the matrix holds u's adjacencies. Row block i covers global
    rows [i*R, min((i+1)*R, n)) with R = ceil(n / p_r), column block j global
    columns [j*C, ...) with C = ceil(n / p_c); share (i, j) is returned at
    index i * p_c + j with local ids (rows ascending within each column).
    Returns (R, C, shares)."""
    n = g.n
    R, C = -(-n // pr), -(-n // pc)
    if (pr - 1) * R >= n or (pc - 1) * C >= n:
        raise ValueError("every share needs at least one row and one column")
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(g.off))
    dst = g.col.astype(np.int64)
    bi, bj = dst // R, src // C
    shares = []
    for i in range(pr):
        nrows = min(R, n - i * R)
        for j in range(pc):
            ncols = min(C, n - j * C)
            sel = (bi == i) & (bj == j)
            r = (dst[sel] - i * R).astype(np.int64)
            k = (src[sel] - j * C).astype(np.int64)
            order = np.lexsort((r, k))
            r, k = r[order], k[order]
            jc, start = np.unique(k, return_index=True)
            cp = np.append(start, r.size).astype(np.int32)
            shares.append(DCSCBlock(nrows, ncols, jc.astype(np.int32), cp, r.astype(np.int32)))
    return R, C, shares
