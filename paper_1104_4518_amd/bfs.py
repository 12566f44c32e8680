"""ctypes binding of libbfs.so: argument marshalling only.

Every step of BFS and SpMSpV runs in the library's HIP kernels. PyTorch
tensors serve as device memory and PyTorch streams as HIP streams; numpy
arrays are accepted for host-side inputs. The binding never falls back to
a CPU path: if the library is missing or fails to load, it raises.

Names follow the C ABI in include/bfs.h.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbfs.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "bfs.h")

BFS_OK = 0
BFS_ERR_ARG = -1
BFS_ERR_FORMAT = -2
BFS_ERR_OOM = -3
BFS_ERR_CAPACITY = -4
BFS_ERR_DEVICE = -5
BFS_ERR_BUSY = -6
BFS_ERR_TIMEOUT = -7
BFS_ERR_UNSUPPORTED = -8

BFS_DEVICE_PTRS = 0x1
BFS_TRUSTED = 0x2
BFS_SYMMETRIC = 0x4
BFS_NO_RELABEL = 0x8
BFS_UPPER = 0x10

_NAMES = {v: k for k, v in globals().items() if k.startswith("BFS_ERR_") or k == "BFS_OK"}


class BfsError(RuntimeError):
    def __init__(self, code: int, func: str, msg: str):
        super().__init__(f"{func} -> {_NAMES.get(code, code)}: {msg}")
        self.code = code


class SVec(ctypes.Structure):
    _fields_ = [("nnz", ctypes.c_int64), ("capacity", ctypes.c_int64),
                ("idx", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class RunStats(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("edges_traversed", ctypes.c_int64), ("reached", ctypes.c_int64),
                ("frontier_total", ctypes.c_int64), ("expand_launches", ctypes.c_int32),
                ("mark_levels", ctypes.c_int32), ("expand_ms", ctypes.c_double),
                ("mark_ms", ctypes.c_double), ("total_ms", ctypes.c_double),
                ("pull_levels", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("pull_ms", ctypes.c_double), ("pull_edges", ctypes.c_int64),
                ("small_levels", ctypes.c_int32), ("reserved2", ctypes.c_int32),
                ("small_ms", ctypes.c_double), ("finish_ms", ctypes.c_double)]


class LevelInfo(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("mark", ctypes.c_int32),
                ("frontier", ctypes.c_int64), ("edges", ctypes.c_int64),
                ("expand_ms", ctypes.c_double), ("mark_ms", ctypes.c_double),
                ("finish_ms", ctypes.c_double), ("pull_ms", ctypes.c_double),
                ("pull_candidates", ctypes.c_int64), ("pull_edges", ctypes.c_int64),
                ("small_ms", ctypes.c_double)]


class Options(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("batch_levels", ctypes.c_int32),
                ("grid_blocks", ctypes.c_int32), ("lds_bitmap", ctypes.c_int32),
                ("profile", ctypes.c_int32), ("claim", ctypes.c_int32),
                ("claim_threshold", ctypes.c_int32), ("claim_min_frontier", ctypes.c_int32),
                ("cold_probe", ctypes.c_int32), ("spmspv_sort_max", ctypes.c_int32),
                ("pull_alpha", ctypes.c_int32), ("small_frontier", ctypes.c_int32)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("memory_budget", ctypes.c_int64),
                ("step_budget_us", ctypes.c_int32), ("large_query_nnz", ctypes.c_int64)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("depth", ctypes.c_int32),
                ("edges_traversed", ctypes.c_int64), ("t_arrive", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


_lib = None
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64


def header_functions() -> list[str]:
    """Function names declared in include/bfs.h."""
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bfs_[a-z_0-9]+)\s*\(", text)))


def load(build_if_missing: bool = True):
    """Loads libbfs.so; builds it first only when no library is present."""
    global _lib
    if _lib is not None:
        return _lib
    # PyTorch ships its own HIP runtime with the same soname as ROCm's. Loading
    # torch first makes libbfs.so bind to that one runtime, so device memory
    # and streams are shared and the process never holds two HIP runtimes.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        if not build_if_missing:
            raise RuntimeError(f"{LIB_PATH} is not built")
        from . import build as _build
        _build.build()
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "bfs_graph_create_csr": [_i64, _i64, _vp, ctypes.c_int, _vp, ctypes.c_uint32,
                                 ctypes.POINTER(_vp)],
        "bfs_graph_create_dcsc": [_i32, _i32, _i32, _i64, _vp, _vp, _vp, ctypes.c_uint32,
                                  ctypes.POINTER(_vp)],
        "bfs_graph_destroy": [_vp],
        "bfs_graph_info": [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64),
                           ctypes.POINTER(_i64)],
        "bfs_graph_set_options": [_vp, ctypes.POINTER(Options)],
        "bfs_graph_get_options": [_vp, ctypes.POINTER(Options)],
        "bfs_run": [_vp, _i32, _vp, _vp],
        "bfs_run_async": [_vp, _i32, _vp, _vp, _vp],
        "bfs_last_stats": [_vp, ctypes.POINTER(RunStats)],
        "bfs_last_level_info": [_vp, ctypes.POINTER(LevelInfo), _i32, ctypes.POINTER(_i32)],
        "bfs_spmspv": [_vp, ctypes.POINTER(SVec), ctypes.POINTER(SVec), _vp],
        "bfs_run_batch": [_i32, ctypes.POINTER(_vp), ctypes.POINTER(_i32), ctypes.POINTER(_vp),
                          ctypes.POINTER(_vp), _vp],
        "bfs_run_2d": [ctypes.POINTER(_vp), _i32, _i32, _i64, _i32, _vp, _vp, _vp],
        "bfs_run_2d_noalloc": [ctypes.POINTER(_vp), _i32, _i32, _i64, _i32, _vp, _vp, _vp],
        "bfs_server_create": [ctypes.POINTER(ServerConfig), ctypes.POINTER(_vp)],
        "bfs_server_submit": [_vp, _vp, _i32, _vp, _vp, ctypes.POINTER(ctypes.c_uint64)],
        "bfs_server_poll": [_vp, ctypes.c_uint64, ctypes.POINTER(Result)],
        "bfs_server_wait": [_vp, ctypes.c_uint64, ctypes.c_double, ctypes.POINTER(Result)],
        "bfs_server_drain": [_vp],
        "bfs_server_destroy": [_vp],
        "bfs_tune": [_vp, ctypes.c_char_p],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.bfs_last_error.restype = ctypes.c_char_p
    lib.bfs_last_error.argtypes = []
    lib.bfs_version.restype = ctypes.c_char_p
    lib.bfs_version.argtypes = []
    _lib = lib
    return lib


def last_error() -> str:
    return load().bfs_last_error().decode()


def _check(rc: int, func: str) -> int:
    if rc != BFS_OK:
        raise BfsError(rc, func, last_error())
    return rc


def _ptr(a) -> Optional[int]:
    """Device or host address of a torch tensor / numpy array (None -> NULL)."""
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return int(a.data_ptr())
    if isinstance(a, np.ndarray):
        return int(a.ctypes.data)
    if isinstance(a, int):
        return a
    raise TypeError(f"unsupported array type {type(a)}")


def _is_device(a) -> bool:
    return hasattr(a, "is_cuda") and bool(a.is_cuda)


def _stream(stream) -> Optional[int]:
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return int(stream.cuda_stream)
    return int(stream)


class Graph:
    """Owning wrapper of a bfs_graph_t handle (CSR graph or DCSC block)."""

    def __init__(self, handle: int, kind: str, n: int, nnz: int):
        self.handle = handle
        self.kind = kind
        self.n = n
        self.nnz = nnz

    # ---------------------------------------------------------------- create
    @classmethod
    def from_csr(cls, n: int, off, col, trusted: bool = False,
                 symmetric: Optional[bool] = None, relabel: bool = True,
                 upper: bool = False) -> "Graph":
        """symmetric=True asserts an undirected graph with ascending rows;
        None lets the library check it (unless trusted). relabel=False
        skips the degree-ordered copy of large graphs. upper=True: the
        arrays hold each undirected edge once, in the row of its smaller
        endpoint (BFS_UPPER); the symmetric closure is searched."""
        lib = load()
        dev = _is_device(off)
        if dev != _is_device(col):
            raise ValueError("off and col must both be host or both be device arrays")
        if not dev:
            off = np.ascontiguousarray(off)
            col = np.ascontiguousarray(col, dtype=np.int32)
        ob = 8 if str(off.dtype).endswith("int64") else 4
        if ob == 4 and not str(off.dtype).endswith("int32"):
            raise TypeError("row offsets must be int32 or int64")
        flags = (BFS_DEVICE_PTRS if dev else 0) | (BFS_TRUSTED if trusted else 0)
        if symmetric:
            flags |= BFS_SYMMETRIC
        if not relabel:
            flags |= BFS_NO_RELABEL
        if upper:
            flags |= BFS_UPPER
        h = _vp()
        nnz = int(col.shape[0])
        _check(lib.bfs_graph_create_csr(n, nnz, _ptr(off), ob, _ptr(col) if nnz else None, flags,
                                        ctypes.byref(h)), "bfs_graph_create_csr")
        g = cls(h.value, "csr", n, nnz)
        if symmetric is False:
            g.set_options(claim=1)
        return g

    @classmethod
    def from_dcsc(cls, nrows: int, ncols: int, jc, cp, ir, trusted: bool = False) -> "Graph":
        lib = load()
        dev = _is_device(ir)
        if not dev:
            jc = np.ascontiguousarray(jc, dtype=np.int32)
            cp = np.ascontiguousarray(cp, dtype=np.int32)
            ir = np.ascontiguousarray(ir, dtype=np.int32)
        flags = (BFS_DEVICE_PTRS if dev else 0) | (BFS_TRUSTED if trusted else 0)
        h = _vp()
        nzc = int(jc.shape[0])
        nnz = int(ir.shape[0])
        _check(lib.bfs_graph_create_dcsc(nrows, ncols, nzc, nnz, _ptr(jc) if nzc else None,
                                         _ptr(cp), _ptr(ir) if nnz else None, flags,
                                         ctypes.byref(h)), "bfs_graph_create_dcsc")
        return cls(h.value, "dcsc", nrows, nnz)

    def destroy(self):
        if self.handle:
            _check(load().bfs_graph_destroy(self.handle), "bfs_graph_destroy")
            self.handle = None

    def __del__(self):
        try:
            if self.handle and _lib is not None:
                _lib.bfs_graph_destroy(self.handle)
                self.handle = None
        except Exception:
            pass

    # ---------------------------------------------------------------- queries
    def info(self):
        n, nnz, b = _i64(), _i64(), _i64()
        _check(load().bfs_graph_info(self.handle, ctypes.byref(n), ctypes.byref(nnz),
                                     ctypes.byref(b)), "bfs_graph_info")
        return n.value, nnz.value, b.value

    def set_options(self, mode=0, batch_levels=0, grid_blocks=0, lds_bitmap=0, profile=0,
                    claim=0, claim_threshold=0, claim_min_frontier=0, cold_probe=0,
                    spmspv_sort_max=0, pull_alpha=0, small_frontier=0):
        o = Options(mode, batch_levels, grid_blocks, lds_bitmap, profile, claim, claim_threshold,
                    claim_min_frontier, cold_probe, spmspv_sort_max, pull_alpha, small_frontier)
        _check(load().bfs_graph_set_options(self.handle, ctypes.byref(o)),
               "bfs_graph_set_options")

    def get_options(self) -> Options:
        o = Options()
        _check(load().bfs_graph_get_options(self.handle, ctypes.byref(o)),
               "bfs_graph_get_options")
        return o

    def run(self, root: int, parent, level=None, stream=None) -> None:
        """BFS from root into parent (required) and level (optional)."""
        lib = load()
        if stream is None:
            _check(lib.bfs_run(self.handle, int(root), _ptr(parent), _ptr(level)), "bfs_run")
        else:
            _check(lib.bfs_run_async(self.handle, int(root), _ptr(parent), _ptr(level),
                                     _stream(stream)), "bfs_run_async")

    def last_stats(self) -> RunStats:
        st = RunStats()
        _check(load().bfs_last_stats(self.handle, ctypes.byref(st)), "bfs_last_stats")
        return st

    def level_info(self) -> list:
        """Per-level records of the last profiled run (dicts)."""
        buf = (LevelInfo * 4096)()
        cnt = _i32()
        _check(load().bfs_last_level_info(self.handle, buf, 4096, ctypes.byref(cnt)),
               "bfs_last_level_info")
        return [{f: getattr(buf[i], f) for f, _ in LevelInfo._fields_}
                for i in range(min(cnt.value, 4095))]

    def spmspv(self, fidx, fnnz: int, out_idx, out_val, capacity: int, fval=None,
               stream=None) -> int:
        """Local product into (out_idx, out_val); returns the output count."""
        f = SVec(int(fnnz), int(fnnz), _ptr(fidx), _ptr(fval))
        o = SVec(0, int(capacity), _ptr(out_idx), _ptr(out_val))
        rc = load().bfs_spmspv(self.handle, ctypes.byref(f), ctypes.byref(o), _stream(stream))
        if rc == BFS_ERR_CAPACITY:
            raise BfsError(rc, "bfs_spmspv", f"{last_error()} (need {o.nnz})")
        _check(rc, "bfs_spmspv")
        return int(o.nnz)

    def tune(self, cache_path: Optional[str] = None) -> None:
        _check(load().bfs_tune(self.handle, cache_path.encode() if cache_path else None),
               "bfs_tune")


def run_batch(graphs: Sequence[Graph], roots, parents, levels=None, stream=None) -> None:
    """One persistent launch for all (graph, root) queries."""
    lib = load()
    cnt = len(graphs)
    hs = (_vp * cnt)(*[g.handle for g in graphs])
    rs = (_i32 * cnt)(*[int(r) for r in roots])
    ps = (_vp * cnt)(*[_ptr(p) for p in parents])
    lv = (_vp * cnt)(*[(_ptr(x) if x is not None else None) for x in
                       (levels if levels is not None else [None] * cnt)])
    _check(lib.bfs_run_batch(cnt, hs, rs, ps, lv, _stream(stream)), "bfs_run_batch")


def run_2d(shares: Sequence[Graph], pr: int, pc: int, n: int, root: int, parent, level=None,
           stream=None) -> None:
    """BFS over a p_r x p_c grid of DCSC share handles (row-major), device outputs."""
    cnt = len(shares)
    hs = (_vp * cnt)(*[g.handle for g in shares])
    _check(load().bfs_run_2d(hs, int(pr), int(pc), int(n), int(root), _ptr(parent), _ptr(level),
                             _stream(stream)), "bfs_run_2d")


def run_2d_noalloc(shares: Sequence[Graph], pr: int, pc: int, n: int, root: int, parent,
                   level=None, stream=None) -> None:
    """bfs_run_2d on the library's fixed device workspace (no allocation)."""
    cnt = len(shares)
    hs = (_vp * cnt)(*[g.handle for g in shares])
    _check(load().bfs_run_2d_noalloc(hs, int(pr), int(pc), int(n), int(root), _ptr(parent),
                                     _ptr(level), _stream(stream)), "bfs_run_2d_noalloc")


class Server:
    """Continuous-batching BFS server (bfs_server_*)."""

    def __init__(self, slots: int = 64, memory_budget: int = 0, step_budget_us: int = 0,
                 large_query_nnz: int = 0):
        cfg = ServerConfig(slots, memory_budget, step_budget_us, large_query_nnz)
        h = _vp()
        _check(load().bfs_server_create(ctypes.byref(cfg), ctypes.byref(h)), "bfs_server_create")
        self.handle = h.value

    def submit(self, g: Graph, root: int, parent, level=None) -> int:
        t = ctypes.c_uint64()
        _check(load().bfs_server_submit(self.handle, g.handle, int(root), _ptr(parent),
                                        _ptr(level), ctypes.byref(t)), "bfs_server_submit")
        return int(t.value)

    def poll(self, ticket: int) -> Result:
        r = Result()
        _check(load().bfs_server_poll(self.handle, ticket, ctypes.byref(r)), "bfs_server_poll")
        return r

    def wait(self, ticket: int, timeout_s: float = 60.0) -> Result:
        r = Result()
        _check(load().bfs_server_wait(self.handle, ticket, timeout_s, ctypes.byref(r)),
               "bfs_server_wait")
        return r

    def drain(self) -> None:
        _check(load().bfs_server_drain(self.handle), "bfs_server_drain")

    def destroy(self) -> None:
        if self.handle:
            _check(load().bfs_server_destroy(self.handle), "bfs_server_destroy")
            self.handle = None


def version() -> str:
    return load().bfs_version().decode()
