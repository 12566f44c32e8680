"""MI355X-native level-synchronous BFS and hypersparse SpMSpV.

The compute path is the HIP library libbfs.so (C ABI in include/bfs.h);
this package only binds it. See :mod:`paper_1104_4518_amd.bfs`.
"""
from .bfs import (BfsError, Graph, Server, load, run_batch, version)  # noqa: F401

__all__ = ["BfsError", "Graph", "Server", "load", "run_batch", "version"]
