"""Shared helpers of the GPU tests: device buffers and calls through the C ABI."""
import sys

import numpy as np

import oracle
from paper_1104_4518_amd import bfs as B


def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


def say(msg: str) -> None:
    """Names the case on stdout before a GPU step (flushed)."""
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def graph_on_device(g, trusted=False):
    return B.Graph.from_csr(g.n, g.off, g.col, trusted=trusted)


def gpu_bfs(G, root, want_level=True, stream=None):
    torch = torch_cuda()
    parent = torch.empty(G.n, dtype=torch.int32, device="cuda")
    level = torch.empty(G.n, dtype=torch.int32, device="cuda") if want_level else None
    G.run(int(root), parent, level, stream=stream)
    torch.cuda.synchronize()
    return parent.cpu().numpy(), (level.cpu().numpy() if want_level else None)


def assert_bfs_equal(g, G, root, want_level=True):
    p, lv = gpu_bfs(G, root, want_level)
    op, ol = oracle.bfs_graph(g, int(root))
    assert np.array_equal(p, op), f"parent mismatch at root {root}: " \
        f"{np.nonzero(p != op)[0][:10]}"
    if want_level:
        assert np.array_equal(lv, ol), f"level mismatch at root {root}"
    return op, ol


def gpu_spmspv(Gb, fidx, fval=None, capacity=None):
    torch = torch_cuda()
    f = torch.from_numpy(np.ascontiguousarray(fidx, dtype=np.int32)).cuda()
    fv = (torch.from_numpy(np.ascontiguousarray(fval, dtype=np.int32)).cuda()
          if fval is not None else None)
    cap = capacity if capacity is not None else max(1, min(Gb.n, Gb.nnz))
    oi = torch.empty(max(cap, 1), dtype=torch.int32, device="cuda")
    ov = torch.empty(max(cap, 1), dtype=torch.int32, device="cuda")
    cnt = Gb.spmspv(f if len(fidx) else None, len(fidx), oi, ov, cap, fval=fv)
    torch.cuda.synchronize()
    return oi[:cnt].cpu().numpy(), ov[:cnt].cpu().numpy()
