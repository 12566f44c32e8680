"""Single-GPU emulated 2D BFS (bfs_run_2d over a p_r x p_c grid of DCSC
shares) against the CPU oracle, bit for bit."""
import numpy as np
import pytest

import graphgen
import oracle
from gpu_helpers import say, torch_cuda
from paper_1104_4518_amd import bfs as B

pytestmark = pytest.mark.gpu


def shares_on_device(g, pr, pc):
    R, C, shares = graphgen.csr_to_2d(g, pr, pc)
    return [B.Graph.from_dcsc(s.nrows, s.ncols, s.jc, s.cp, s.ir) for s in shares]


def run_2d(handles, pr, pc, n, root):
    torch = torch_cuda()
    p = torch.empty(n, dtype=torch.int32, device="cuda")
    lv = torch.empty(n, dtype=torch.int32, device="cuda")
    B.run_2d(handles, pr, pc, n, root, p, lv)
    torch.cuda.synchronize()
    return p.cpu().numpy(), lv.cpu().numpy()


def directed_graph(n, m, seed):
    rng = np.random.default_rng(seed)
    src, dst = rng.integers(0, n, m), rng.integers(0, n, m)
    order = np.lexsort((dst, src))
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum(np.bincount(src[order], minlength=n))
    return graphgen.CSR(n, off, dst[order].astype(np.int32))


@pytest.mark.parametrize("pr,pc", [(1, 1), (2, 2), (2, 3), (4, 4)])
def test_2d_grids_match_oracle(pr, pc):
    graphs = [("rmat14", graphgen.rmat_csr(14, 16, 51)), ("grid40", graphgen.grid_csr(40)),
              ("directed", directed_graph(5000, 30000, 8))]
    for name, g in graphs:
        hs = shares_on_device(g, pr, pc)
        for r in graphgen.roots(g, 3, 17):
            say(f"2d {pr}x{pc} {name} root {r}")
            p, lv = run_2d(hs, pr, pc, g.n, int(r))
            op, ol = oracle.bfs_graph(g, int(r))
            assert np.array_equal(p, op) and np.array_equal(lv, ol)


def test_2d_share_at_scale_18_and_tuned_shares():
    """R-MAT scale 18 on a 4 x 4 grid, once with the shares' default SpMSpV
    switch and once after bfs_tune picked it per share."""
    g = graphgen.rmat_csr(18, 16, 52)
    hs = shares_on_device(g, 4, 4)
    r = int(graphgen.roots(g, 1, 3)[0])
    op, ol = oracle.bfs_graph(g, r)
    say("2d 4x4 rmat18")
    p, lv = run_2d(hs, 4, 4, g.n, r)
    assert np.array_equal(p, op) and np.array_equal(lv, ol)
    for h in hs:
        h.tune()
    say("2d 4x4 rmat18 tuned")
    p, lv = run_2d(hs, 4, 4, g.n, r)
    assert np.array_equal(p, op) and np.array_equal(lv, ol)


def test_2d_errors():
    g = graphgen.rmat_csr(10, 16, 5)
    hs = shares_on_device(g, 2, 2)
    torch = torch_cuda()
    p = torch.empty(g.n, dtype=torch.int32, device="cuda")
    with pytest.raises(B.BfsError) as ei:           # wrong grid shape for the shares
        B.run_2d(hs, 1, 4, g.n, 0, p)
    assert ei.value.code == B.BFS_ERR_ARG
    with pytest.raises(B.BfsError) as ei:           # a handle twice
        B.run_2d([hs[0], hs[0], hs[2], hs[3]], 2, 2, g.n, 0, p)
    assert ei.value.code == B.BFS_ERR_ARG
    with pytest.raises(B.BfsError) as ei:           # host output
        B.run_2d(hs, 2, 2, g.n, 0, np.empty(g.n, np.int32))
    assert ei.value.code == B.BFS_ERR_ARG
    with pytest.raises(B.BfsError) as ei:           # root out of range
        B.run_2d(hs, 2, 2, g.n, g.n, p)
    assert ei.value.code == B.BFS_ERR_ARG
    # the shares still work afterwards
    r = int(graphgen.roots(g, 1, 2)[0])
    pp, lv = run_2d(hs, 2, 2, g.n, r)
    op, ol = oracle.bfs_graph(g, r)
    assert np.array_equal(pp, op) and np.array_equal(lv, ol)
