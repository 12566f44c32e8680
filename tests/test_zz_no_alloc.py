"""bfs_run_2d_noalloc (the 2D search on the library's fixed device workspace,
for callers that cannot allocate) against bfs_run_2d, bit for bit, through
the C ABI: two calls in a row, the second on a smaller input, and the
limits it rejects."""
import numpy as np
import pytest

import graphgen
from gpu_helpers import say, torch_cuda
from paper_1104_4518_amd import bfs as B

pytestmark = pytest.mark.gpu


def shares_on_device(g, pr, pc):
    _, _, shares = graphgen.csr_to_2d(g, pr, pc)
    return [B.Graph.from_dcsc(s.nrows, s.ncols, s.jc, s.cp, s.ir) for s in shares]


def both(handles, pr, pc, n, root):
    torch = torch_cuda()
    out = []
    for fn in (B.run_2d, B.run_2d_noalloc):
        p = torch.full((n,), -9, dtype=torch.int32, device="cuda")
        lv = torch.full((n,), -9, dtype=torch.int32, device="cuda")
        fn(handles, pr, pc, n, root, p, lv)
        torch.cuda.synchronize()
        out.append((p.cpu().numpy(), lv.cpu().numpy()))
    return out


def test_noalloc_matches_allocating_2d_run_then_a_smaller_one():
    big = graphgen.rmat_csr(19, 16, 61)          # 2^19 vertices, a 3 x 2 grid
    small = graphgen.grid_csr(60)                 # 3,600 vertices, 2 x 2
    hb = shares_on_device(big, 3, 2)
    hs = shares_on_device(small, 2, 2)
    for name, g, h, pr, pc in (("rmat19", big, hb, 3, 2), ("grid60", small, hs, 2, 2)):
        r = int(graphgen.roots(g, 1, 7)[0])
        say(f"noalloc 2d {name} {pr}x{pc} root {r}")
        (p0, l0), (p1, l1) = both(h, pr, pc, g.n, r)
        assert np.array_equal(p0, p1) and np.array_equal(l0, l1)
        assert (l1 >= 0).sum() > 1
    # and the large one again after the small one (the scratch keeps the
    # small run's contents; every call initialises what it reads)
    r = int(graphgen.roots(big, 2, 8)[1])
    say(f"noalloc 2d rmat19 again root {r}")
    (p0, l0), (p1, l1) = both(hb, 3, 2, big.n, r)
    assert np.array_equal(p0, p1) and np.array_equal(l0, l1)


def test_noalloc_rejects_sizes_beyond_its_workspace():
    torch = torch_cuda()
    g = graphgen.grid_csr(1025)                   # 1,050,625 vertices > 2^20
    h = shares_on_device(g, 1, 1)
    p = torch.empty(g.n, dtype=torch.int32, device="cuda")
    say("noalloc rejects n > 2^20")
    with pytest.raises(B.BfsError) as ei:
        B.run_2d_noalloc(h, 1, 1, g.n, 0, p)
    assert ei.value.code == B.BFS_ERR_CAPACITY
    # the allocating entry point still runs it
    B.run_2d(h, 1, 1, g.n, 0, p)
    torch.cuda.synchronize()
    assert int(p[0].item()) == 0
