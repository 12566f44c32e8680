"""Full-size parity: the scale-26 R-MAT and Erdos-Renyi configurations, each
searched as bench.py does (degree-ordered copy, symmetric graph, default
launch shapes) from its first four seeded roots, and checked against the
definition (oracle checker: levels are hop distances, parents the
minimum-id neighbour one level up, every reached vertex and no other). The
checks run on host threads in parallel while the GPU searches the next
root."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import graphgen
import oracle
from gpu_helpers import gpu_bfs, say
from paper_1104_4518_amd import bfs as B

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.mark.parametrize("workload", ["rmat26", "er26"])
def test_scale26_config_checked_against_definition(workload):
    say(f"{workload}: generating")
    g = graphgen.config_graph(workload)
    roots = graphgen.config_roots(workload, g)
    G = B.Graph.from_csr(g.n, g.off, g.col, trusted=True, symmetric=True)
    pending = []
    with ThreadPoolExecutor(max_workers=4) as pool:
        for r in [int(x) for x in roots[:4]]:
            say(f"{workload}: root {r}")
            p, lv = gpu_bfs(G, r)
            st = G.last_stats()
            assert st.reached == int((lv >= 0).sum())
            assert st.depth == int(lv.max())
            pending.append((r, st, lv, pool.submit(oracle.check_bfs, g, r, p, lv)))
        for r, st, lv, fut in pending:
            say(f"{workload}: checking root {r} ({st.reached} reached)")
            assert fut.result() == (0, -1), r
            assert st.edges_traversed == 2 * oracle.reached_edges(g, lv)
    # a second run on the same handle (workspace reuse) gives the same arrays
    r = int(roots[0])
    p0, l0 = gpu_bfs(G, r)
    p1, l1 = gpu_bfs(G, r)
    assert np.array_equal(p0, p1) and np.array_equal(l0, l1)
