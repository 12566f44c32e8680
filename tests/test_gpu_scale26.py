"""Full-size parity: the scale-26 R-MAT and Erdos-Renyi configurations, each
searched as bench.py does (degree-ordered copy, symmetric graph, default
launch shapes), from its first seeded root, and checked against the
definition (oracle checker: levels are hop distances, parents the minimum-id
neighbour one level up, every reached vertex and no other)."""
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
    r = int(roots[0])
    say(f"{workload}: root {r}")
    p, lv = gpu_bfs(G, r)
    st = G.last_stats()
    assert st.reached == int((lv >= 0).sum())
    assert st.depth == int(lv.max())
    say(f"{workload}: checking {st.reached} reached vertices")
    assert oracle.check_bfs(g, r, p, lv) == (0, -1)
    assert st.edges_traversed == 2 * oracle.reached_edges(g, lv)
    # a second run on the same handle (workspace reuse) gives the same arrays
    p2, lv2 = gpu_bfs(G, r)
    assert np.array_equal(p, p2) and np.array_equal(lv, lv2)
