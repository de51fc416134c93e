"""Input generators: the near-regular permutation graph used by the size sweeps
is a valid simple symmetric CSR with (almost) every degree equal to d."""

import numpy as np

from workloads import csr_from_edges, random_permutation_graph


def test_permutation_graph_is_simple_symmetric_and_near_regular():
    g = random_permutation_graph(5000, 20, seed=3)
    rp, ci = g.row_ptr.astype(np.int64), g.col_idx.astype(np.int64)
    deg = np.diff(rp)
    rows = np.repeat(np.arange(g.n), deg)
    assert np.all(ci != rows)                                        # no self loops
    for i in range(0, g.n, 97):
        seg = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(seg) > 0)                              # sorted, no repeats
    a = set(zip(rows.tolist(), ci.tolist()))
    assert all((j, i) in a for i, j in list(a)[:20000])              # symmetric
    assert deg.max() <= 20 and np.mean(deg == 20) > 0.95   # O(d^2 / n) defects
    # the same edge set through the general constructor gives the same CSR
    ei, ej, _ = g.edge_list()
    h = csr_from_edges(g.n, ei, ej)
    assert np.array_equal(h.row_ptr, g.row_ptr) and np.array_equal(h.col_idx, g.col_idx)
