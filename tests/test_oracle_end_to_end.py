"""The oracle's full training loop on the 100-node cubic-graph workload, checked
against the exact independence number (MILP) and networkx."""

import networkx as nx
import numpy as np

from oracle import evaluate, exact, train
from workloads import get_preset, init_params


def test_c1_oracle_solve_reaches_near_optimal_independent_sets():
    p = get_preset("C1")
    g = p.graph()
    params = init_params(p.layer_kind, g.n, p.n_layers, p.hidden, p.S, seed=11)
    cfg = train.StepConfig(problem="mis", lam=p.lam, alpha=p.alpha, lr=p.lr)
    res = train.solve(params, g, cfg, p.T, p.gamma_start, p.gamma_end)
    ev = res["eval"][0]
    alpha_g = exact.mis_size_milp(g)
    best = evaluate.best_feasible_mis(ev)
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    ei, ej, _ = g.edge_list()
    G.add_edges_from(zip(ei.tolist(), ej.tolist()))
    for s in range(p.S):
        chosen = np.nonzero(res["X"][:, s])[0].tolist()
        assert ev["violations"][s] == G.subgraph(chosen).number_of_edges()
        if ev["violations"][s] == 0:
            assert len(chosen) <= alpha_g
    # every head with lambda > 1 is feasible after annealing; quality near the optimum
    assert np.all(ev["violations"][p.lam > 1.0] == 0)
    assert best <= alpha_g and best >= 0.9 * alpha_g
    # annealing leaves the relaxed solutions near-binary (training-setting appendix)
    assert np.min(np.abs(res["Z"])) > 1e-2
