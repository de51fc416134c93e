"""FP64 CPU oracle for the CPRA training step -- TEST INFRASTRUCTURE ONLY.

This package is the checker, not the product.  Only the tests, the smoke
check and the benchmark's CPU-baseline leg may import it; the library in
``paper_2402_02190_amd`` never does, and nothing here imports that library.
It shares no code with the HIP path: the only common dependency is the
``workloads`` package, which generates seeded graphs and initial parameters
and contains none of the method's arithmetic.

Everything is plain NumPy/SciPy in float64, written from the paper
(Ichikawa & Iwashita, "Continuous Parallel Relaxation for Finding Diverse
Solutions in Combinatorial Optimization Problems", TMLR 2025):

* ``objective`` -- the penalty objectives of the problem table in the
  problem-specification appendix, their relaxation (Sec. 2.2), the
  annealing term S(P) and the CPRA loss (Sec. 3.1, Eq. CPRA-loss-function-GNN),
  the diversity term Psi (Sec. 3.3, Eq. CPRA-loss-function-GNN-variation) and
  the analytic gradient with respect to P and to the logits Z.
* ``gnn`` -- the aggregate/combine GNN of the GNN appendix (mean
  aggregation, GCN form, GraphSAGE = GCN form plus bias) and its backward.
* ``train`` -- the gamma schedule (Sec. 4.1 Implementation), Adam/AdamW,
  one training step and the full solve loop.
* ``evaluate`` -- threshold rounding (training-setting appendix), MIS size,
  violations, cut value, DScore (Sec. 4.1 Evaluation Metrics) and the
  max-sum Hamming distance (Proposition 3.2).
* ``exact`` -- brute-force and MILP optima for small graphs.
* ``warmstart`` -- the learned warm start: bfloat16 rounding, triangle counts
  and clustering features, the BF16 message-passing network, its backward and
  its training objective (CPRA loss + distillation onto converged solutions).

Pins (tests marked ``not gpu``) tie each function to something other than
itself: the relaxed loss equals the discrete objective on {0,1} (checked
against networkx), finite differences, Proposition 3.2 by brute force,
Lemma A.1 endpoints, Theorem 3.1 limits, the parameter-count identities of
the MIS/DBM result tables, Adam against torch.optim on CPU, textbook optima.
"""
