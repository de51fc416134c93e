"""Seeded synthetic inputs shared by the HIP path, the oracle and the benchmarks.

This package holds input generation only: random graphs in CSR form, the
seeded initial parameters of the GNN and the named workload presets (sizes,
penalty grids, schedules).  It contains none of the method's arithmetic (no
loss, no gradient, no aggregation), so that the oracle and the GPU path can
both consume it without sharing any computation.
"""

from .graphs import (  # noqa: F401
    CSRGraph,
    csr_from_edges,
    random_regular_graph,
    random_permutation_graph,
    erdos_renyi_graph,
    disjoint_union,
    induced_subgraph,
    bfs_ball,
    instance_edge_weights,
)
from .params import init_mpnn_params, init_params, init_params_per_graph, param_shapes, \
    random_channels  # noqa: F401
from .presets import PRESETS, Preset, get_preset  # noqa: F401
