"""MI355X (gfx950) implementation of the CPRA training step.

CPRA (Continuous Parallel Relaxation Annealing, Ichikawa & Iwashita, TMLR
2025) trains S relaxed solutions of a combinatorial problem at once: a GNN
maps the graph to an N x S matrix of per-node, per-head probabilities, and
one loss -- each head's penalty objective, an annealing term and a
cross-head diversity term -- is minimised by gradient steps.

All computation runs in ``libcpra.so`` (hand-written HIP kernels behind the C
ABI of ``include/cpra.h``); this package is its ctypes binding
(``api``, same names as the C entry points), a solver that owns the device
buffers (``solver``) and a ``torch.autograd.Function`` around the
hand-written backward (``autograd``).  torch provides device memory and
streams only.
"""

from ._lib import CpraError  # noqa: F401
from .api import DeviceGraph  # noqa: F401
from .solver import CPRAConfig, CPRASolver, SolveResult, gamma_schedule, solve  # noqa: F401
