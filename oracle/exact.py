"""Exact optima for small graphs.  TEST INFRASTRUCTURE ONLY.

* ``bruteforce_min`` enumerates all 2^N binary vectors (N <= 22) and
  returns the minimum of a penalty objective of the problem table together
  with every minimiser.
* ``mis_size_milp`` solves the independent-set integer program
  max sum x_i s.t. x_i + x_j <= 1 for every edge, x binary, with
  scipy's HiGHS MILP solver (for graphs too large to enumerate).
"""

from __future__ import annotations

import numpy as np
from scipy.optimize import Bounds, LinearConstraint, milp

from .objective import edges_of


def _all_codes(n: int):
    codes = np.arange(1 << n, dtype=np.int64)
    return codes, [((codes >> i) & 1).astype(np.int8) for i in range(n)]


def bruteforce_values(graph, problem: str, lam: float = 2.0) -> np.ndarray:
    """Objective value of every x in {0,1}^N, indexed by the integer code of x (bit i = x_i)."""
    n = len(graph.row_ptr) - 1
    if n > 22:
        raise ValueError("brute force limited to N <= 22")
    ei, ej, w = edges_of(graph.row_ptr, graph.col_idx, graph.weight)
    codes, bits = _all_codes(n)
    vals = np.zeros(codes.size, dtype=np.float64)
    if problem == "mis":
        for i in range(n):
            vals -= bits[i]
        for a, b, wt in zip(ei, ej, w):
            vals += lam * wt * (bits[a] & bits[b])
    elif problem == "maxcut":
        for a, b, wt in zip(ei, ej, w):
            xa, xb = bits[a].astype(np.float64), bits[b].astype(np.float64)
            vals += wt * (2 * xa * xb - xa - xb)
    else:
        raise ValueError(problem)
    return vals


def bruteforce_min(graph, problem: str, lam: float = 2.0):
    vals = bruteforce_values(graph, problem, lam)
    best = vals.min()
    return float(best), np.nonzero(vals == best)[0]


def code_to_x(code: int, n: int) -> np.ndarray:
    return np.array([(code >> i) & 1 for i in range(n)], dtype=np.uint8)


def mis_size_bruteforce(graph) -> int:
    """alpha(G): the largest set with no edge inside, by enumeration."""
    n = len(graph.row_ptr) - 1
    ei, ej, _ = edges_of(graph.row_ptr, graph.col_idx, None)
    codes, bits = _all_codes(n)
    ok = np.ones(codes.size, dtype=bool)
    for a, b in zip(ei, ej):
        ok &= ~((bits[a] & bits[b]).astype(bool))
    size = np.zeros(codes.size, dtype=np.int64)
    for i in range(n):
        size += bits[i]
    return int(size[ok].max())


def maxcut_bruteforce(graph) -> float:
    vals = bruteforce_values(graph, "maxcut")
    return float(-vals.min())


def mis_size_milp(graph) -> int:
    n = len(graph.row_ptr) - 1
    ei, ej, _ = edges_of(graph.row_ptr, graph.col_idx, None)
    if ei.size == 0:
        return n
    A = np.zeros((ei.size, n))
    A[np.arange(ei.size), ei] = 1.0
    A[np.arange(ei.size), ej] = 1.0
    res = milp(c=-np.ones(n), constraints=LinearConstraint(A, -np.inf, 1.0),
               integrality=np.ones(n), bounds=Bounds(0, 1))
    if not res.success:
        raise RuntimeError(res.message)
    return int(round(-res.fun))
