"""Seeded random graphs in symmetric CSR form.

Generators:

* ``random_regular_graph(n, d, seed)`` -- the pairing (configuration) model:
  every node gets ``d`` stubs, a uniformly random perfect matching of the
  stubs gives a multigraph, and each self loop or repeated edge is then
  removed by a random degree-preserving switch with a uniformly chosen
  other edge (the switching repair of McKay and Wormald).  Plain rejection
  of the pairing model is hopeless for d=20 (a simple draw has probability
  about exp(-(d*d-1)/4)), while the number of defects to repair is O(d^2)
  independent of n.
* ``erdos_renyi_graph(n, p, seed)`` -- G(n, p) by geometric skipping over the
  n(n-1)/2 node pairs (Batagelj and Brandes, 2005).

Every generator draws from ``numpy.random.Generator(PCG64(seed))``.

The CSR produced here is the graph format of the whole project: int32
``row_ptr[n+1]`` and ``col_idx[nnz]``, each row sorted ascending, no self
loops, no duplicate entries, and symmetric (j in row i iff i in row j).
``nnz`` is twice the number of undirected edges.  An optional float32
``weight[nnz]`` holds A_ij for each stored entry (symmetric as well).
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np


@dataclass
class CSRGraph:
    """A symmetric simple graph (or a block-diagonal batch of them) in CSR form.

    ``graph_ptr`` holds the node offsets of the member graphs when the graph
    is a disjoint union; for a single graph it is ``[0, n]``.
    """

    n: int
    row_ptr: np.ndarray  # int32 [n+1]
    col_idx: np.ndarray  # int32 [nnz]
    weight: Optional[np.ndarray] = None  # float32 [nnz] or None (all ones)
    graph_ptr: np.ndarray = field(default=None)  # int32 [n_graphs+1]

    def __post_init__(self):
        if self.graph_ptr is None:
            self.graph_ptr = np.array([0, self.n], dtype=np.int32)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def n_edges(self) -> int:
        return self.nnz // 2

    @property
    def n_graphs(self) -> int:
        return len(self.graph_ptr) - 1

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)

    def edge_list(self):
        """Undirected edges (i < j) as two int64 arrays, plus weights (or None)."""
        rows = np.repeat(np.arange(self.n, dtype=np.int64), self.degrees())
        cols = self.col_idx.astype(np.int64)
        keep = rows < cols
        w = None if self.weight is None else self.weight[keep]
        return rows[keep], cols[keep], w

    def save_npz(self, path: str) -> None:
        arrays = dict(n=np.int64(self.n), row_ptr=self.row_ptr, col_idx=self.col_idx,
                      graph_ptr=self.graph_ptr)
        if self.weight is not None:
            arrays["weight"] = self.weight
        np.savez_compressed(path, **arrays)

    @staticmethod
    def load_npz(path: str) -> "CSRGraph":
        z = np.load(path, allow_pickle=False)
        w = z["weight"] if "weight" in z.files else None
        return CSRGraph(int(z["n"]), z["row_ptr"], z["col_idx"], w, z["graph_ptr"])


def csr_from_edges(n: int, u: np.ndarray, v: np.ndarray,
                   w: Optional[np.ndarray] = None) -> CSRGraph:
    """Symmetric CSR from a list of undirected edges with u != v and no repeats."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    if u.size and (np.any(u == v) or u.min() < 0 or v.min() < 0 or max(u.max(), v.max()) >= n):
        raise ValueError("edges must join two distinct nodes in [0, n)")
    src = np.concatenate([u, v])
    dst = np.concatenate([v, u])
    order = np.lexsort((dst, src))
    src = src[order]
    dst = dst[order]
    if src.size > 1:
        dup = (src[1:] == src[:-1]) & (dst[1:] == dst[:-1])
        if np.any(dup):
            raise ValueError("repeated edge")
    if src.size >= 2 ** 31:
        raise ValueError("nnz does not fit int32 indexing")
    counts = np.bincount(src, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    weight = None
    if w is not None:
        w = np.asarray(w, dtype=np.float32)
        weight = np.concatenate([w, w])[order].astype(np.float32)
    return CSRGraph(n, row_ptr.astype(np.int32), dst.astype(np.int32), weight)


def random_permutation_graph(n: int, d: int, seed: int) -> CSRGraph:
    """Near-d-regular random graph for very large n (d even): the union of d/2
    uniformly random permutations, each contributing the edges {i, pi(i)}, with
    self-loops and repeated edges dropped (an O(d^2 / n) fraction of each node's
    edges in expectation).  Fully vectorised, so graphs of millions of nodes take
    seconds; used for size sweeps where the exact-regular generator is too slow."""
    if d % 2:
        raise ValueError("d must be even")
    rng = np.random.default_rng(seed)
    us, vs = [], []
    for _ in range(d // 2):
        pi = rng.permutation(n)
        us.append(np.arange(n, dtype=np.int64))
        vs.append(pi.astype(np.int64))
    u = np.concatenate(us)
    v = np.concatenate(vs)
    keep = u != v
    a = np.minimum(u[keep], v[keep])
    b = np.maximum(u[keep], v[keep])
    key = np.unique(a * n + b)
    lo, hi = key // n, key % n
    both = np.sort(np.concatenate([lo * n + hi, hi * n + lo]))  # (row, col) order
    src, dst = both // n, both % n
    if src.size >= 2 ** 31:
        raise ValueError("nnz does not fit int32 indexing")
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(src, minlength=n), out=row_ptr[1:])
    return CSRGraph(n, row_ptr.astype(np.int32), dst.astype(np.int32), None)


def random_regular_graph(n: int, d: int, seed: int) -> CSRGraph:
    """Uniform-ish random d-regular simple graph on n nodes (pairing + switchings)."""
    if d < 0 or d >= n or (n * d) % 2:
        raise ValueError("need 0 <= d < n and n*d even")
    rng = np.random.Generator(np.random.PCG64(seed))
    if d == 0:
        return csr_from_edges(n, np.zeros(0, np.int64), np.zeros(0, np.int64))
    stubs = np.repeat(np.arange(n, dtype=np.int64), d)
    perm = rng.permutation(stubs.size)
    pairs = stubs[perm].reshape(-1, 2)
    a = np.minimum(pairs[:, 0], pairs[:, 1])
    b = np.maximum(pairs[:, 0], pairs[:, 1])
    m = a.size
    key = a * n + b
    # Mark defects: self loops, and every copy after the first of a repeated pair.
    order = np.argsort(key, kind="stable")
    sk = key[order]
    repeat = np.zeros(m, dtype=bool)
    repeat[order[1:][sk[1:] == sk[:-1]]] = True
    bad = (a == b) | repeat
    present = {}
    for e in np.nonzero(~bad)[0]:
        present[int(key[e])] = int(e)
    bad_list: List[int] = [int(e) for e in np.nonzero(bad)[0]]
    good = np.ones(m, dtype=bool)
    good[bad] = False
    attempts = 0
    max_attempts = 1000 * (len(bad_list) + 10)
    while bad_list:
        attempts += 1
        if attempts > max_attempts:
            raise RuntimeError("switching repair did not converge")
        e = bad_list[-1]
        f = int(rng.integers(m))
        if f == e or not good[f]:
            continue
        x, y = int(a[e]), int(b[e])
        p, q = int(a[f]), int(b[f])
        if rng.integers(2):
            p, q = q, p
        # Switch {x,y},{p,q} -> {x,p},{y,q}
        if x == p or y == q:
            continue
        k1 = min(x, p) * n + max(x, p)
        k2 = min(y, q) * n + max(y, q)
        if k1 == k2 or k1 in present or k2 in present:
            continue
        del present[int(key[f])]
        a[e], b[e] = min(x, p), max(x, p)
        a[f], b[f] = min(y, q), max(y, q)
        key[e], key[f] = k1, k2
        present[k1] = e
        present[k2] = f
        good[e] = True
        bad_list.pop()
    # Random relabelling so that node order carries no structure.
    relabel = rng.permutation(n)
    g = csr_from_edges(n, relabel[a], relabel[b])
    deg = g.degrees()
    assert np.all(deg == d)
    return g


def erdos_renyi_graph(n: int, p: float, seed: int) -> CSRGraph:
    """G(n, p) by geometric skipping over the upper-triangular pair index."""
    if not (0.0 <= p <= 1.0):
        raise ValueError("p must lie in [0, 1]")
    rng = np.random.Generator(np.random.PCG64(seed))
    total = n * (n - 1) // 2
    if p == 0.0 or total == 0:
        return csr_from_edges(n, np.zeros(0, np.int64), np.zeros(0, np.int64))
    if p == 1.0:
        idx = np.arange(total, dtype=np.int64)
    else:
        chunks = []
        pos = -1
        expect = int(total * p + 10 * np.sqrt(total * p + 1) + 16)
        while True:
            skips = rng.geometric(p, size=max(expect, 1024)).astype(np.int64)
            cs = pos + np.cumsum(skips)
            cs = cs[cs < total]
            chunks.append(cs)
            if cs.size < skips.size:
                break
            pos = int(cs[-1])
        idx = np.concatenate(chunks)
    # Pair index k -> (i, j), i < j, enumerating row i's pairs (i, i+1..n-1) in order.
    # Row i starts at off(i) = i*(2n - i - 1)/2.
    i = np.floor(((2 * n - 1) - np.sqrt((2 * n - 1) ** 2 - 8.0 * idx)) / 2).astype(np.int64)
    off = i * (2 * n - i - 1) // 2
    # Repair floating point rounding of the square root at row boundaries.
    low = idx < off
    while np.any(low):
        i[low] -= 1
        off = i * (2 * n - i - 1) // 2
        low = idx < off
    nxt = (i + 1) * (2 * n - i - 2) // 2
    high = idx >= nxt
    while np.any(high):
        i[high] += 1
        off = i * (2 * n - i - 1) // 2
        nxt = (i + 1) * (2 * n - i - 2) // 2
        high = idx >= nxt
    j = idx - off + i + 1
    return csr_from_edges(n, i, j)


def disjoint_union(graphs: Sequence[CSRGraph]) -> CSRGraph:
    """Block-diagonal union; ``graph_ptr`` records each member's node offset."""
    n_tot = int(sum(g.n for g in graphs))
    nnz_tot = int(sum(g.nnz for g in graphs))
    if nnz_tot >= 2 ** 31 or n_tot >= 2 ** 31:
        raise ValueError("union too large for int32 indexing")
    row_ptr = np.zeros(n_tot + 1, dtype=np.int64)
    col_idx = np.empty(nnz_tot, dtype=np.int32)
    graph_ptr = np.zeros(len(graphs) + 1, dtype=np.int32)
    weighted = any(g.weight is not None for g in graphs)
    weight = np.empty(nnz_tot, dtype=np.float32) if weighted else None
    node_off = 0
    nz_off = 0
    for k, g in enumerate(graphs):
        row_ptr[node_off + 1: node_off + g.n + 1] = nz_off + g.row_ptr[1:].astype(np.int64)
        col_idx[nz_off: nz_off + g.nnz] = g.col_idx + node_off
        if weighted:
            weight[nz_off: nz_off + g.nnz] = 1.0 if g.weight is None else g.weight
        node_off += g.n
        nz_off += g.nnz
        graph_ptr[k + 1] = node_off
    return CSRGraph(n_tot, row_ptr.astype(np.int32), col_idx, weight, graph_ptr)


def bfs_ball(g: CSRGraph, size: int, root: int = 0) -> np.ndarray:
    """The first ``size`` nodes reached by breadth-first search from ``root``."""
    seen = np.zeros(g.n, dtype=bool)
    order = [root]
    seen[root] = True
    head = 0
    while head < len(order) and len(order) < size:
        v = order[head]
        head += 1
        for u in g.col_idx[g.row_ptr[v]: g.row_ptr[v + 1]]:
            if not seen[u]:
                seen[u] = True
                order.append(int(u))
                if len(order) >= size:
                    break
    return np.array(order[:size], dtype=np.int64)


def induced_subgraph(g: CSRGraph, nodes: np.ndarray) -> CSRGraph:
    """Subgraph induced by ``nodes``, relabelled 0..len(nodes)-1 in the given order."""
    nodes = np.asarray(nodes, dtype=np.int64)
    remap = -np.ones(g.n, dtype=np.int64)
    remap[nodes] = np.arange(nodes.size)
    u, v, w = g.edge_list()
    keep = (remap[u] >= 0) & (remap[v] >= 0)
    return csr_from_edges(nodes.size, remap[u[keep]], remap[v[keep]],
                          None if w is None else w[keep])


def instance_edge_weights(g: CSRGraph, S: int, seed: int, kind: str = "uniform",
                          drop: float = 0.0) -> np.ndarray:
    """S weighted instances on the pattern of g, one per head: float32 [nnz, S],
    symmetric (both CSR entries of an edge carry the same S values).

    kind: "uniform" U(0.5, 1.5), "signed" +-1 with equal odds (Gset-style
    couplings), "integer" U{1, ..., 4}, "unit" 1 (with drop: an edge subset per
    head).  drop: fraction of (edge, head) pairs set to 0, i.e. the edge is
    absent from that head's instance."""
    rng = np.random.default_rng(seed)
    n = g.n
    rows = np.repeat(np.arange(n, dtype=np.int64), g.degrees())
    cols = g.col_idx.astype(np.int64)
    upper = rows < cols
    E = int(upper.sum())
    if kind == "uniform":
        vals = rng.uniform(0.5, 1.5, (E, S))
    elif kind == "signed":
        vals = np.where(rng.random((E, S)) < 0.5, -1.0, 1.0)
    elif kind == "integer":
        vals = rng.integers(1, 5, (E, S)).astype(np.float64)
    elif kind == "unit":
        vals = np.ones((E, S))
    else:
        raise ValueError(kind)
    if drop > 0:
        vals[rng.random((E, S)) < drop] = 0.0
    # edge id of every CSR entry: its position among the upper entries (i < j)
    keys = rows[upper] * n + cols[upper]
    lo = np.minimum(rows, cols)
    hi = np.maximum(rows, cols)
    eid = np.searchsorted(keys, lo * n + hi)
    return vals[eid].astype(np.float32)
