"""Zeta and its adjoint at chosen nodes of posets too large for a closure matrix.

Oracle / test infrastructure only (see the package docstring).  For a node
x, the down-set out(x) = {y : y ⪯ x} is found by breadth-first search along
the child edges (the definition of reachability, §2.1); then
g(x) = Σ_{y ∈ out(x)} f(y) (Theorem 1).  The adjoint searches along the
reversed edges for the up-set {y : y ⪰ x}.
"""

from __future__ import annotations

import numpy as np
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import breadth_first_order


def _graph(n, indptr, indices, reverse=False):
    data = np.ones(len(indices), dtype=np.int8)
    G = csr_matrix((data, np.asarray(indices, np.int64), np.asarray(indptr, np.int64)), shape=(n, n))
    return G.T.tocsr() if reverse else G


def _sum_rows(f, rows):
    """Σ over the given rows, per column.

    int: modulo 2**64 via uint64.  float: float64 pairwise summation over a
    contiguous axis, error ≤ ~log2(m)·2**-53·Σ|f| for m rows.
    """
    if f.dtype in (np.int64, np.int32):
        return f[rows].astype(np.int64).view(np.uint64).sum(axis=0, dtype=np.uint64).view(np.int64)
    sub = np.ascontiguousarray(f[rows].astype(np.float64).T)
    return sub.sum(axis=1)


def _at(n, indptr, indices, f, nodes, reverse):
    G = _graph(n, indptr, indices, reverse)
    f = np.asarray(f)
    out = []
    for x in nodes:
        rows = breadth_first_order(G, int(x), directed=True, return_predecessors=False)
        out.append(_sum_rows(f, np.sort(rows)))
    return np.stack(out) if out else np.zeros((0, f.shape[1]), f.dtype)


def zeta_at(n, indptr, indices, f, nodes):
    """g(x) = Σ_{y ⪯ x} f(y) for each x in ``nodes``; returns [len(nodes), B]."""
    return _at(n, indptr, indices, f, nodes, reverse=False)


def zeta_adjoint_at(n, indptr, indices, w, nodes):
    """(Z^T w)(y) = Σ_{x ⪰ y} w(x) for each y in ``nodes``."""
    return _at(n, indptr, indices, w, nodes, reverse=True)
