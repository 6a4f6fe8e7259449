"""Reachability of a DAG by brute force, and maps defined from it.

Oracle / test infrastructure only (see the package docstring).
"""

from __future__ import annotations

import numpy as np


def _adjacency(n, indptr, indices):
    A = np.zeros((n, n), dtype=np.float64)
    src = np.repeat(np.arange(n), np.diff(np.asarray(indptr)))
    A[src, np.asarray(indices, dtype=np.int64)] = 1.0
    return A


def reachability(n, indptr, indices) -> np.ndarray:
    """R[x, y] = True iff y ⪯ x, i.e. y = x or y is reachable from x (§2.1).

    Brute force: start from R = I ∨ A (paths of length ≤ 1) and square until
    nothing changes; after t squarings R holds every path of length ≤ 2**t.
    The products are float64 counts, exact below 2**53.  R is then the
    adjacency matrix Z of the transitive closure (Corollary 1, §2.2).
    """
    if n == 0:
        return np.zeros((0, 0), dtype=bool)
    R = (_adjacency(n, indptr, indices) + np.eye(n)) > 0
    while True:
        Rf = R.astype(np.float64)
        nxt = R | ((Rf @ Rf) > 0)
        if np.array_equal(nxt, R):
            return R
        R = nxt


def is_acyclic(R: np.ndarray) -> bool:
    """A relation from a DAG is antisymmetric: x ⪯ y and y ⪯ x imply x = y (§2.1)."""
    both = R & R.T
    np.fill_diagonal(both, False)
    return not both.any()


def linear_extension(R: np.ndarray) -> np.ndarray:
    """Nodes ordered bottom-up: y ≺ x means down(y) ⊊ down(x), so |down(y)| < |down(x)|."""
    return np.argsort(R.sum(axis=1), kind="stable")


def niv_from_closure(R: np.ndarray, chain_of, chain_pos, k: int) -> np.ndarray:
    """niv_j(x) = the highest element of chain j below x (§2.4), by its definition.

    Returns node ids, -1 where no element of chain j lies below x (the
    paper's ∞).  "Highest" is the element of largest chain position in
    out(x) ∩ Z_j; the paper's topological numbering makes that the smallest
    index, which the printed matrix N of the worked example confirms.
    """
    n = R.shape[0]
    chain_of = np.asarray(chain_of); chain_pos = np.asarray(chain_pos)
    out = np.full((n, k), -1, dtype=np.int64)
    for x in range(n):
        below = np.nonzero(R[x])[0]
        for j in range(k):
            cand = below[chain_of[below] == j]
            if cand.size:
                out[x, j] = cand[np.argmax(chain_pos[cand])]
    return out


def mirsky_levels(R: np.ndarray) -> np.ndarray:
    """Level of x = number of elements on a longest chain ending at x, minus one.

    Minimal elements get level 0; the number of levels equals the length of
    the longest chain (Mirsky's theorem, §4).  Computed from the closure:
    level(x) = 1 + max level over the elements strictly below x.
    """
    n = R.shape[0]
    lev = np.zeros(n, dtype=np.int64)
    for x in linear_extension(R):
        below = np.nonzero(R[x])[0]
        below = below[below != x]
        lev[x] = 0 if below.size == 0 else 1 + lev[below].max()
    return lev


def width(R: np.ndarray) -> int:
    """The width of the poset: the size of its largest antichain, which equals the
    fewest chains that partition it (Dilworth; Theorem 2, §2.3).

    Computed from the equivalent matching form (Fulkerson): a chain partition
    with m links (x directly above y in its chain) has n - m chains, and the
    links of chains are a matching of the bipartite graph with an edge (x, y)
    for every strict comparability y ≺ x; so the fewest chains are n minus a
    maximum matching of that graph (König), found by scipy's maximum bipartite
    matching on the closure.
    """
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import maximum_bipartite_matching
    n = R.shape[0]
    if n == 0:
        return 0
    strict = R.copy()
    np.fill_diagonal(strict, False)
    match = maximum_bipartite_matching(csr_matrix(strict.astype(np.int8)), perm_type="column")
    return int(n - np.count_nonzero(match >= 0))
