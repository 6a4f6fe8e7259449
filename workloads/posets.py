"""Seeded synthetic posets and function matrices.

Every input that the oracle, the tests and the benchmark use is drawn here,
from a seed, so that the CPU oracle and the GPU library see identical data.
This module holds none of the transform arithmetic: it only draws DAGs (as
CSR child lists), optional planted chain decompositions, and random function
matrices.

Conventions (paper §2.1): an edge u -> v means v is below u (v precedes u in
the partial order); ``indices[indptr[u]:indptr[u+1]]`` are the children of u.
A planted chain decomposition (Definition 1, §2.3) is given as
``chain_of[node]`` and ``chain_pos[node]``, position 0 being the minimal
element of the chain.

Recipes:

* ``chain_poset``: the random-height workload.  A seeded permutation ``t``
  gives every node a height rank.  Node ids are split into ``k`` contiguous
  blocks (``np.array_split``); each block, sorted by ``t``, is a chain, and
  every chain element has an edge to the element just below it.  Every node
  also gets ``cross`` distinct edges to nodes of *other* chains with lower
  height, drawn uniformly without replacement (fewer when fewer exist).
* ``er_dag``: the paper's experimental workload (§5): Erdős–Rényi edges over
  a random topological order, average out-degree ``deg``.
* ``grid_poset``: the product of two chains, node (i, j) = i*w + j, edges
  (i,j)->(i-1,j) and (i,j)->(i,j-1); planted chains are the columns j.
* ``boolean_lattice``: subsets of {0..m-1} ordered by inclusion, cover edges
  S -> S minus one element.
* ``chain_only`` / ``antichain``: a total order and an edgeless poset.
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "Poset",
    "chain_poset",
    "er_dag",
    "grid_poset",
    "boolean_lattice",
    "chain_only",
    "antichain",
    "random_small_dag",
    "batched_posets",
    "functions",
    "worked_example",
]


class Poset:
    """A DAG as CSR child lists plus an optional planted chain decomposition."""

    def __init__(self, n, indptr, indices, chain_of=None, chain_pos=None, name=""):
        self.n = int(n)
        self.indptr = np.ascontiguousarray(indptr, dtype=np.int64)
        self.indices = np.ascontiguousarray(indices, dtype=np.int32)
        self.chain_of = None if chain_of is None else np.ascontiguousarray(chain_of, dtype=np.int32)
        self.chain_pos = None if chain_pos is None else np.ascontiguousarray(chain_pos, dtype=np.int32)
        self.name = name
        assert self.indptr.shape == (self.n + 1,)
        assert self.indptr[-1] == self.indices.shape[0]

    @property
    def nedges(self) -> int:
        return int(self.indices.shape[0])

    @property
    def k_planted(self):
        return None if self.chain_of is None else int(self.chain_of.max()) + 1 if self.n else 0

    def edges(self):
        """(src, dst) arrays of all edges."""
        src = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.indptr))
        return src, self.indices.astype(np.int64)

    def __repr__(self):
        return f"Poset({self.name!r}, n={self.n}, edges={self.nedges})"


def _csr_from_lists(n, src, dst):
    """CSR child lists from edge arrays, edges of one source kept in input order."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    order = np.argsort(src, kind="stable")
    counts = np.bincount(src, minlength=n)
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=indptr[1:])
    return indptr, dst[order].astype(np.int32)


def chain_poset(n: int, k: int, cross: int, seed: int) -> Poset:
    """Random-height poset with ``k`` planted chains and ``cross`` cross edges per node."""
    rng = np.random.default_rng(seed)
    t = rng.permutation(n).astype(np.int64)          # height rank of each node
    chain_of = np.empty(n, dtype=np.int32)
    chain_pos = np.empty(n, dtype=np.int32)
    src_l, dst_l = [], []
    for c, ids in enumerate(np.array_split(np.arange(n, dtype=np.int64), k)):
        order = ids[np.argsort(t[ids], kind="stable")]   # bottom first
        chain_of[order] = c
        chain_pos[order] = np.arange(order.size, dtype=np.int32)
        if order.size > 1:
            src_l.append(order[1:])
            dst_l.append(order[:-1])
    by_height = np.argsort(t, kind="stable")             # node at each height
    # number of lower nodes that lie on other chains
    eligible = t - chain_pos.astype(np.int64)
    want = np.minimum(eligible, cross)
    # nodes that must take every eligible node
    few = np.nonzero((eligible <= cross) & (eligible > 0))[0]
    for u in few:
        lower = by_height[: t[u]]
        lower = lower[chain_of[lower] != chain_of[u]]
        src_l.append(np.full(lower.size, u, dtype=np.int64))
        dst_l.append(lower)
    many = np.nonzero(eligible > cross)[0]
    if many.size and cross > 0:
        picks = np.full((many.size, cross), -1, dtype=np.int64)
        hu = t[many]
        cu = chain_of[many]
        todo = np.ones((many.size, cross), dtype=bool)
        for _ in range(10000):
            rows, cols = np.nonzero(todo)
            if rows.size == 0:
                break
            cand = by_height[(rng.random(rows.size) * hu[rows]).astype(np.int64)]
            picks[rows, cols] = cand
            bad = chain_of[cand] == cu[rows]
            # duplicates inside a row: keep the first occurrence
            srt = np.sort(picks, axis=1)
            dup_rows = np.nonzero((srt[:, 1:] == srt[:, :-1]).any(axis=1))[0]
            todo[:] = False
            todo[rows[bad], cols[bad]] = True
            for r in dup_rows:
                seen = set()
                for j in range(cross):
                    v = picks[r, j]
                    if v in seen:
                        todo[r, j] = True
                    elif v >= 0 and not todo[r, j]:
                        seen.add(v)
        else:  # pragma: no cover - the loop always converges for eligible > cross
            raise RuntimeError("cross-edge sampling did not converge")
        src_l.append(np.repeat(many, cross))
        dst_l.append(picks.reshape(-1))
    src = np.concatenate(src_l) if src_l else np.zeros(0, np.int64)
    dst = np.concatenate(dst_l) if dst_l else np.zeros(0, np.int64)
    assert int(want.sum()) + (n - k if n >= k else 0) == src.size
    indptr, indices = _csr_from_lists(n, src, dst)
    return Poset(n, indptr, indices, chain_of, chain_pos, name=f"chain_poset(n={n},k={k},cross={cross},seed={seed})")


def er_dag(n: int, deg: float, seed: int) -> Poset:
    """Erdős–Rényi DAG over a random topological order, average out-degree ``deg`` (§5)."""
    rng = np.random.default_rng(seed)
    order = rng.permutation(n).astype(np.int64)       # order[h] = node at height h
    m = int(round(deg * n))
    a = rng.integers(0, n, size=2 * m + 16)
    b = rng.integers(0, n, size=2 * m + 16)
    keep = a != b
    a, b = a[keep], b[keep]
    hi, lo = np.maximum(a, b), np.minimum(a, b)
    key = np.unique(hi * n + lo)
    key = rng.permutation(key)[:m]
    hi, lo = key // n, key % n
    src, dst = order[hi], order[lo]
    indptr, indices = _csr_from_lists(n, src, dst)
    return Poset(n, indptr, indices, name=f"er_dag(n={n},deg={deg},seed={seed})")


def grid_poset(h: int, w: int) -> Poset:
    """Product of a chain of length ``h`` and one of length ``w``; chains are the columns."""
    n = h * w
    i, j = np.divmod(np.arange(n, dtype=np.int64), w)
    src_l, dst_l = [], []
    m = i > 0
    src_l.append(np.nonzero(m)[0]); dst_l.append(np.nonzero(m)[0] - w)
    m = j > 0
    src_l.append(np.nonzero(m)[0]); dst_l.append(np.nonzero(m)[0] - 1)
    indptr, indices = _csr_from_lists(n, np.concatenate(src_l), np.concatenate(dst_l))
    return Poset(n, indptr, indices, chain_of=j.astype(np.int32), chain_pos=i.astype(np.int32),
                 name=f"grid({h}x{w})")


def boolean_lattice(m: int) -> Poset:
    """All subsets of an m-set (bitmasks) with cover edges S -> S minus {e}."""
    n = 1 << m
    src_l, dst_l = [], []
    s = np.arange(n, dtype=np.int64)
    for e in range(m):
        has = (s >> e) & 1 == 1
        src_l.append(s[has]); dst_l.append(s[has] ^ (1 << e))
    indptr, indices = _csr_from_lists(n, np.concatenate(src_l), np.concatenate(dst_l))
    return Poset(n, indptr, indices, name=f"boolean_lattice(2^{m})")


def chain_only(n: int, seed: int | None = None) -> Poset:
    """A total order; with a seed the node ids are shuffled along the chain."""
    perm = np.arange(n, dtype=np.int64) if seed is None else np.random.default_rng(seed).permutation(n)
    # perm[p] = node at position p (bottom first)
    indptr, indices = _csr_from_lists(n, perm[1:], perm[:-1])
    pos = np.empty(n, dtype=np.int32); pos[perm] = np.arange(n, dtype=np.int32)
    return Poset(n, indptr, indices, chain_of=np.zeros(n, np.int32), chain_pos=pos,
                 name=f"chain({n})")


def antichain(n: int) -> Poset:
    return Poset(n, np.zeros(n + 1, np.int64), np.zeros(0, np.int32), name=f"antichain({n})")


def random_small_dag(n: int, p: float, seed: int) -> Poset:
    """Dense-ish random DAG for brute-force property tests (n up to a few hundred)."""
    rng = np.random.default_rng(seed)
    order = rng.permutation(n)
    a = rng.random((n, n)) < p
    hi, lo = np.nonzero(np.triu(a, 1).T)   # hi > lo in height
    src, dst = order[hi], order[lo]
    indptr, indices = _csr_from_lists(n, src, dst)
    return Poset(n, indptr, indices, name=f"random_small_dag(n={n},p={p},seed={seed})")


def batched_posets(count: int, seed: int, nmin=1000, nmax=65536, ks=tuple(range(4, 129, 4)),
                   deg=(2, 5)):
    """Many posets of uneven size: n log-uniform in [nmin, nmax], k from ``ks``, cross degree in ``deg``."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(np.floor(np.exp(rng.uniform(np.log(nmin), np.log(nmax)))))
        k = int(rng.choice(ks))
        k = min(k, n)
        d = int(rng.integers(deg[0], deg[1] + 1))
        out.append(chain_poset(n, k, d, seed=int(rng.integers(0, 2**31 - 1))))
    return out


def functions(n: int, B: int, kind: str, seed: int, lo=None, hi=None):
    """A seeded [n, B] function matrix (row = node, column = right-hand side).

    kind: 'normal' (float32 N(0,1)), 'normal64' (float64 N(0,1)),
    'uniform' (float32 U(lo, hi)), 'int' (int64 uniform in [lo, hi]).
    """
    rng = np.random.default_rng(seed)
    if kind == "normal":
        return rng.standard_normal((n, B), dtype=np.float32)
    if kind == "normal64":
        return rng.standard_normal((n, B))
    if kind == "uniform":
        return rng.uniform(lo, hi, size=(n, B)).astype(np.float32)
    if kind == "int":
        return rng.integers(lo, hi + 1, size=(n, B), dtype=np.int64)
    raise ValueError(kind)


def worked_example() -> Poset:
    """The 12-element cover graph of the paper's running example (§2.2), 0-based ids.

    Node i here is the paper's x_{i+1}; the planted chains are the four chains
    of the example's decomposition (§2.3), read from the niv matrix N (§2.4).
    """
    children = {1: [3, 4, 6], 2: [4, 5], 3: [7, 8], 4: [7, 9], 5: [10], 6: [8, 9],
                7: [10], 8: [11], 9: [12], 10: [11, 12], 11: [], 12: []}
    src, dst = [], []
    for u, vs in children.items():
        for v in vs:
            src.append(u - 1); dst.append(v - 1)
    chains = [[12, 9, 4, 2], [7, 3, 1], [10, 5], [11, 8, 6]]   # bottom first, 1-based
    chain_of = np.empty(12, np.int32); chain_pos = np.empty(12, np.int32)
    for c, ch in enumerate(chains):
        for p, x in enumerate(ch):
            chain_of[x - 1] = c; chain_pos[x - 1] = p
    indptr, indices = _csr_from_lists(12, src, dst)
    return Poset(12, indptr, indices, chain_of, chain_pos, name="worked_example")
