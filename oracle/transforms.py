"""Zeta and Möbius transforms straight from their definitions (§2.2).

Oracle / test infrastructure only (see the package docstring).  Every
function takes the closure R from ``oracle.closure.reachability``:
R[x, y] = True iff y ⪯ x, which is the zeta matrix Z of Corollary 1.
Function matrices are [n, B]: row = poset element, column = right-hand side.
"""

from __future__ import annotations

import math

import numpy as np

_INT = (np.int64, np.int32, np.uint64)


def _is_int(a) -> bool:
    return np.asarray(a).dtype in _INT


def _wrap_matmul(Z: np.ndarray, f: np.ndarray) -> np.ndarray:
    """Z @ f modulo 2**64 (uint64 arithmetic wraps), returned as int64."""
    out = Z.astype(np.uint64) @ np.asarray(f).astype(np.int64).view(np.uint64)
    return out.view(np.int64)


def _fsum_matmul(W: np.ndarray, f: np.ndarray) -> np.ndarray:
    """out[x, b] = fsum_y W[x, y] * f[y, b] over the nonzeros of row x (float64)."""
    f = np.asarray(f, dtype=np.float64)
    n, B = W.shape[0], f.shape[1]
    out = np.empty((n, B), dtype=np.float64)
    for x in range(n):
        idx = np.nonzero(W[x])[0]
        w = W[x, idx].astype(np.float64)
        for b in range(B):
            out[x, b] = math.fsum(w * f[idx, b])
    return out


def zeta(R: np.ndarray, f: np.ndarray, exact: bool = True) -> np.ndarray:
    """g(x) = Σ_{y ⪯ x} f(y), i.e. g = Z f (Theorem 1, Corollary 1).

    int inputs: exact modulo 2**64.  Float inputs: float64 result, the
    correctly rounded exact sum when ``exact`` (math.fsum), else a float64
    product with error ≤ n·2**-53·Σ|f|.
    """
    if _is_int(f):
        return _wrap_matmul(R, f)
    if exact:
        return _fsum_matmul(R, f)
    return R.astype(np.float64) @ np.asarray(f, dtype=np.float64)


def zeta_adjoint(R: np.ndarray, w: np.ndarray, exact: bool = True) -> np.ndarray:
    """(Z^T w)(y) = Σ_{x ⪰ y} w(x): the transpose of the zeta matrix applied to w."""
    return zeta(np.ascontiguousarray(R.T), w, exact=exact)


def mobius_function(R: np.ndarray) -> np.ndarray:
    """mu[x, y] = μ(x, y) by the recursion of Theorem 1.

    μ(x, x) = 1 and μ(x, y) = -Σ_{x ⪯ z ≺ y} μ(x, z) for x ≠ y.  Columns are
    filled for y in a bottom-up linear extension, so every μ(x, z) with
    z ≺ y is known when column y is formed.  Entries with x ⋠ z stay 0, so
    summing column entries over all z ≺ y sums exactly over x ⪯ z ≺ y.
    """
    n = R.shape[0]
    mu = np.zeros((n, n), dtype=np.int64)
    from .closure import linear_extension
    for y in linear_extension(R):
        strictly_below = R[y].copy()
        strictly_below[y] = False
        col = -mu[:, strictly_below].sum(axis=1)
        col[y] += 1
        mu[:, y] = col
    assert np.abs(mu).max(initial=0) < 2**62
    return mu


def mobius_matrix(R: np.ndarray, mu: np.ndarray | None = None) -> np.ndarray:
    """M = [μ(y, x)]_{x, y} of Corollary 1, so that f = M g inverts g = Z f."""
    if mu is None:
        mu = mobius_function(R)
    return np.ascontiguousarray(mu.T)


def mobius(R: np.ndarray, g: np.ndarray, mu: np.ndarray | None = None, exact: bool = True) -> np.ndarray:
    """f(x) = Σ_{y ⪯ x} μ(y, x) g(y) (Theorem 1).

    int inputs: exact modulo 2**64.  Float inputs with ``exact``: each term
    μ·g is formed in float64 (exact when g has ≤ 24 significant bits, as
    float32 data does, and |μ| < 2**29) and summed with math.fsum.
    """
    M = mobius_matrix(R, mu)
    if _is_int(g):
        return _wrap_matmul(M, g)
    if exact:
        return _fsum_matmul(M, g)
    return M.astype(np.float64) @ np.asarray(g, dtype=np.float64)


def mobius_adjoint(R: np.ndarray, v: np.ndarray, mu: np.ndarray | None = None, exact: bool = True) -> np.ndarray:
    """(M^T v)(y) = Σ_{x ⪰ y} μ(y, x) v(x): the transpose of M applied to v."""
    if mu is None:
        mu = mobius_function(R)
    if _is_int(v):
        return _wrap_matmul(mu, v)
    if exact:
        return _fsum_matmul(mu, v)
    return mu.astype(np.float64) @ np.asarray(v, dtype=np.float64)


def mobius_by_substitution(R: np.ndarray, g: np.ndarray) -> np.ndarray:
    """Solve Z f = g by substitution (§2.2): f(x) = g(x) - Σ_{y ≺ x} f(y).

    Elements are visited bottom-up, so every f(y), y ≺ x, is known.  Exact
    modulo 2**64 for int input (Z is unimodular, so the solution mod 2**64
    is unique); float64 arithmetic otherwise.
    """
    from .closure import linear_extension
    integer = _is_int(g)
    f = np.asarray(g).astype(np.int64).view(np.uint64).copy() if integer else np.asarray(g, dtype=np.float64).copy()
    for x in linear_extension(R):
        below = R[x].copy(); below[x] = False
        if below.any():
            f[x] = f[x] - f[below].sum(axis=0)
    return f.view(np.int64) if integer else f


def mobius_adjoint_by_substitution(R: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Solve Z^T h = v top-down: h(y) = v(y) - Σ_{x ≻ y} h(x)."""
    return mobius_by_substitution(np.ascontiguousarray(R.T), v)
