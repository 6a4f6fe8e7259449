"""Reference oracle for the poset zeta / Möbius transforms — TEST INFRASTRUCTURE ONLY.

This package is a plain, slow CPU implementation of what the fast transforms
compute, written from the definitions in the paper (Pegolotti, Seifert,
Püschel, "Fast Möbius and Zeta Transforms"):

* ``closure``   — the reachability relation (transitive closure) of a DAG by
                  brute force, and the chain maps (id, niv) read off it by
                  their definitions (§2.4); the width (Theorem 2) by matching
                  on the closure.
* ``transforms``— zeta g = Z f and its adjoint Z^T w (Corollary 1, §2.2),
                  the Möbius function by its recursion (Theorem 1), and the
                  Möbius transform both as f = M g and by substitution on
                  the unit-triangular system Z f = g (§2.2).
* ``sampled``   — zeta / adjoint at single nodes of large posets by graph
                  search over the down-set (up-set) of the node.

It shares no code with the GPU library and never imports it.  Only the
tests, the smoke check and the benchmark's CPU-baseline leg may use it; the
product path must never route through it.

Arithmetic conventions:
  int64  — two's-complement wrap-around (exact modulo 2**64), computed with
           uint64 numpy arithmetic, which wraps by definition.
  float  — inputs are converted to float64; ``exact=True`` sums with
           ``math.fsum`` (correctly rounded exact sum), otherwise float64
           matrix products whose error is bounded by n * 2**-53 * sum|f|.

Parity pins: every function here is checked in ``tests/test_oracle_*.py``
against the paper's worked example (§2.2-§3), closed forms (chain, antichain,
Boolean lattice, grid) and brute-force invariants; see each docstring.
"""

from .closure import reachability, is_acyclic, linear_extension, niv_from_closure, mirsky_levels, width
from .transforms import (zeta, zeta_adjoint, mobius_function, mobius_matrix, mobius,
                         mobius_adjoint, mobius_by_substitution, mobius_adjoint_by_substitution)
from .sampled import zeta_at, zeta_adjoint_at

__all__ = [
    "reachability", "is_acyclic", "linear_extension", "niv_from_closure", "mirsky_levels", "width",
    "zeta", "zeta_adjoint", "mobius_function", "mobius_matrix", "mobius", "mobius_adjoint",
    "mobius_by_substitution", "mobius_adjoint_by_substitution", "zeta_at", "zeta_adjoint_at",
]
