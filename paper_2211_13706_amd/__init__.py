"""posetx: fast zeta and Möbius transforms on posets for MI355X (gfx950).

The transforms of Pegolotti, Seifert and Püschel ("Fast Möbius and Zeta
Transforms") computed through a chain decomposition and the niv map, with
hand-written HIP kernels behind a C ABI (include/posetx.h, libposetx.so).

    import paper_2211_13706_amd as px
    P = px.poset_build(n, indptr, indices)        # one-time preprocessing
    g = px.zeta(P, f)                             # g = Z f
    f2 = px.mobius(P, g)                          # f = M g
    w2 = px.zeta_adjoint(P, w)                    # Z^T w
"""

from ._lib import (PX_BUILD_HOST_ONLY, PX_BUILD_LEVELS_MIRSKY, PX_BUILD_MIN_CHAINS, PX_BUILD_NO_ADJOINT,
                   PX_BUILD_SPARSE_NIV, PX_F32, PX_F64, PX_I64, PosetxError, lib)
from .poset import (Batch, Poset, batch_build, mobius, mobius_adjoint, poset_build, poset_build_many, poset_load,
                    zeta, zeta_adjoint, zeta_adjoint_batched, zeta_batched, zeta_noalloc)

__all__ = [
    "Poset", "Batch", "PosetxError", "poset_build", "poset_build_many", "poset_load", "batch_build", "zeta",
    "zeta_adjoint", "mobius", "mobius_adjoint", "zeta_batched", "zeta_adjoint_batched", "zeta_noalloc", "lib",
    "PX_I64", "PX_F32", "PX_F64", "PX_BUILD_HOST_ONLY", "PX_BUILD_NO_ADJOINT", "PX_BUILD_LEVELS_MIRSKY",
    "PX_BUILD_SPARSE_NIV", "PX_BUILD_MIN_CHAINS",
]
