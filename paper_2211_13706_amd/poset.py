"""Python binding of the posetx C ABI: poset handles and the four transforms.

Function matrices are torch tensors on the poset's GPU, shape [n, B] with
unit column stride (rows may be padded: the row stride is passed as the
leading dimension).  PyTorch only provides device memory and the current
stream; all computation runs in libposetx.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

from . import _lib

_DTYPES = None


def _dtype_code(t) -> int:
    global _DTYPES
    import torch
    if _DTYPES is None:
        _DTYPES = {torch.int64: _lib.PX_I64, torch.float32: _lib.PX_F32, torch.float64: _lib.PX_F64}
    try:
        return _DTYPES[t.dtype]
    except KeyError:
        raise TypeError(f"unsupported dtype {t.dtype}; use int64, float32 or float64") from None


def _as_matrix(t, name, device=None):
    """t as a 2-D GPU matrix whose rows the library can address as ptr + row * ld:
    unit column stride and rows that do not overlap.  Other views (transposes,
    broadcasts such as expand(n, B) with row stride 0) are copied."""
    if t.dim() == 1:
        t = t.unsqueeze(1)
    if t.dim() != 2:
        raise ValueError(f"{name} must be [n] or [n, B]")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor (the library has no CPU path)")
    if device is not None and t.device.index != device:
        raise ValueError(f"{name} is on {t.device}, the poset on cuda:{device}")
    if (t.shape[1] > 1 and t.stride(1) != 1) or (t.shape[0] > 1 and t.stride(0) < t.shape[1]):
        t = t.contiguous()
    return t


def _out_matrix(out, x):
    """The output matrix for input x: a new contiguous one, or the caller's `out`
    after checking that it has x's shape, dtype and device, unit column stride
    and non-overlapping rows (the library writes n rows of B elements at ld)."""
    import torch
    if out is None:
        out = torch.empty_like(x, memory_format=torch.contiguous_format)
        return out, out
    out2 = out.unsqueeze(1) if out.dim() == 1 else out
    if (out2.dim() != 2 or tuple(out2.shape) != tuple(x.shape) or out2.dtype != x.dtype
            or out2.device != x.device):
        raise ValueError(f"out must be a {tuple(x.shape)} {x.dtype} tensor on {x.device}")
    if (out2.shape[1] > 1 and out2.stride(1) != 1) or (out2.shape[0] > 1 and out2.stride(0) < out2.shape[1]):
        raise ValueError("out must have unit column stride and non-overlapping rows")
    return out, out2


def _ld(t):
    return max(int(t.stride(0)), int(t.shape[1])) if t.shape[0] > 1 else int(t.shape[1])


def _stream(t):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


class Poset:
    """A preprocessed poset on one GPU (px_poset_build)."""

    def __init__(self, handle, n, device):
        self._h = handle
        self.n = int(n)
        self.device = device
        self.info = self.info_dict()
        self.k = int(self.info["k"])

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            try:
                _lib.lib().px_poset_free(h)
            except Exception:
                pass
            self._h = None

    def free(self):
        self.__del__()

    @property
    def handle(self):
        if not self._h:
            raise ValueError("poset handle was freed")
        return self._h

    def info_dict(self) -> dict:
        info = _lib.Info()
        _lib.check(_lib.lib().px_poset_info(self.handle, ctypes.byref(info)), "px_poset_info")
        return info.as_dict()

    def chains(self):
        co = np.empty(self.n, np.int32)
        cp = np.empty(self.n, np.int32)
        _lib.check(_lib.lib().px_poset_chains(self.handle, co.ctypes.data, cp.ctypes.data), "px_poset_chains")
        return co, cp

    def save(self, path) -> None:
        """Write the preprocessing to a file (px_poset_save)."""
        _lib.check(_lib.lib().px_poset_save(self.handle, os.fsencode(path)), "px_poset_save")

    def rows(self) -> np.ndarray:
        """Chain-major row of every node (px_poset_rows)."""
        out = np.empty(self.n, np.int64)
        _lib.check(_lib.lib().px_poset_rows(self.handle, out.ctypes.data), "px_poset_rows")
        return out

    def set_layout(self, layout: str) -> None:
        """"nodes" (default): matrix row x is node x; "rows": matrix row r is chain-major row r
        (self.rows()), the order the kernels run in (px_poset_set_layout)."""
        code = {"nodes": _lib.PX_LAYOUT_NODES, "rows": _lib.PX_LAYOUT_ROWS}[layout]
        _lib.check(_lib.lib().px_poset_set_layout(self.handle, code), "px_poset_set_layout")
        self.info = self.info_dict()

    def niv(self, up: bool = False) -> np.ndarray:
        out = np.empty((self.n, self.k), np.int32)
        _lib.check(_lib.lib().px_poset_niv(self.handle, int(up), out.ctypes.data), "px_poset_niv")
        return out

    def niv_csr(self, up: bool = False):
        """The niv map by rows of its finite entries (px_poset_niv_csr): (ptr, node ids)."""
        info = self.info_dict()
        ptr = np.empty(self.n + 1, np.int64)
        nodes = np.empty(max(1, info["nnz_niv_up" if up else "nnz_niv"]), np.int32)
        _lib.check(_lib.lib().px_poset_niv_csr(self.handle, int(up), ptr.ctypes.data, nodes.ctypes.data),
                   "px_poset_niv_csr")
        return ptr, nodes[: ptr[-1]]

    def levels(self, up: bool = False) -> np.ndarray:
        out = np.empty(self.n, np.int32)
        _lib.check(_lib.lib().px_poset_levels(self.handle, int(up), out.ctypes.data), "px_poset_levels")
        return out

    # transforms as methods (the module functions with the same names)
    def zeta(self, f, out=None):
        """g = Z f."""
        return zeta(self, f, out)

    def zeta_T(self, w, out=None):
        """Z^T w."""
        return zeta_adjoint(self, w, out)

    def mobius(self, g, out=None, max_refine: int = 3, tol: float = 0.0, report: bool = False):
        """f = M g (float32: float64-residual refinement)."""
        return mobius(self, g, out, max_refine, tol, report)

    def mobius_T(self, v, out=None, max_refine: int = 3, tol: float = 0.0, report: bool = False):
        """M^T v."""
        return mobius_adjoint(self, v, out, max_refine, tol, report)

    def reserve(self, dtype, B: int):
        import torch
        code = {torch.int64: 0, torch.float32: 1, torch.float64: 2}[dtype]
        _lib.check(_lib.lib().px_reserve(self.handle, code, int(B)), "px_reserve")

    def autotune(self, dtype, B: int) -> dict:
        """Pick the gather tile shapes for this poset and B by timing them (px_autotune)."""
        import torch
        code = {torch.int64: 0, torch.float32: 1, torch.float64: 2}[dtype]
        rep = _lib.TuneReport()
        _lib.check(_lib.lib().px_autotune(self.handle, code, int(B), ctypes.byref(rep)), "px_autotune")
        self.info = self.info_dict()
        return rep.as_dict()


def poset_build(n, indptr, indices, chain_of=None, chain_pos=None, flags: int = 0, device: int = 0) -> Poset:
    """Preprocess a DAG given as CSR child lists (px_poset_build)."""
    indptr = np.ascontiguousarray(indptr, dtype=np.int64)
    indices = np.ascontiguousarray(indices, dtype=np.int32)
    if indptr.shape != (int(n) + 1,):
        raise ValueError("indptr must have n+1 entries")
    co = cp = None
    if chain_of is not None:
        co = np.ascontiguousarray(chain_of, dtype=np.int32)
        cp = np.ascontiguousarray(chain_pos, dtype=np.int32)
        if co.shape != (int(n),) or cp.shape != (int(n),):
            raise ValueError("chain_of and chain_pos must have n entries")
    h = ctypes.c_void_p()
    _lib.check(_lib.lib().px_poset_build(
        int(n), indptr.ctypes.data, indices.ctypes.data if indices.size else None,
        None if co is None else co.ctypes.data, None if cp is None else cp.ctypes.data,
        int(flags), int(device), ctypes.byref(h)), "px_poset_build")
    return Poset(h, n, device)


def poset_build_many(specs, flags: int = 0, device: int = 0, threads: int = 0):
    """Many posets preprocessed at once, e.g. for a batch: specs is a sequence of
    (n, indptr, indices, chain_of, chain_pos) tuples (chains may be None).  The builds run
    on up to `threads` host threads (0: min(16, CPUs)); px_poset_build calls are
    independent, so concurrent builds give the same handles as one after another."""
    from concurrent.futures import ThreadPoolExecutor
    specs = list(specs)
    nt = threads if threads > 0 else min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity")
                                           else (os.cpu_count() or 1))
    nt = max(1, min(nt, len(specs)))

    def one(sp):
        n, ip, ix, co, cp = sp
        return poset_build(n, ip, ix, co, cp, flags=flags, device=device)
    if nt == 1:
        return [one(sp) for sp in specs]
    with ThreadPoolExecutor(max_workers=nt) as ex:
        return list(ex.map(one, specs))


def poset_load(path, flags: int = 0, device: int = 0) -> Poset:
    """A handle from a file written by Poset.save, without preprocessing again (px_poset_load)."""
    h = ctypes.c_void_p()
    _lib.check(_lib.lib().px_poset_load(os.fsencode(path), int(flags), int(device), ctypes.byref(h)),
               "px_poset_load")
    info = _lib.Info()
    _lib.check(_lib.lib().px_poset_info(h, ctypes.byref(info)), "px_poset_info")
    return Poset(h, info.n, device)


def _transform(fn_name, P, x, out):
    x = _as_matrix(x, "input", P.device)
    if x.shape[0] != P.n:
        raise ValueError(f"input has {x.shape[0]} rows, poset has {P.n}")
    out, out2 = _out_matrix(out, x)
    code = _dtype_code(x)
    fn = getattr(_lib.lib(), fn_name)
    _lib.check(fn(P.handle, code, ctypes.c_void_p(x.data_ptr()), _ld(x), ctypes.c_void_p(out2.data_ptr()),
                  _ld(out2), int(x.shape[1]), _stream(x)), fn_name)
    return out


def zeta(P: Poset, f, out=None):
    """g = Z f (px_zeta)."""
    return _transform("px_zeta", P, f, out)


def zeta_adjoint(P: Poset, w, out=None):
    """Z^T w (px_zeta_adjoint)."""
    return _transform("px_zeta_adjoint", P, w, out)


def zeta_noalloc(P: Poset, f, out=None):
    """g = Z f through px_zeta_noalloc: the library allocates nothing (its scratch is a
    static 64 MiB device array); pass `out` to keep torch from allocating the result."""
    return _transform("px_zeta_noalloc", P, f, out)


def _mobius(fn_name, P, g, out, max_refine, tol, report):
    g = _as_matrix(g, "input", P.device)
    if g.shape[0] != P.n:
        raise ValueError(f"input has {g.shape[0]} rows, poset has {P.n}")
    out, out2 = _out_matrix(out, g)
    rep = _lib.RefineReport() if report else None
    code = _dtype_code(g)
    fn = getattr(_lib.lib(), fn_name)
    _lib.check(fn(P.handle, code, ctypes.c_void_p(g.data_ptr()), _ld(g), ctypes.c_void_p(out2.data_ptr()),
                  _ld(out2), int(g.shape[1]), int(max_refine), float(tol), _stream(g),
                  ctypes.byref(rep) if rep is not None else None), fn_name)
    return (out, rep.as_dict()) if report else out


def mobius(P: Poset, g, out=None, max_refine: int = 3, tol: float = 0.0, report: bool = False):
    """f = M g = Z^{-1} g (px_mobius).  float32 uses float64-residual refinement.

    tol > 0 stops the refinement early on the correction test; tol = 0 runs
    max_refine steps and then checks the result for NaN / Inf (PosetxError
    PX_ENONFINITE; one stream synchronisation); tol < 0 runs asynchronously
    without value checks (for graph capture).  int64 ignores tol."""
    return _mobius("px_mobius", P, g, out, max_refine, tol, report)


def mobius_adjoint(P: Poset, v, out=None, max_refine: int = 3, tol: float = 0.0, report: bool = False):
    """M^T v (px_mobius_adjoint)."""
    return _mobius("px_mobius_adjoint", P, v, out, max_refine, tol, report)


class Batch:
    """Many posets run together (px_batch_build); matrices stack the posets' rows."""

    def __init__(self, posets):
        self.posets = list(posets)
        arr = (ctypes.c_void_p * len(self.posets))(*[p.handle for p in self.posets])
        h = ctypes.c_void_p()
        _lib.check(_lib.lib().px_batch_build(len(self.posets), arr, ctypes.byref(h)), "px_batch_build")
        self._h = h
        rows = ctypes.c_int64()
        _lib.check(_lib.lib().px_batch_rows(h, ctypes.byref(rows)), "px_batch_rows")
        self.rows = rows.value
        self.offsets = np.concatenate([[0], np.cumsum([p.n for p in self.posets])]).astype(np.int64)
        self.device = self.posets[0].device if self.posets else 0

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            try:
                _lib.lib().px_batch_free(h)
            except Exception:
                pass
            self._h = None

    @property
    def handle(self):
        if not self._h:
            raise ValueError("batch handle was freed")
        return self._h

    def reserve(self, dtype, B: int):
        import torch
        code = {torch.int64: 0, torch.float32: 1, torch.float64: 2}[dtype]
        _lib.check(_lib.lib().px_batch_reserve(self.handle, code, int(B)), "px_batch_reserve")

    def set_layout(self, layout: str) -> None:
        """"nodes" (default): each poset's rows in node order; "rows": each poset's chain-major
        rows (self.row_order()), the order the kernels run in (px_batch_set_layout)."""
        code = {"nodes": _lib.PX_LAYOUT_NODES, "rows": _lib.PX_LAYOUT_ROWS}[layout]
        _lib.check(_lib.lib().px_batch_set_layout(self.handle, code), "px_batch_set_layout")

    def row_order(self) -> np.ndarray:
        """Batch row of every batch node (px_batch_row_order)."""
        out = np.empty(self.rows, np.int64)
        _lib.check(_lib.lib().px_batch_row_order(self.handle, out.ctypes.data), "px_batch_row_order")
        return out

    def autotune(self, dtype, B: int) -> dict:
        """Pick the RHS tile of the batched gather by timing the candidates (px_batch_autotune)."""
        import torch
        code = {torch.int64: 0, torch.float32: 1, torch.float64: 2}[dtype]
        rep = _lib.TuneReport()
        _lib.check(_lib.lib().px_batch_autotune(self.handle, code, int(B), ctypes.byref(rep)),
                   "px_batch_autotune")
        return rep.as_dict()


def batch_build(posets) -> Batch:
    return Batch(posets)


def _batched(fn_name, b, x, out):
    x = _as_matrix(x, "input", b.device)
    if x.shape[0] != b.rows:
        raise ValueError(f"input has {x.shape[0]} rows, batch has {b.rows}")
    out, out2 = _out_matrix(out, x)
    fn = getattr(_lib.lib(), fn_name)
    _lib.check(fn(b.handle, _dtype_code(x), ctypes.c_void_p(x.data_ptr()), _ld(x), ctypes.c_void_p(out2.data_ptr()),
                  _ld(out2), int(x.shape[1]), _stream(x)), fn_name)
    return out


def zeta_batched(b: Batch, f, out=None):
    return _batched("px_zeta_batched", b, f, out)


def zeta_adjoint_batched(b: Batch, w, out=None):
    return _batched("px_zeta_adjoint_batched", b, w, out)
