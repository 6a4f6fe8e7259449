"""px_zeta_noalloc: the zeta entry point whose scratch is a static device array.

Called through the C ABI with caller-allocated outputs, it must return what
px_zeta returns (the same kernels: bit-identical for int64 and float32) on
consecutive calls, the second one smaller than the first, so that it runs on
the scratch contents the first call left behind.  A call whose scratch would
exceed the static array is refused before anything is launched.  On a small
poset the result is also checked against the closure oracle.
"""

import ctypes

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def px():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2211_13706_amd as px
    px.lib()
    return px


def _call(px, fn, P, x, out):
    import torch
    code = {torch.int64: px.PX_I64, torch.float32: px.PX_F32, torch.float64: px.PX_F64}[x.dtype]
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return getattr(px.lib(), fn)(P.handle, code, ctypes.c_void_p(x.data_ptr()), x.shape[1],
                                 ctypes.c_void_p(out.data_ptr()), out.shape[1], x.shape[1], stream)


def _both(px, P, x):
    """(px_zeta result, px_zeta_noalloc result) on the host."""
    import torch
    ref = torch.full_like(x, -7)
    got = torch.full_like(x, -7)
    assert _call(px, "px_zeta", P, x, ref) == 0, px.lib().px_last_error()
    assert _call(px, "px_zeta_noalloc", P, x, got) == 0, px.lib().px_last_error()
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy()


def _poset(px, n, k, seed):
    p = W.chain_poset(n, k, 3, seed=seed)
    return p, px.poset_build(p.n, p.indptr, p.indices, p.chain_of, p.chain_pos, device=0)


@pytest.mark.parametrize("kind", ["normal", "int"])
def test_noalloc_matches_px_zeta_on_two_calls(px, kind):
    import torch
    dtype = torch.float32 if kind == "normal" else torch.int64
    # first call: the compact walk (k <= 64, B = 64) over 2^17 rows; then smaller
    # ones: B = 8 (the narrow compact walk) and B = 4 (the scan over P and the
    # lane-split walk)
    for n, k, B, seed in ((1 << 17, 64, 64, 11), (3000, 24, 8, 12), (2000, 24, 4, 13)):
        p, P = _poset(px, n, k, seed)
        f = W.functions(n, B, kind, seed=seed + 100, lo=-1000, hi=1000)
        x = torch.from_numpy(f).cuda()
        ref, got = _both(px, P, x)
        print(f"noalloc {kind} n={n} k={P.k} B={B}", flush=True)
        assert np.array_equal(ref, got)


def test_noalloc_matches_oracle_small(px):
    import torch
    p, P = _poset(px, 2000, 16, 0)
    R = O.reachability(p.n, p.indptr, p.indices)
    f = W.functions(p.n, 3, "int", seed=1, lo=-100, hi=100)
    out = torch.empty((p.n, 3), dtype=torch.int64, device="cuda:0")
    assert _call(px, "px_zeta_noalloc", P, torch.from_numpy(f).cuda(), out) == 0
    assert np.array_equal(out.cpu().numpy(), O.zeta(R, f))


def test_noalloc_refuses_oversized_scratch(px, monkeypatch):
    import torch
    # int64, B = 32 through the scan over P (narrow blocks kept off the compact
    # walk) over 300,000 rows: the prefix matrix alone is 76.8 MB > 64 MiB
    monkeypatch.setenv("POSETX_COMPACT_NARROW", "0")
    p, P = _poset(px, 300000, 32, 5)
    x = torch.ones((p.n, 32), dtype=torch.int64, device="cuda:0")
    out = torch.full_like(x, 3)
    st = _call(px, "px_zeta_noalloc", P, x, out)
    assert st == 1  # PX_EINVAL
    assert b"static scratch" in px.lib().px_last_error()
    torch.cuda.synchronize()
    assert bool((out == 3).all())
    # the same call through px_zeta is fine, and a smaller one still runs after the refusal
    ref, got = _both(px, P, x[:, :4].contiguous())
    assert np.array_equal(ref, got)
