"""GPU parity at the full sizes of the benchmarked workloads (run on an MI355X).

  * n = 2**23, k = 32 chains of 262,144 elements, 3 cross edges, B = 16: the
    chain scan's carry runs over four windows of 256 tiles per chain.  float32
    zeta and its adjoint at sampled elements against the down-set / up-set sums
    of the oracle; int64 zeta at sampled elements; int64 Möbius(zeta f) = f and
    M^T(Z^T f) = f at every element (Corollary 1).
  * chains of 20,000 elements at B = 64: more than 256 tiles of 64 rows per
    chain, so the compact walk's carry (and the scan that forms P) runs over two
    windows.
  * 512 uneven posets (n log-uniform in [1000, 65536], k in {4, ..., 128},
    cross degree 2-5), B = 8 float32, forward zeta and the adjoint recorded in
    one HIP graph and replayed; the replays are compared with the closure
    oracle on the 16 smallest posets (Z f and Z^T w, the gradient of
    loss = Σ w·ζ(f)), with sampled elements of the 4 largest, and with the
    eager autograd gradient; float64 gradcheck through the batch.

Sampled oracle: one breadth-first search per element covers several function
matrices stacked as columns (float64 sums; integer data stays below 2**53, so
those sums are exact).
"""

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def px():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2211_13706_amd as px
    px.lib()
    return px


def dev():
    import torch
    return torch.device("cuda:0")


def T(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def H(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def build(px, p, **kw):
    return px.poset_build(p.n, p.indptr, p.indices, p.chain_of, p.chain_pos, device=0, **kw)


def check_f32(got, want, zabs):
    """Componentwise |ĝ - g| <= 3 u32 (Z|f|)(x), and normwise <= 1e-5 per column."""
    got = np.asarray(got, np.float64)
    err = np.abs(got - want)
    assert (err <= 3 * U32 * zabs + 1e-30).all(), float((err / (zabs + 1e-30)).max())
    den = np.maximum(np.abs(want).max(axis=0), 1e-300)
    assert float((err.max(axis=0) / den).max()) <= 1e-5


def sampled(p, cols, nodes, adjoint=False):
    """The oracle at `nodes` for the column blocks in `cols` (one search per element)."""
    stack = np.concatenate([np.asarray(c, np.float64) for c in cols], axis=1)
    fn = O.zeta_adjoint_at if adjoint else O.zeta_at
    out = fn(p.n, p.indptr, p.indices, stack, nodes)
    widths = np.cumsum([0] + [c.shape[1] for c in cols])
    return [out[:, widths[i]:widths[i + 1]] for i in range(len(cols))]


# ------------------------------------------------------- n = 2**23, k = 32
@pytest.fixture(scope="module")
def cfg4(px):
    print("[full-size] generating n=2^23, k=32, cross 3, seed 4", flush=True)
    q = W.chain_poset(1 << 23, 32, 3, seed=4)
    L = build(px, q)
    rng = np.random.default_rng(23)
    tops = [int(np.flatnonzero((q.chain_of == c))[np.argmax(q.chain_pos[q.chain_of == c])]) for c in (0, 17)]
    nodes = np.concatenate([rng.choice(q.n, 4, replace=False), tops])
    return q, L, nodes


def test_config4_f32_zeta_and_adjoint_sampled(px, cfg4):
    q, L, nodes = cfg4
    print(f"[full-size] n=2^23 float32 zeta/adjoint, nodes {nodes.tolist()}", flush=True)
    assert L.k == 32 and L.info["max_chain"] == 262144
    f = W.functions(q.n, 16, "normal", seed=5)
    ft = T(f)
    g = H(px.zeta(L, ft))[nodes]
    a = H(px.zeta_adjoint(L, ft))[nodes]
    want, zabs = sampled(q, [f, np.abs(f)], nodes)
    check_f32(g, want, zabs)
    want_a, zabs_a = sampled(q, [f, np.abs(f)], nodes, adjoint=True)
    check_f32(a, want_a, zabs_a)


def test_config4_int64_zeta_sampled_and_exact_roundtrips(px, cfg4):
    q, L, nodes = cfg4
    print("[full-size] n=2^23 int64 zeta sampled, Möbius and adjoint round trips", flush=True)
    f = W.functions(q.n, 16, "int", seed=6, lo=-1000, hi=1000)
    ft = T(f)
    g = px.zeta(L, ft)
    (want,) = sampled(q, [f], nodes)         # |sums| <= 2**23 * 1000 < 2**53: exact
    assert np.array_equal(H(g)[nodes], want.astype(np.int64))
    assert np.array_equal(H(px.mobius(L, g)), f)
    del g
    w = px.zeta_adjoint(L, ft)
    (want_a,) = sampled(q, [f], nodes, adjoint=True)
    assert np.array_equal(H(w)[nodes], want_a.astype(np.int64))
    assert np.array_equal(H(px.mobius_adjoint(L, w)), f)


def test_config4_f32_mobius_reports_nonfinite(px, cfg4):
    """The float32 Möbius of this poset overflows (its entries of μ grow far beyond float32's
    range): the default call reports PX_ENONFINITE instead of returning Inf / NaN silently."""
    q, L, _ = cfg4
    f = T(W.functions(q.n, 16, "normal", seed=5))
    g = px.zeta(L, f)
    with pytest.raises(px.PosetxError) as e:
        px.mobius(L, g, max_refine=1)
    assert e.value.name == "PX_ENONFINITE"


# ------------------------------------- chains longer than one carry window
SCAN_MODES = {"compact": {}, "rows": {"POSETX_WALK": "rows"}}


@pytest.fixture(scope="module")
def long_chains(px):
    p = W.chain_poset(100_000, 5, 3, seed=9)    # 5 chains of 20,000: 313 tiles of 64 rows each
    rng = np.random.default_rng(9)
    tops = [int(np.flatnonzero(p.chain_of == c)[np.argmax(p.chain_pos[p.chain_of == c])]) for c in range(5)]
    bottoms = [int(np.flatnonzero(p.chain_of == c)[np.argmin(p.chain_pos[p.chain_of == c])]) for c in (1, 3)]
    return p, np.concatenate([rng.choice(p.n, 6, replace=False), tops, bottoms])


@pytest.mark.parametrize("mode", list(SCAN_MODES))
def test_two_carry_windows_int64_exact(px, long_chains, mode, monkeypatch):
    for k, v in SCAN_MODES[mode].items():
        monkeypatch.setenv(k, v)
    p, nodes = long_chains
    P = build(px, p)
    assert P.info["max_chain"] == 20000
    f = W.functions(p.n, 64, "int", seed=10, lo=-(2**40), hi=2**40)
    ft = T(f)
    g, a = px.zeta(P, ft), px.zeta_adjoint(P, ft)
    small = W.functions(p.n, 64, "int", seed=11, lo=-1000, hi=1000)
    gs, as_ = H(px.zeta(P, T(small)))[nodes], H(px.zeta_adjoint(P, T(small)))[nodes]
    want, want_a = sampled(p, [small], nodes)[0], sampled(p, [small], nodes, adjoint=True)[0]
    assert np.array_equal(gs, want.astype(np.int64)) and np.array_equal(as_, want_a.astype(np.int64))
    # Möbius is a bijection, so M(ĝ) = f at every element means ĝ = Z f everywhere
    assert np.array_equal(H(px.mobius(P, g)), f)
    assert np.array_equal(H(px.mobius_adjoint(P, a)), f)


@pytest.mark.parametrize("mode", list(SCAN_MODES))
def test_two_carry_windows_f32(px, long_chains, mode, monkeypatch):
    for k, v in SCAN_MODES[mode].items():
        monkeypatch.setenv(k, v)
    p, nodes = long_chains
    P = build(px, p)
    f = W.functions(p.n, 64, "normal", seed=12)
    ft = T(f)
    g, a = H(px.zeta(P, ft))[nodes], H(px.zeta_adjoint(P, ft))[nodes]
    want, zabs = sampled(p, [f, np.abs(f)], nodes)
    check_f32(g, want, zabs)
    want_a, zabs_a = sampled(p, [f, np.abs(f)], nodes, adjoint=True)
    check_f32(a, want_a, zabs_a)
    # integer data below 2**24 per chain prefix (20,000 * 500): every output is the exact
    # integer rounded once to float32
    fi = W.functions(p.n, 64, "int", seed=13, lo=-500, hi=500)
    gi = H(px.zeta(P, T(fi.astype(np.float32))))
    (wi,) = sampled(p, [fi], nodes)
    assert np.array_equal(gi[nodes], wi.astype(np.float32))


# ------------------------------------------------ 512 posets, graph replay
@pytest.fixture(scope="module")
def cfg3(px):
    print("[full-size] building the 512-poset batch (seed 40)", flush=True)
    posets = W.batched_posets(512, seed=40)
    Ps = [build(px, q) for q in posets]
    b = px.batch_build(Ps)
    del Ps
    return posets, b


def test_config3_graph_replay_matches_oracle(px, cfg3):
    import torch
    from paper_2211_13706_amd.autograd import batch_zeta_fn
    posets, b = cfg3
    assert len(posets) == 512 and b.rows == sum(q.n for q in posets)
    Bb = 8
    b.reserve(torch.float32, Bb)
    f = torch.empty(b.rows, Bb, device=dev())
    w = torch.empty(b.rows, Bb, device=dev())
    g = torch.empty(b.rows, Bb, device=dev())
    gw = torch.empty(b.rows, Bb, device=dev())
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):       # warm-up off the capture
        px.zeta_batched(b, f, out=g)
        px.zeta_adjoint_batched(b, w, out=gw)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        px.zeta_batched(b, f, out=g)
        px.zeta_adjoint_batched(b, w, out=gw)
    smallest = np.argsort([q.n for q in posets], kind="stable")[:16]
    largest = np.argsort([q.n for q in posets], kind="stable")[-4:]
    closures = {int(i): O.reachability(posets[i].n, posets[i].indptr, posets[i].indices) for i in smallest}
    for rep in range(3):
        print(f"[full-size] config 3 replay {rep}", flush=True)
        fh = W.functions(b.rows, Bb, "normal", seed=60 + rep)
        wh = W.functions(b.rows, Bb, "normal", seed=70 + rep)
        f.copy_(T(fh))
        w.copy_(T(wh))
        torch.cuda.synchronize()
        graph.replay()
        gh, gwh = H(g).astype(np.float64), H(gw).astype(np.float64)
        for i in smallest:
            s0, e0 = b.offsets[i], b.offsets[i + 1]
            R = closures[int(i)]
            Rf = R.astype(np.float64)
            check_f32(gh[s0:e0], Rf @ fh[s0:e0].astype(np.float64), Rf @ np.abs(fh[s0:e0]).astype(np.float64))
            check_f32(gwh[s0:e0], Rf.T @ wh[s0:e0].astype(np.float64), Rf.T @ np.abs(wh[s0:e0]).astype(np.float64))
        if rep == 0:
            for i in largest:
                q = posets[i]
                s0 = b.offsets[i]
                nodes = np.random.default_rng(int(i)).choice(q.n, 2, replace=False)
                want, zabs = sampled(q, [fh[s0:s0 + q.n], np.abs(fh[s0:s0 + q.n])], nodes)
                check_f32(gh[s0 + nodes], want, zabs)
                want_a, zabs_a = sampled(q, [wh[s0:s0 + q.n], np.abs(wh[s0:s0 + q.n])], nodes, adjoint=True)
                check_f32(gwh[s0 + nodes], want_a, zabs_a)
        # the eager autograd gradient of loss = Σ w·ζ(f) is the replayed adjoint
        ff = f.clone().requires_grad_(True)
        (batch_zeta_fn(b, ff) * w).sum().backward()
        assert torch.equal(ff.grad, gw)


def test_config3_float64_gradcheck(px, cfg3):
    """Finite differences through the whole 512-poset batch in float64 (gradcheck's fast
    mode: a random projection of the Jacobian against its numerical estimate)."""
    import torch
    from paper_2211_13706_amd.autograd import batch_zeta_fn
    _, b = cfg3
    f = torch.randn(b.rows, 2, dtype=torch.float64, device=dev(), requires_grad=True)
    assert torch.autograd.gradcheck(lambda x: batch_zeta_fn(b, x), (f,), eps=1e-3, atol=1e-6, rtol=1e-6,
                                    fast_mode=True)
