"""GPU parity of the HIP path against the CPU oracle (run on an MI355X).

Every case builds a seeded poset, runs the library through the C ABI
(paper_2211_13706_amd, ctypes) and compares with the oracle computed from the
same seeded inputs:
  int64   bit-exact (wrap-around modulo 2**64);
  float64 normwise relative error <= 1e-12;
  float32 zeta: componentwise |g_hat - g| <= 3 u32 (Z|f|)(x), u32 = 2**-24
          (compensated chain scan: each chain prefix within ~u32 of its exact
          value; the k prefixes are added in float64; one final rounding), and
          normwise per column <= 1e-5;
  float32 Möbius after float64-residual refinement: normwise per column <= 1e-5
          on the well-posed cases (grid, small posets).
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


def px_int64():
    import torch
    return torch.int64


def H(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def build(px, p, planted=True, **kw):
    return px.poset_build(p.n, p.indptr, p.indices, p.chain_of if planted else None,
                          p.chain_pos if planted else None, device=0, **kw)


def rel(a, b):
    """Normwise relative error per column, max over columns."""
    a = np.asarray(a, np.float64); b = np.asarray(b, np.float64)
    den = np.maximum(np.abs(b).max(axis=0), 1e-300)
    return float((np.abs(a - b).max(axis=0) / den).max())


def check_f32_zeta(got, want, zabs):
    got = np.asarray(got, np.float64)
    assert (np.abs(got - want) <= 3 * U32 * zabs + 1e-30).all(), float((np.abs(got - want) / (zabs + 1e-30)).max())
    assert rel(got, want) <= 1e-5


# ------------------------------------------------------------- worked example
@pytest.mark.parametrize("kind", ["int", "f32", "f64"])
def test_worked_example_all_transforms(px, kind):
    p = W.worked_example()
    R = O.reachability(p.n, p.indptr, p.indices)
    P = build(px, p)
    f = W.functions(12, 3, "int", seed=7, lo=-50, hi=50)
    if kind != "int":
        f = f.astype(np.float32 if kind == "f32" else np.float64)
    fi = f.astype(np.int64)
    assert np.array_equal(H(px.zeta(P, T(f))).astype(np.int64), O.zeta(R, fi))
    assert np.array_equal(H(px.zeta_adjoint(P, T(f))).astype(np.int64), O.zeta_adjoint(R, fi))
    assert np.array_equal(H(px.mobius(P, T(f))).astype(np.int64), O.mobius(R, fi))
    assert np.array_equal(H(px.mobius_adjoint(P, T(f))).astype(np.int64), O.mobius_adjoint(R, fi))


# ---------------------------------------------------- config-0 shaped, int64
@pytest.fixture(scope="module")
def cfg0():
    p = W.chain_poset(2000, 16, 4, seed=0)
    R = O.reachability(p.n, p.indptr, p.indices)
    return p, R


@pytest.mark.parametrize("B,ld", [(1, 1), (3, 5), (64, 64), (100, 104)])
def test_cfg0_int64_bit_exact(px, cfg0, B, ld):
    p, R = cfg0
    P = build(px, p)
    f = W.functions(p.n, B, "int", seed=1, lo=-100, hi=100)
    fp = np.zeros((p.n, ld), np.int64); fp[:, :B] = f
    ft = T(fp)[:, :B]
    g = H(px.zeta(P, ft))
    assert np.array_equal(g, O.zeta(R, f))
    assert np.array_equal(H(px.mobius(P, T(g))), f)
    assert np.array_equal(H(px.zeta_adjoint(P, ft)), O.zeta_adjoint(R, f))
    # Möbius of an arbitrary g (not a zeta image): substitution oracle, exact mod 2**64
    gr = W.functions(p.n, B, "int", seed=3, lo=-1000, hi=1000)
    assert np.array_equal(H(px.mobius(P, T(gr))), O.mobius_by_substitution(R, gr))
    assert np.array_equal(H(px.mobius_adjoint(P, T(gr))), O.mobius_adjoint_by_substitution(R, gr))


def test_int64_wraparound(px, cfg0):
    p, R = cfg0
    P = build(px, p)
    f = W.functions(p.n, 2, "int", seed=4, lo=-(2**62), hi=2**62)
    g = H(px.zeta(P, T(f)))
    assert np.array_equal(g, O.zeta(R, f))
    assert np.array_equal(H(px.mobius(P, T(g))), f)


def test_results_independent_of_decomposition_and_schedule(px, cfg0):
    """Planted chains, matching chains, Mirsky and U-dependency schedules agree exactly."""
    p, R = cfg0
    f = T(W.functions(p.n, 4, "int", seed=5, lo=-100, hi=100))
    ff = T(W.functions(p.n, 4, "normal", seed=5))
    outs = []
    for planted, flags in ((True, 0), (False, 0), (True, px.PX_BUILD_LEVELS_MIRSKY)):
        P = build(px, p, planted=planted, flags=flags)
        outs.append((H(px.zeta(P, f)), H(px.mobius(P, f)), H(px.mobius_adjoint(P, f)),
                     H(px.mobius(P, ff, max_refine=0)), P.k))
    for o in outs[1:]:
        for a, b in zip(outs[0][:3], o[:3]):
            assert np.array_equal(a, b)
    # same chains, different schedule: the per-element float arithmetic is identical
    assert np.array_equal(outs[0][3], outs[2][3])


# ------------------------------------------------------------ float accuracy
@pytest.mark.parametrize("B", [1, 5, 16, 33, 64, 100])
def test_f32_zeta_tolerance(px, cfg0, B):
    p, R = cfg0
    P = build(px, p)
    f = W.functions(p.n, B, "normal", seed=11 + B)
    want = O.zeta(R, f, exact=False)
    zabs = O.zeta(R, np.abs(f).astype(np.float64), exact=False)
    check_f32_zeta(H(px.zeta(P, T(f))), want, zabs)
    wantT = O.zeta_adjoint(R, f, exact=False)
    zabsT = O.zeta_adjoint(R, np.abs(f).astype(np.float64), exact=False)
    check_f32_zeta(H(px.zeta_adjoint(P, T(f))), wantT, zabsT)


@pytest.mark.parametrize("B", [8, 40])
def test_f64_zeta_and_mobius(px, cfg0, B):
    """B = 40: one 64-wide column block, 24 lanes idle (uniform-row kernels)."""
    p, R = cfg0
    P = build(px, p)
    f = W.functions(p.n, B, "normal64", seed=12)
    g = H(px.zeta(P, T(f)))
    assert rel(g, O.zeta(R, f, exact=False)) <= 1e-12
    assert rel(H(px.zeta_adjoint(P, T(f))), O.zeta_adjoint(R, f, exact=False)) <= 1e-12
    # Möbius on a zeta image returns f (well-posed: the data are consistent)
    assert rel(H(px.mobius(P, T(g))), f) <= 1e-9


@pytest.mark.parametrize("B", [8, 48])
def test_f32_mobius_refined_small_poset(px, B):
    """g = Z f with integer f is exact in float32, so M g = f exactly is the target.
    B = 48 takes the uniform-row solve and walk (float32 solve, float64 residual)."""
    p = W.chain_poset(1500, 12, 3, seed=21)
    R = O.reachability(p.n, p.indptr, p.indices)
    P = build(px, p)
    f = W.functions(p.n, B, "int", seed=22, lo=-100, hi=100)
    g32 = O.zeta(R, f).astype(np.float32)
    got, rep = px.mobius(P, T(g32), max_refine=8, tol=1e-8, report=True)
    assert rel(H(got), f) <= 1e-5, rep
    assert not rep["nonfinite"]
    v32 = O.zeta_adjoint(R, f).astype(np.float32)
    gotT, repT = px.mobius_adjoint(P, T(v32), max_refine=8, tol=1e-8, report=True)
    assert rel(H(gotT), f) <= 1e-5, repT


# ------------------------------------------------------------ special cases
@pytest.mark.parametrize("B", [1, 64])
def test_chain_prefix_sum_and_difference(px, B):
    p = W.chain_only(5000, seed=2)
    P = build(px, p)
    order = np.argsort(p.chain_pos)
    f = W.functions(p.n, B, "int", seed=3, lo=-9, hi=9)
    g = H(px.zeta(P, T(f)))
    assert np.array_equal(g[order], np.cumsum(f[order], axis=0))
    a = H(px.zeta_adjoint(P, T(f)))
    assert np.array_equal(a[order], np.cumsum(f[order][::-1], axis=0)[::-1])
    m = H(px.mobius(P, T(f)))
    fo = f[order]
    assert np.array_equal(m[order], fo - np.vstack([np.zeros((1, B), np.int64), fo[:-1]]))
    ff = W.functions(p.n, B, "normal", seed=4)
    gf = H(px.zeta(P, T(ff))).astype(np.float64)
    ex = np.cumsum(ff[order].astype(np.float64), axis=0)
    exabs = np.cumsum(np.abs(ff[order]).astype(np.float64), axis=0)
    check_f32_zeta(gf[order], ex, exabs)


def test_antichain_identity(px):
    p = W.antichain(3000)
    P = build(px, p, planted=False)
    assert P.k == 3000
    f = W.functions(p.n, 3, "normal", seed=5)
    assert np.array_equal(H(px.zeta(P, T(f))), f)
    assert np.array_equal(H(px.mobius(P, T(f), max_refine=0)), f)


def test_boolean_lattice_yates(px):
    m = 10
    p = W.boolean_lattice(m)
    P = build(px, p, planted=False)
    assert P.k == 252
    f = W.functions(p.n, 4, "int", seed=6, lo=-9, hi=9)
    want = f.copy()
    for e in range(m):
        bit = 1 << e
        idx = np.nonzero(np.arange(p.n) & bit)[0]
        want[idx] += want[idx ^ bit]
    g = H(px.zeta(P, T(f)))
    assert np.array_equal(g, want)
    assert np.array_equal(H(px.mobius(P, T(g))), f)
    # μ(S,T) = (-1)^{|T \ S|}: Möbius of the indicator of the empty set's zeta column
    pc = np.array([bin(v).count("1") for v in range(p.n)])
    e0 = np.zeros((p.n, 1), np.int64); e0[p.n - 1] = 1        # f = delta at the full set
    mt = H(px.mobius_adjoint(P, T(e0)))[:, 0]                  # M^T e_full = μ(·, full)
    assert np.array_equal(mt, 1 - 2 * ((m - pc) % 2))


def _grid_closed_forms(g3):
    h, w, B = g3.shape
    pad = np.zeros((h + 1, w + 1, B), g3.dtype); pad[1:, 1:] = g3
    return pad[1:, 1:] - pad[:-1, 1:] - pad[1:, :-1] + pad[:-1, :-1]


def test_grid_config2_int64(px):
    h, w = 4096, 64
    p = W.grid_poset(h, w)
    P = build(px, p)
    assert P.info["udep_levels"] == 64
    f = W.functions(p.n, 16, "int", seed=8, lo=-1000, hi=1000)
    g = H(px.zeta(P, T(f)))
    assert np.array_equal(g.reshape(h, w, 16), f.reshape(h, w, 16).cumsum(0).cumsum(1))
    assert np.array_equal(H(px.mobius(P, T(g))), f)
    gr = W.functions(p.n, 16, "int", seed=9, lo=-1000, hi=1000)
    assert np.array_equal(H(px.mobius(P, T(gr))).reshape(h, w, 16), _grid_closed_forms(gr.reshape(h, w, 16)))


def test_grid_config2_f32_refined(px):
    h, w, B = 4096, 64, 16
    p = W.grid_poset(h, w)
    P = build(px, p)
    g = W.functions(p.n, B, "uniform", seed=10, lo=-1.0, hi=1.0)
    want = _grid_closed_forms(g.astype(np.float64).reshape(h, w, B)).reshape(p.n, B)
    got, rep = px.mobius(P, T(g), max_refine=6, tol=1e-6, report=True)
    assert rel(H(got), want) <= 1e-5, rep
    assert rep["correction"] <= 1e-6 and not rep["nonfinite"]
    plain = H(px.mobius(P, T(g), max_refine=0))
    got64 = H(px.mobius(P, T(g.astype(np.float64))))
    assert rel(got64, want) <= 1e-12
    print(f"grid f32 Möbius: plain err {rel(plain, want):.2e}, refined {rel(H(got), want):.2e}, {rep}")


# ------------------------------------------------------------ scan schedules
# "compact": the default at 64-column blocks (the scan records P only at the
# walk's gathered rows and the combine is fused into it); the others write P
# with the named scan and walk over it.
SCAN_MODES = {"compact": {}, "3phase": {"POSETX_WALK": "rows"},
              "onepass": {"POSETX_WALK": "rows", "POSETX_SCAN": "onepass"},
              "fallback": {"POSETX_WALK": "rows", "POSETX_SCAN": "onepass", "POSETX_LB_SPIN": "0"}}


@pytest.mark.parametrize("mode", list(SCAN_MODES))
def test_scan_schedules_grid_exact(px, mode, monkeypatch):
    """Every chain-scan schedule gives the exact 2-D prefix sums at full size.

    Grid 4096 x 64 with B = 64: one 64-wide column block and chains of 64 tiles,
    so the single-pass look-back crosses several super-tiles.  "fallback" makes
    every look-back wait give up at once, so tiles sum their predecessors from
    the input.  int64 is compared with the closed form; float32 runs on integer
    data whose chain prefixes stay below 2**24 and whose k-term sums are exact in
    float64, so it must equal the closed form rounded once to float32.  The
    adjoint (suffix scan) is the reversed 2-D prefix sum.
    """
    for k, v in SCAN_MODES[mode].items():
        monkeypatch.setenv(k, v)
    h, w, B = 4096, 64, 64
    p = W.grid_poset(h, w)
    P = build(px, p)
    f = W.functions(p.n, B, "int", seed=40, lo=-1000, hi=1000)
    f3 = f.reshape(h, w, B)
    want = f3.cumsum(0).cumsum(1).reshape(p.n, B)
    want_adj = f3[::-1, ::-1].cumsum(0).cumsum(1)[::-1, ::-1].reshape(p.n, B)
    assert np.array_equal(H(px.zeta(P, T(f))), want)
    assert np.array_equal(H(px.zeta_adjoint(P, T(f))), want_adj)
    f32 = T(f.astype(np.float32))
    assert np.array_equal(H(px.zeta(P, f32)), want.astype(np.float32))
    assert np.array_equal(H(px.zeta_adjoint(P, f32)), want_adj.astype(np.float32))


# ---------------------------------------------------------- compact walk
@pytest.mark.parametrize("shape", ["cfg0", "short_chains", "one_chain", "k64", "tile64", "tile65"])
@pytest.mark.parametrize("B", [33, 64, 65, 100, 128])
def test_compact_walk_matches_oracle_and_rows_walk(px, shape, B, monkeypatch):
    """The compact walk (no P matrix) against the oracle and the walk over P.

    Shapes: chains of 125 rows (two 64-row tiles, the second ragged); chains of
    about 8 rows (every tile ragged, many slots per tile); one chain (no other
    chain, so no gathered rows at all); 64 chains (the widest compact form);
    chains of exactly 64 rows (one full tile each, bit 63 of the tile masks) and
    of 65 rows (a one-row tail tile).  B = 33, 65 and 100 leave lanes of the
    last 64-column block idle; B = 128 is two full blocks.  int64 is bit-exact
    both ways; float64 agrees to rounding.
    """
    p = {"cfg0": lambda: W.chain_poset(2000, 16, 4, seed=0),
         "short_chains": lambda: W.chain_poset(400, 50, 3, seed=60),
         "one_chain": lambda: W.chain_only(300, seed=61),
         "k64": lambda: W.chain_poset(3000, 64, 3, seed=62),
         "tile64": lambda: W.chain_poset(64 * 16, 16, 3, seed=75),
         "tile65": lambda: W.chain_poset(65 * 16, 16, 3, seed=76)}[shape]()
    R = O.reachability(p.n, p.indptr, p.indices)
    P = build(px, p)
    f = W.functions(p.n, B, "int", seed=63, lo=-10**6, hi=10**6)
    ff = W.functions(p.n, B, "normal64", seed=64)
    got = {}
    for mode in ("compact", "rows"):
        if mode == "rows":
            monkeypatch.setenv("POSETX_WALK", "rows")
        got[mode] = (H(px.zeta(P, T(f))), H(px.zeta_adjoint(P, T(f))),
                     H(px.zeta(P, T(ff))), H(px.zeta_adjoint(P, T(ff))))
    for mode, (g, a, gf, af) in got.items():
        assert np.array_equal(g, O.zeta(R, f)), mode
        assert np.array_equal(a, O.zeta_adjoint(R, f)), mode
        assert rel(gf, O.zeta(R, ff, exact=False)) <= 1e-12, mode
        assert rel(af, O.zeta_adjoint(R, ff, exact=False)) <= 1e-12, mode
    assert P.info["walk_rows_distinct"] == 0 if shape == "one_chain" else P.info["walk_rows_distinct"] > 0


@pytest.mark.parametrize("B", [8, 64])
def test_zeta_in_place(px, cfg0, B):
    """f == g (same pointer and leading dimension) is allowed for zeta and its
    adjoint: the compact walk (B = 64) writes an element only after the same
    thread has read it; the walk over P (B = 8) reads f only in the scan."""
    p, R = cfg0
    P = build(px, p)
    f = W.functions(p.n, B, "int", seed=67, lo=-100, hi=100)
    x = T(f)
    assert px.zeta(P, x, out=x) is x
    assert np.array_equal(H(x), O.zeta(R, f))
    y = T(f)
    px.zeta_adjoint(P, y, out=y)
    assert np.array_equal(H(y), O.zeta_adjoint(R, f))


def test_compact_walk_refinement_residual(px, monkeypatch):
    """float32 Möbius with float64 residuals: the compact residual (fused
    res - (P + S)) and the residual over P reach the same accuracy."""
    p = W.chain_poset(2500, 20, 3, seed=65)
    R = O.reachability(p.n, p.indptr, p.indices)
    P = build(px, p)
    f = W.functions(p.n, 64, "int", seed=66, lo=-100, hi=100)
    g32 = O.zeta(R, f).astype(np.float32)
    v32 = O.zeta_adjoint(R, f).astype(np.float32)
    for mode in ("compact", "rows"):
        if mode == "rows":
            monkeypatch.setenv("POSETX_WALK", "rows")
        got, rep = px.mobius(P, T(g32), max_refine=8, tol=1e-8, report=True)
        assert rel(H(got), f) <= 1e-5, (mode, rep)
        assert rep["residual"] <= 1e-6 and not rep["nonfinite"], (mode, rep)
        gotT, repT = px.mobius_adjoint(P, T(v32), max_refine=8, tol=1e-8, report=True)
        assert rel(H(gotT), f) <= 1e-5, (mode, repT)


# ------------------------------------------------------------ Möbius shapes
@pytest.mark.parametrize("shape", ["cfg0", "mirsky", "long_chains", "grid"])
@pytest.mark.parametrize("B", [1, 40, 64])
def test_mobius_shapes_exact_and_backward_stable(px, shape, B):
    """Möbius and its adjoint against the substitution oracle on level
    schedules of different shapes: cfg0; the Mirsky schedule (one row per chain
    and level); 4 long chains with few cross edges; a 96 x 16 grid (whole chains
    per level).  int64 is exact.  float64 on zeta images: the solve is backward
    stable (residual at rounding level); the forward error carries the inputs'
    own float64 rounding amplified by the Möbius transform (about 1e-9 here).
    """
    p = {"cfg0": lambda: W.chain_poset(2000, 16, 4, seed=0),
         "mirsky": lambda: W.chain_poset(600, 8, 3, seed=70),
         "long_chains": lambda: W.chain_poset(1200, 4, 1, seed=71),
         "grid": lambda: W.grid_poset(96, 16)}[shape]()
    R = O.reachability(p.n, p.indptr, p.indices)
    P = build(px, p, flags=px.PX_BUILD_LEVELS_MIRSKY if shape == "mirsky" else 0)
    g = W.functions(p.n, B, "int", seed=72, lo=-1000, hi=1000)
    assert np.array_equal(H(px.mobius(P, T(g))), O.mobius_by_substitution(R, g))
    assert np.array_equal(H(px.mobius_adjoint(P, T(g))), O.mobius_adjoint_by_substitution(R, g))
    f64 = W.functions(p.n, B, "normal64", seed=73)
    z64, zt64 = O.zeta(R, f64, exact=False), O.zeta_adjoint(R, f64, exact=False)
    mf, maf = H(px.mobius(P, T(z64))), H(px.mobius_adjoint(P, T(zt64)))
    assert rel(O.zeta(R, mf, exact=False), z64) <= 1e-12
    assert rel(O.zeta_adjoint(R, maf, exact=False), zt64) <= 1e-12
    assert rel(mf, f64) <= 1e-8 and rel(maf, f64) <= 1e-8
    f = W.functions(p.n, B, "int", seed=74, lo=-100, hi=100)
    assert np.array_equal(H(px.mobius(P, px.zeta(P, T(f)))), f)


@pytest.mark.parametrize("B", [5, 8, 16, 32, 64, 130])
@pytest.mark.parametrize("mirsky", [False, True])
def test_int64_solve_by_runs_matches_oracle_and_direct(px, B, mirsky, monkeypatch):
    """The int64 level solve by runs (chunks of up to 32 consecutive rows of one
    chain in one level: a full sum at the chunk's first row, change events after
    it, a scan in LDS; all levels in one persistent launch whose chunks wait for
    the chunks they read from) against the substitution oracle and, bit for bit,
    against the same launch waiting on the rows it reads or on the whole level
    below (POSETX_FLOW_WAIT=rows / level), the chunks launched level by level
    and the row-by-row solve (POSETX_USOLVE=levels / direct).  Chains of 250 elements give
    long runs; the Mirsky schedule gives runs of one row; B covers every column
    tile width of the kernel and two column blocks."""
    p = W.chain_poset(2000, 8, 3, seed=90)
    R = O.reachability(p.n, p.indptr, p.indices)
    P = build(px, p, flags=px.PX_BUILD_LEVELS_MIRSKY if mirsky else 0)
    assert P.info["run_chunks"] > 0
    g = W.functions(p.n, B, "int", seed=91, lo=-(2 ** 40), hi=2 ** 40)
    runs = H(px.mobius(P, T(g))), H(px.mobius_adjoint(P, T(g)))
    assert np.array_equal(runs[0], O.mobius_by_substitution(R, g))
    assert np.array_equal(runs[1], O.mobius_adjoint_by_substitution(R, g))
    # waits on the rows read instead of the level below; one launch per level; row by row
    for var, mode in (("POSETX_FLOW_WAIT", "rows"), ("POSETX_FLOW_WAIT", "level"), ("POSETX_USOLVE", "levels"),
                      ("POSETX_USOLVE", "direct")):
        monkeypatch.setenv(var, mode)
        other = H(px.mobius(P, T(g))), H(px.mobius_adjoint(P, T(g)))
        assert np.array_equal(runs[0], other[0]) and np.array_equal(runs[1], other[1]), mode


@pytest.mark.parametrize("wait", ["values", "rows"])
@pytest.mark.parametrize("B", [8, 40])
def test_int64_solve_values_equal_to_unwritten_mark(px, B, wait, monkeypatch):
    """The persistent int64 solve polling the values marks unwritten rows with the
    int64 minimum; rows whose solution is that very value (columns 0 and 1: chain
    prefix sums of f pinned to it, downward and upward) are taken once their ready
    flags are set.  Zeta against the closure oracle (wrapping int64), and both
    Möbius round trips exact."""
    p = W.chain_poset(3000, 8, 3, seed=88)
    R = O.reachability(p.n, p.indptr, p.indices)
    P = build(px, p)
    assert P.info["run_chunks"] > 0
    lo = np.iinfo(np.int64).min
    f = W.functions(p.n, B, "int", seed=89, lo=-1000, hi=1000)
    f[:, :2] = 0
    ends = np.zeros(int(p.chain_of.max()) + 1, dtype=np.int64)
    np.maximum.at(ends, p.chain_of, p.chain_pos)
    f[p.chain_pos == 0, 0] = lo                   # prefixes from the bottom: every row of a chain
    f[p.chain_pos == ends[p.chain_of], 1] = lo    # suffixes from the top
    f[::7, 1] += 1                                # some rows off the mark
    monkeypatch.setenv("POSETX_FLOW_WAIT", wait)
    with np.errstate(over="ignore"):
        gz, ga = O.zeta(R, f), O.zeta_adjoint(R, f)
    g = px.zeta(P, T(f))
    assert np.array_equal(H(g), gz)
    a = px.zeta_adjoint(P, T(f))
    assert np.array_equal(H(a), ga)
    assert np.array_equal(H(px.mobius(P, g)), f)
    assert np.array_equal(H(px.mobius_adjoint(P, a)), f)


def _level_poll_shape(shape):
    if shape == "cfg0":
        return W.chain_poset(2000, 16, 4, seed=71)
    if shape == "grid":
        return W.grid_poset(96, 24)
    return W.chain_poset(3000, 130, 3, seed=72)  # k > 64: dense rows read in two batches


@pytest.mark.parametrize("shape", ["cfg0", "grid", "k130"])
def test_level_poll_solve_matches_per_level_launches(px, shape, monkeypatch):
    """The row-by-row level solve in one persistent launch that polls the values it
    reads (the default for floating point, and for int64 rows without runs) equals one
    launch per level (POSETX_LEVEL_POLL=2 forces the one, 0 the other) bit for bit: float32 Möbius with its
    float64-residual refinement, float64 Möbius and both adjoints, at B = 1, 16, 24 (8,
    4 and 2 rows per wavefront, whose rows of different levels go one level after the
    other), 64 and 100 (one row per wavefront, two 64-column blocks); int64 row by row
    against the substitution oracle."""
    import torch
    p = _level_poll_shape(shape)
    R = O.reachability(p.n, p.indptr, p.indices)
    P = build(px, p)
    assert P.info["levels_down"] >= 2
    for B in (1, 16, 24, 64, 100):
        f = W.functions(p.n, B, "int", seed=73 + B, lo=-100, hi=100)
        g32 = T(O.zeta(R, f).astype(np.float32))
        g64 = T(O.zeta(R, f).astype(np.float64))
        got = {}
        for poll in ("2", "0"):
            monkeypatch.setenv("POSETX_LEVEL_POLL", poll)
            got[poll] = (px.mobius(P, g32, tol=-1), px.mobius_adjoint(P, g32, tol=-1),
                         px.mobius(P, g64, tol=-1), px.mobius_adjoint(P, g64, tol=-1))
        for a, b in zip(got["2"], got["0"]):
            assert torch.equal(a, b), (shape, B)
        assert rel(H(got["2"][2]), f) <= 1e-9
        monkeypatch.setenv("POSETX_LEVEL_POLL", "2")
        monkeypatch.setenv("POSETX_USOLVE", "direct")
        gi = W.functions(p.n, B, "int", seed=74 + B, lo=-(2 ** 40), hi=2 ** 40)
        assert np.array_equal(H(px.mobius(P, T(gi))), O.mobius_by_substitution(R, gi))
        assert np.array_equal(H(px.mobius_adjoint(P, T(gi))), O.mobius_adjoint_by_substitution(R, gi))
        monkeypatch.delenv("POSETX_USOLVE")


@pytest.mark.parametrize("spin", ["0", "default"])
def test_level_poll_solve_marks_and_fallback(px, spin, monkeypatch):
    """int64 row by row in the persistent launch with solutions equal to its
    unwritten mark (every row of column 0 downward, of column 1 upward): taken once
    the rows' ready flags are set; and with a spin limit of 0 every wait gives up, the
    fallback solves level by level, and float32, float64 and int64 results still equal
    the per-level launches (the give-up path forced from the host)."""
    import torch
    monkeypatch.setenv("POSETX_LEVEL_POLL", "2")
    p = W.chain_poset(2500, 8, 3, seed=75)
    R = O.reachability(p.n, p.indptr, p.indices)
    P = build(px, p)
    if spin == "0":
        monkeypatch.setenv("POSETX_FLOW_SPIN", "0")
    monkeypatch.setenv("POSETX_USOLVE", "direct")
    B = 6
    lo = np.iinfo(np.int64).min
    f = W.functions(p.n, B, "int", seed=76, lo=-1000, hi=1000)
    f[:, :2] = 0
    ends = np.zeros(int(p.chain_of.max()) + 1, dtype=np.int64)
    np.maximum.at(ends, p.chain_of, p.chain_pos)
    f[p.chain_pos == 0, 0] = lo
    f[p.chain_pos == ends[p.chain_of], 1] = lo
    g, a = px.zeta(P, T(f)), px.zeta_adjoint(P, T(f))
    assert np.array_equal(H(px.mobius(P, g)), f)
    assert np.array_equal(H(px.mobius_adjoint(P, a)), f)
    fl = W.functions(p.n, 16, "int", seed=77, lo=-100, hi=100)
    g32 = T(O.zeta(R, fl).astype(np.float32))
    g64 = T(O.zeta(R, fl).astype(np.float64))
    res = {}
    for poll in ("2", "0"):
        monkeypatch.setenv("POSETX_LEVEL_POLL", poll)
        res[poll] = (px.mobius(P, g32, tol=-1), px.mobius(P, g64, tol=-1), px.mobius_adjoint(P, g32, tol=-1))
    for x, y in zip(res["2"], res["0"]):
        assert torch.equal(x, y)


def test_persistent_solves_in_a_hip_graph(px):
    """The persistent Möbius solves captured in one HIP graph (after px_reserve; tol < 0,
    so no host synchronisation): the int64 solve by runs, and the float32 (refined) and
    float64 row-by-row solves.  Each of three replays, with new inputs copied in and eager
    work between them, equals the eager calls bit for bit, and int64 equals the oracle."""
    import torch
    p = W.chain_poset(3000, 16, 3, seed=81)
    R = O.reachability(p.n, p.indptr, p.indices)
    P = build(px, p)
    assert P.info["run_chunks"] > 0
    B = 8
    gi = torch.empty(p.n, B, dtype=torch.int64, device=dev())
    g32 = torch.empty(p.n, B, dtype=torch.float32, device=dev())
    g64 = torch.empty(p.n, B, dtype=torch.float64, device=dev())
    oi, o32, o64 = torch.empty_like(gi), torch.empty_like(g32), torch.empty_like(g64)
    for dt in (torch.int64, torch.float32, torch.float64):
        P.reserve(dt, B)

    def calls():
        px.mobius(P, gi, out=oi)
        px.mobius(P, g32, out=o32, tol=-1)
        px.mobius_adjoint(P, g64, out=o64, tol=-1)

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # warm-up off the capture
        calls()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        calls()
    for rep in range(3):
        print(f"graph replay {rep}", flush=True)
        f = W.functions(p.n, B, "int", seed=82 + rep, lo=-1000, hi=1000)
        gi.copy_(T(O.zeta(R, f)))
        g32.copy_(T(O.zeta(R, f).astype(np.float32)))
        g64.copy_(T(O.zeta_adjoint(R, f).astype(np.float64)))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = (oi.clone(), o32.clone(), o64.clone())
        calls()  # eager, between the replays
        torch.cuda.synchronize()
        assert torch.equal(got[0], oi) and torch.equal(got[1], o32) and torch.equal(got[2], o64)
        assert np.array_equal(H(got[0]), f)
        assert rel(H(got[2]), f) <= 1e-9


@pytest.mark.parametrize("wait", ["deps", "level", "rows", "values"])
@pytest.mark.parametrize("B", [8, 64])
def test_int64_persistent_solve_fallback(px, B, wait, monkeypatch):
    """With a spin limit of 0 polls every wait of the persistent solve gives up at
    once: the error word is set and the one-workgroup fallback solves again, so
    the result is still exact (the give-up path forced from the host; every
    kernel exits normally)."""
    p = W.chain_poset(1500, 6, 3, seed=92)
    R = O.reachability(p.n, p.indptr, p.indices)
    P = build(px, p)
    assert P.info["run_chunks"] > 0
    g = W.functions(p.n, B, "int", seed=93, lo=-(2 ** 40), hi=2 ** 40)
    monkeypatch.setenv("POSETX_FLOW_SPIN", "0")
    monkeypatch.setenv("POSETX_FLOW_WAIT", wait)
    assert np.array_equal(H(px.mobius(P, T(g))), O.mobius_by_substitution(R, g))
    assert np.array_equal(H(px.mobius_adjoint(P, T(g))), O.mobius_adjoint_by_substitution(R, g))
    f = W.functions(p.n, B, "int", seed=94, lo=-100, hi=100)
    assert np.array_equal(H(px.mobius(P, px.zeta(P, T(f)))), f)


@pytest.mark.parametrize("n,deg,seed", [(2000, 12, 4), (2000, 4, 2)])
def test_min_chains_transforms_exact(px, n, deg, seed):
    """Posets built with PX_BUILD_MIN_CHAINS (a minimum chain decomposition):
    int64 zeta, adjoint, Möbius and its adjoint against the closure oracle, bit
    for bit, and float32 zeta within the compensated bound.  ER n = 2000: degree
    12 gives 137 chains (dense rows; the path cover has 145), degree 4 gives 379
    (sparse rows; the path cover has 399)."""
    p = W.er_dag(n, deg, seed=seed)
    R = O.reachability(p.n, p.indptr, p.indices)
    P = px.poset_build(p.n, p.indptr, p.indices, flags=px.PX_BUILD_MIN_CHAINS, device=0)
    assert P.k == O.width(R) < P.info["path_cover"]
    for B in (1, 16, 64):
        f = W.functions(p.n, B, "int", seed=seed + B, lo=-1000, hi=1000)
        g = H(px.zeta(P, T(f)))
        assert np.array_equal(g, O.zeta(R, f))
        assert np.array_equal(H(px.zeta_adjoint(P, T(f))), O.zeta_adjoint(R, f))
        assert np.array_equal(H(px.mobius(P, T(g))), f)
        assert np.array_equal(H(px.mobius(P, T(f))), O.mobius_by_substitution(R, f))
        assert np.array_equal(H(px.mobius_adjoint(P, T(f))), O.mobius_adjoint_by_substitution(R, f))
    ff = W.functions(p.n, 64, "normal", seed=seed)
    check_f32_zeta(H(px.zeta(P, T(ff))), O.zeta(R, ff, exact=False), O.zeta(R, np.abs(ff).astype(np.float64), exact=False))


@pytest.mark.parametrize("B", [1, 8, 16, 32])
def test_masked_compact_walk_for_narrow_blocks(px, cfg0, B, monkeypatch):
    """POSETX_COMPACT_NARROW=1: narrow blocks through the compact walk in 64-column
    tiles (columns beyond B masked) equal the scan over P and the oracle: int64
    bit-exact, float32 zeta and the refinement residual within the bound."""
    p, R = cfg0
    P = build(px, p)
    fi = W.functions(p.n, B, "int", seed=20 + B, lo=-1000, hi=1000)
    ff = W.functions(p.n, B, "normal", seed=20 + B)
    g = O.zeta(R, fi).astype(np.float32)        # exact in float32 (|g| < 2**24)
    monkeypatch.setenv("POSETX_COMPACT_NARROW", "0")   # the scan over P
    base = [H(px.zeta(P, T(fi))), H(px.zeta_adjoint(P, T(fi))), H(px.zeta(P, T(ff))),
            H(px.mobius(P, T(g), max_refine=3))]
    monkeypatch.setenv("POSETX_COMPACT_NARROW", "1")
    got = [H(px.zeta(P, T(fi))), H(px.zeta_adjoint(P, T(fi))), H(px.zeta(P, T(ff))),
           H(px.mobius(P, T(g), max_refine=3))]
    assert np.array_equal(got[0], O.zeta(R, fi)) and np.array_equal(got[1], O.zeta_adjoint(R, fi))
    assert np.array_equal(got[0], base[0]) and np.array_equal(got[1], base[1])
    check_f32_zeta(got[2], O.zeta(R, ff, exact=False), O.zeta(R, np.abs(ff).astype(np.float64), exact=False))
    # the refinement's residual through the masked compact walk converges as through P
    assert rel(got[3], fi) <= max(2 * rel(base[3], fi), 1e-6)


@pytest.mark.parametrize("B", [5, 8, 12, 16, 24, 32])
def test_narrow_compact_walk(px, B, monkeypatch):
    """Blocks of 8 to 32 columns take the compact walk with narrow kernels by default
    (k_scan_reduce_cn, the shared carry, the walk on Q, k_scan_apply_cn: P is never
    formed).  Zeta and its adjoint equal the scan over P (POSETX_COMPACT_NARROW=0) and
    the closure oracle: int64 bit for bit, float32 within the compensated bound, float64
    to rounding; with the walk on Q in both its vector-lane and lane-split forms.  The
    refined float32 Möbius, whose float64 residuals take the same path, recovers f.
    Chains of about 167 rows put chain ends inside the 64-row tiles a workgroup spans."""
    p = W.chain_poset(4000, 24, 3, seed=B)
    R = O.reachability(p.n, p.indptr, p.indices)
    P = build(px, p)
    fi = W.functions(p.n, B, "int", seed=B, lo=-10**6, hi=10**6)
    ff = W.functions(p.n, B, "normal", seed=B + 1)
    fd = W.functions(p.n, B, "normal64", seed=B + 2)
    za = O.zeta(R, np.abs(ff).astype(np.float64), exact=False)
    zta = O.zeta_adjoint(R, np.abs(ff).astype(np.float64), exact=False)
    fs = W.functions(p.n, B, "int", seed=B + 3, lo=-1000, hi=1000)
    gs = O.zeta(R, fs).astype(np.float32)       # exact in float32 (|g| < 2**24)
    monkeypatch.setenv("POSETX_COMPACT_NARROW", "0")
    base = (H(px.zeta(P, T(fi))), H(px.zeta_adjoint(P, T(fi))))
    mob0 = H(px.mobius(P, T(gs), max_refine=3))
    monkeypatch.delenv("POSETX_COMPACT_NARROW")
    # the refined float32 Möbius, whose residuals now run through the narrow compact walk
    mob = H(px.mobius(P, T(gs), max_refine=3))
    assert rel(mob, fs) <= max(2 * rel(mob0, fs), 1e-6)
    for vec in ("0", "1"):
        monkeypatch.setenv("POSETX_WALK_VEC", vec)
        g, a = H(px.zeta(P, T(fi))), H(px.zeta_adjoint(P, T(fi)))
        assert np.array_equal(g, O.zeta(R, fi)) and np.array_equal(a, O.zeta_adjoint(R, fi))
        assert np.array_equal(g, base[0]) and np.array_equal(a, base[1])
        check_f32_zeta(H(px.zeta(P, T(ff))), O.zeta(R, ff, exact=False), za)
        check_f32_zeta(H(px.zeta_adjoint(P, T(ff))), O.zeta_adjoint(R, ff, exact=False), zta)
        assert rel(H(px.zeta(P, T(fd))), O.zeta(R, fd, exact=False)) <= 1e-12
        assert rel(H(px.zeta_adjoint(P, T(fd))), O.zeta_adjoint(R, fd, exact=False)) <= 1e-12


@pytest.mark.parametrize("case", ["cfg0", "er", "grid"])
def test_row_layout_equals_permuted_node_layout(px, case):
    """PX_LAYOUT_ROWS: matrices indexed by chain-major row give the node-order
    results permuted by px_poset_rows, bit for bit (int64 and float32, every
    transform, the refined float32 Möbius included), and switching back to node
    order restores them; int64 results also match the oracle."""
    import torch
    p = {"cfg0": lambda: W.chain_poset(2000, 16, 4, seed=0), "er": lambda: W.er_dag(2000, 4, seed=2),
         "grid": lambda: W.grid_poset(64, 12)}[case]()
    R = O.reachability(p.n, p.indptr, p.indices)
    P = build(px, p, planted=case != "er")
    rows = P.rows()
    fns = (px.zeta, px.zeta_adjoint, px.mobius, px.mobius_adjoint)
    for B in (1, 8, 64):
        fi = W.functions(p.n, B, "int", seed=B, lo=-1000, hi=1000)
        ff = W.functions(p.n, B, "normal", seed=B)
        node = [[H(fn(P, T(x))) for fn in fns] for x in (fi, ff)]
        P.set_layout("rows")
        assert P.info["layout"] == 1
        perm = np.empty_like(rows); perm[rows] = np.arange(p.n)   # perm[row] = node
        got = [[H(fn(P, T(x[perm])))[rows] for fn in fns] for x in (fi, ff)]
        P.set_layout("nodes")
        for a, b in zip(node, got):
            for u, v in zip(a, b):
                assert np.array_equal(u, v)
        assert np.array_equal(node[0][0], O.zeta(R, fi))
        assert np.array_equal(node[0][2], O.mobius_by_substitution(R, fi))
    assert np.array_equal(H(px.zeta(P, T(fi))), node[0][0])


# ------------------------------------------------------- full-size, sampled
@pytest.fixture(scope="module")
def cfg1():
    p = W.chain_poset(1 << 20, 64, 3, seed=1)
    rng = np.random.default_rng(17)
    nodes = np.concatenate([rng.choice(p.n, 6, replace=False), [int(np.argmax(p.chain_pos)), 0]])
    return p, nodes


def test_config1_f32_zeta_sampled(px, cfg1):
    p, nodes = cfg1
    P = build(px, p)
    f = W.functions(p.n, 64, "normal", seed=2)
    g = H(px.zeta(P, T(f)))[nodes]
    want = O.zeta_at(p.n, p.indptr, p.indices, f, nodes)
    zabs = O.zeta_at(p.n, p.indptr, p.indices, np.abs(f), nodes)
    check_f32_zeta(g, want, zabs)


@pytest.mark.parametrize("mode", list(SCAN_MODES))
def test_config1_f32_integer_data_exact_roundtrip(px, cfg1, mode, monkeypatch):
    """float32 zeta at n = 2**20, B = 64 checked at every element.

    Integer data in [-1000, 1000]: each chain prefix is below 16384 * 1000 < 2**24
    and the k-term sums are exact in float64, so every float32 output is the
    exact integer result, which the exact int64 Möbius must map back to f.
    """
    for k, v in SCAN_MODES[mode].items():
        monkeypatch.setenv(k, v)
    p, nodes = cfg1
    P = build(px, p)
    f = W.functions(p.n, 64, "int", seed=41, lo=-1000, hi=1000)
    g32 = px.zeta(P, T(f.astype(np.float32)))
    assert np.array_equal(H(g32)[nodes], O.zeta_at(p.n, p.indptr, p.indices, f, nodes).astype(np.float32))
    assert np.array_equal(H(px.mobius(P, g32.to(dtype=px_int64()))), f)


@pytest.fixture(scope="module")
def cfg1_b512(cfg1):
    p, nodes = cfg1
    rng = np.random.default_rng(77)
    f16 = rng.integers(-1000, 1001, size=(p.n, 512), dtype=np.int16)
    sel = nodes[-2:]  # the top of a chain and node 0
    return f16, sel, O.zeta_at(p.n, p.indptr, p.indices, f16, sel)


@pytest.mark.parametrize("walk", ["compact", "rows"])
def test_config1_f32_B512_sampled_exact(px, cfg1, cfg1_b512, walk, monkeypatch):
    """B = 512 at n = 2**20: eight 64-column blocks, and for the walk over P a P
    matrix of (n + 1) * 512 * 4 bytes > 2**31, so the walk's gathers take
    64-bit row offsets.  Integer data in [-1000, 1000] (chain prefixes below
    2**24, k-term sums exact in float64): every output is the exact integer
    rounded once to float32."""
    import torch
    if walk == "rows":
        monkeypatch.setenv("POSETX_WALK", "rows")
    p, _ = cfg1
    f16, sel, want = cfg1_b512
    P = build(px, p)
    g = px.zeta(P, torch.from_numpy(f16).to(dev()).float())
    assert np.array_equal(H(g)[sel], want.astype(np.float32))


def test_config1_int64_zeta_sampled_and_roundtrip(px, cfg1):
    p, nodes = cfg1
    P = build(px, p)
    f = W.functions(p.n, 64, "int", seed=3, lo=-1000, hi=1000)
    ft = T(f)
    g = px.zeta(P, ft)
    assert np.array_equal(H(g)[nodes], O.zeta_at(p.n, p.indptr, p.indices, f, nodes))
    # Möbius(zeta(f)) = f exactly at every element (Corollary 1), at full size
    assert np.array_equal(H(px.mobius(P, g)), f)
    a = H(px.zeta_adjoint(P, ft))[nodes]
    assert np.array_equal(a, O.zeta_adjoint_at(p.n, p.indptr, p.indices, f, nodes))
    assert np.array_equal(H(px.mobius_adjoint(P, px.zeta_adjoint(P, ft))), f)


# ----------------------------------------------------------------- autograd
def test_autograd_gradcheck_and_dense_transpose(px):
    import torch
    from paper_2211_13706_amd.autograd import mobius_fn, zeta_fn
    p = W.chain_poset(60, 5, 3, seed=30)
    R = O.reachability(p.n, p.indptr, p.indices)
    P = build(px, p)
    f = torch.randn(p.n, 3, dtype=torch.float64, device=dev(), requires_grad=True)
    assert torch.autograd.gradcheck(lambda x: zeta_fn(P, x), (f,), eps=1e-6, atol=1e-7)
    assert torch.autograd.gradcheck(lambda x: mobius_fn(P, x), (f,), eps=1e-6, atol=1e-7)
    # the Jacobian of zeta is the dense closure Z; its transpose is what backward applies
    w = torch.randn(p.n, 3, dtype=torch.float64, device=dev())
    y = zeta_fn(P, f)
    (gf,) = torch.autograd.grad((y * w).sum(), f)
    assert np.allclose(H(gf), R.astype(np.float64).T @ H(w), rtol=1e-12, atol=1e-12)


# ------------------------------------------------------------------ batched
def test_batched_zeta_and_adjoint(px):
    import torch
    from paper_2211_13706_amd.autograd import batch_zeta_fn
    posets = W.batched_posets(16, seed=40, nmin=100, nmax=1500)
    Ps = [build(px, q) for q in posets]
    b = px.batch_build(Ps)
    f = W.functions(b.rows, 8, "int", seed=41, lo=-100, hi=100)
    g = H(px.zeta_batched(b, T(f)))
    a = H(px.zeta_adjoint_batched(b, T(f)))
    for i, q in enumerate(posets):
        s, e = b.offsets[i], b.offsets[i + 1]
        R = O.reachability(q.n, q.indptr, q.indices)
        assert np.array_equal(g[s:e], O.zeta(R, f[s:e]))
        assert np.array_equal(a[s:e], O.zeta_adjoint(R, f[s:e]))
    # autograd through the batch: loss = Σ w·ζ(f), gradient = Z^T w per poset
    ff = torch.randn(b.rows, 8, dtype=torch.float32, device=dev(), requires_grad=True)
    w = torch.randn(b.rows, 8, dtype=torch.float32, device=dev())
    (batch_zeta_fn(b, ff) * w).sum().backward()
    grad = H(ff.grad).astype(np.float64)
    for i, q in enumerate(posets):
        s, e = b.offsets[i], b.offsets[i + 1]
        R = O.reachability(q.n, q.indptr, q.indices)
        want = R.astype(np.float64).T @ H(w)[s:e].astype(np.float64)
        zabs = R.astype(np.float64).T @ np.abs(H(w)[s:e]).astype(np.float64)
        assert (np.abs(grad[s:e] - want) <= 3 * U32 * zabs + 1e-30).all()


def test_batched_autograd_gradcheck(px):
    """Finite differences through the batched zeta (float64, three tiny posets
    of different width): the backward pass is the batched adjoint."""
    import torch
    from paper_2211_13706_amd.autograd import batch_zeta_fn
    posets = W.batched_posets(3, seed=83, nmin=20, nmax=60, ks=(2, 3, 5))
    b = px.batch_build([build(px, q) for q in posets])
    f = torch.randn(b.rows, 2, dtype=torch.float64, device=dev(), requires_grad=True)
    assert torch.autograd.gradcheck(lambda x: batch_zeta_fn(b, x), (f,), eps=1e-6, atol=1e-7)


@pytest.mark.parametrize("B", [1, 33, 100])
def test_batched_widths_and_dtypes(px, B):
    """Batches at other widths: B = 1 (one lane per run), 33 (64-column lane
    groups in the split walk) and 100 (more than 64 columns: one thread per row
    and column over every niv entry).  int64 exact, float64 to rounding."""
    posets = W.batched_posets(10, seed=80, nmin=50, nmax=700)
    Ps = [build(px, q) for q in posets]
    b = px.batch_build(Ps)
    f = W.functions(b.rows, B, "int", seed=81, lo=-1000, hi=1000)
    f64 = W.functions(b.rows, B, "normal64", seed=82)
    g, a = H(px.zeta_batched(b, T(f))), H(px.zeta_adjoint_batched(b, T(f)))
    g64, a64 = H(px.zeta_batched(b, T(f64))), H(px.zeta_adjoint_batched(b, T(f64)))
    for i, q in enumerate(posets):
        s0, e0 = b.offsets[i], b.offsets[i + 1]
        R = O.reachability(q.n, q.indptr, q.indices)
        assert np.array_equal(g[s0:e0], O.zeta(R, f[s0:e0]))
        assert np.array_equal(a[s0:e0], O.zeta_adjoint(R, f[s0:e0]))
        assert rel(g64[s0:e0], O.zeta(R, f64[s0:e0], exact=False)) <= 1e-12
        assert rel(a64[s0:e0], O.zeta_adjoint(R, f64[s0:e0], exact=False)) <= 1e-12


# ---------------------------------------------------------- flat scan tiles
@pytest.mark.parametrize("shape", [(3000, 40, 3), (3000, 4, 2), (2500, 150, 4)])
@pytest.mark.parametrize("B", [1, 3, 8, 16, 32])
def test_flat_tile_scan_matches_oracle(px, shape, B, monkeypatch):
    """The chain scan over flat tiles (fixed blocks of rows whatever chains they hold, a
    chain's first row in scan order resetting the sum), forced on every poset, against the
    closure oracle: zeta and its adjoint, int64 exact and float64 to rounding, at column
    blocks of 1 to 32 (tile heights 4096 down to 128 rows).  Four chains of 750 rows span
    up to six flat tiles, so carries fold several earlier tiles; 40 and 150 chains put
    many chain starts inside one tile.  The int64 results also equal those of the
    chain-aligned tiles bit for bit."""
    n, k, d = shape
    p = W.chain_poset(n, k, d, seed=n + k + B)
    P = build(px, p)
    R = O.reachability(p.n, p.indptr, p.indices)
    f = W.functions(p.n, B, "int", seed=B, lo=-10**6, hi=10**6)
    f64 = W.functions(p.n, B, "normal64", seed=B + 1)
    out = {}
    for flat in ("1", "0"):
        monkeypatch.setenv("POSETX_SCAN_FLAT", flat)
        out[flat] = (H(px.zeta(P, T(f))), H(px.zeta_adjoint(P, T(f))))
        if flat == "1":
            assert np.array_equal(out[flat][0], O.zeta(R, f))
            assert np.array_equal(out[flat][1], O.zeta_adjoint(R, f))
            assert rel(H(px.zeta(P, T(f64))), O.zeta(R, f64, exact=False)) <= 1e-12
            assert rel(H(px.zeta_adjoint(P, T(f64))), O.zeta_adjoint(R, f64, exact=False)) <= 1e-12
    assert np.array_equal(out["1"][0], out["0"][0]) and np.array_equal(out["1"][1], out["0"][1])


def test_flat_tiles_chosen_for_short_chains(px):
    """Chains of 600 rows fill chain-aligned tiles of 512 rows (8 columns) to 59% and take
    flat tiles there, but not at 32 columns (128-row tiles, 94% full); chains of 16,384
    rows fill every tile height and keep chain-aligned tiles.  (Chains within one tile
    keep the single-pass scan of their own tiles.)"""
    mid = build(px, W.chain_poset(6000, 10, 2, seed=5)).info_dict()["scan_flat"]
    assert mid & (1 << 3) and not mid & (1 << 5)
    long_ = build(px, W.chain_poset(1 << 16, 4, 3, seed=6))
    assert long_.info_dict()["scan_flat"] == 0


@pytest.mark.parametrize("B", [8, 16])
def test_batched_flat_tiles(px, B, monkeypatch):
    """A batch of uneven posets through flat and chain-aligned scan tiles: int64 zeta and
    adjoint equal bit for bit and equal the closure oracle per poset."""
    posets = W.batched_posets(12, seed=90 + B, nmin=100, nmax=2000)
    b = px.batch_build([build(px, q) for q in posets])
    f = W.functions(b.rows, B, "int", seed=91, lo=-1000, hi=1000)
    res = {}
    for flat in ("1", "0"):
        monkeypatch.setenv("POSETX_SCAN_FLAT", flat)
        res[flat] = (H(px.zeta_batched(b, T(f))), H(px.zeta_adjoint_batched(b, T(f))))
    assert np.array_equal(res["1"][0], res["0"][0]) and np.array_equal(res["1"][1], res["0"][1])
    g, a = res["1"]
    for i, q in enumerate(posets):
        s0, e0 = b.offsets[i], b.offsets[i + 1]
        R = O.reachability(q.n, q.indptr, q.indices)
        assert np.array_equal(g[s0:e0], O.zeta(R, f[s0:e0]))
        assert np.array_equal(a[s0:e0], O.zeta_adjoint(R, f[s0:e0]))


@pytest.mark.parametrize("B", [8, 100])
def test_batched_row_layout(px, B):
    """A batch with its matrices in the kernels' row order (px_batch_set_layout): zeta and
    its adjoint equal the node-order results permuted by px_batch_row_order, bit for bit
    (int64 and float32), at B = 8 (scans and the vector-lane walk) and B = 100 (the
    one-thread-per-row gather); switching back restores node order."""
    import torch
    posets = W.batched_posets(12, seed=95, nmin=100, nmax=2000)
    b = px.batch_build([build(px, q) for q in posets])
    perm = torch.from_numpy(b.row_order()).to(dev())
    assert np.array_equal(np.sort(b.row_order()), np.arange(b.rows))
    for kind in ("int", "normal"):
        f = T(W.functions(b.rows, B, kind, seed=96, lo=-1000, hi=1000))
        g, a = px.zeta_batched(b, f), px.zeta_adjoint_batched(b, f)
        fr = torch.empty_like(f)
        fr[perm] = f
        b.set_layout("rows")
        gr, ar = px.zeta_batched(b, fr), px.zeta_adjoint_batched(b, fr)
        b.set_layout("nodes")
        assert torch.equal(gr[perm], g) and torch.equal(ar[perm], a)
        assert torch.equal(px.zeta_batched(b, f), g)


def test_batch_from_concurrent_builds(px):
    """Device handles built on several host threads at once (poset_build_many) form a batch
    whose zeta and adjoint equal those of a batch built one poset after another, bit for
    bit (int64), and the closure oracle."""
    import torch
    posets = W.batched_posets(16, seed=98, nmin=200, nmax=4000)
    specs = [(q.n, q.indptr, q.indices, None if i % 3 == 0 else q.chain_of, None if i % 3 == 0 else q.chain_pos)
             for i, q in enumerate(posets)]
    many = px.batch_build(px.poset_build_many(specs, device=0, threads=8))
    one = px.batch_build([px.poset_build(*s, device=0) for s in specs])
    f = T(W.functions(one.rows, 8, "int", seed=99, lo=-1000, hi=1000))
    g, a = px.zeta_batched(many, f), px.zeta_adjoint_batched(many, f)
    assert torch.equal(g, px.zeta_batched(one, f)) and torch.equal(a, px.zeta_adjoint_batched(one, f))
    fh, gh = f.cpu().numpy(), g.cpu().numpy()
    for i, q in enumerate(posets[:4]):
        lo, hi = int(one.offsets[i]), int(one.offsets[i + 1])
        R = O.reachability(q.n, q.indptr, q.indices)
        assert np.array_equal(gh[lo:hi], O.zeta(R, fh[lo:hi]))


@pytest.mark.parametrize("B", [2, 4, 8, 12, 16, 24, 32, 64])
def test_vector_lane_walk(px, B, monkeypatch):
    """The vector-lane walk (each lane gathers 16 bytes of a row: 4 float32 or 2 int64 /
    float64 columns), forced on, against the lane-split walk bit for bit and the closure
    oracle, for one poset (B < 32; wider blocks take the uniform walk there) and for a
    batch, int64, float32 and float64.  Widths that are no multiple of the lane's columns,
    or give fewer than 2 lanes per run, keep the lane-split walk."""
    import torch
    cases = []
    if B < 32:
        p = W.chain_poset(3000, 24, 3, seed=B)
        cases.append(([p], build(px, p), False))
    posets = W.batched_posets(8, seed=97 + B, nmin=100, nmax=1500)
    cases.append((posets, px.batch_build([build(px, q) for q in posets]), True))
    for posets_, h, batched in cases:
        rows = h.rows if batched else h.n
        offs = h.offsets if batched else np.array([0, rows])
        zf, af = ((px.zeta_batched, px.zeta_adjoint_batched) if batched else (px.zeta, px.zeta_adjoint))
        for kind in ("int", "normal", "normal64"):
            f = T(W.functions(rows, B, kind, seed=B + 7, lo=-1000, hi=1000))
            res = {}
            for vec in ("1", "0"):
                monkeypatch.setenv("POSETX_WALK_VEC", vec)
                res[vec] = (zf(h, f), af(h, f))
            assert torch.equal(res["1"][0], res["0"][0]) and torch.equal(res["1"][1], res["0"][1])
            if kind == "int":
                g, a = H(res["1"][0]), H(res["1"][1])
                for i, q in enumerate(posets_):
                    s0, e0 = offs[i], offs[i + 1]
                    R = O.reachability(q.n, q.indptr, q.indices)
                    assert np.array_equal(g[s0:e0], O.zeta(R, H(f)[s0:e0]))
                    assert np.array_equal(a[s0:e0], O.zeta_adjoint(R, H(f)[s0:e0]))


@pytest.mark.parametrize("B", [4, 16])
def test_offsets_32_and_64_bit(px, B, monkeypatch):
    """The narrow scans, flat scans and combine address matrices with 32-bit offsets when
    every offset fits (the usual case) and with 64-bit offsets otherwise; both forms give
    the same values bit for bit (POSETX_O32=0 forces 64-bit), in node and row layout, and
    equal the closure oracle."""
    import torch
    p = W.chain_poset(3000, 30, 3, seed=40 + B)
    P = build(px, p)
    R = O.reachability(p.n, p.indptr, p.indices)
    f = W.functions(p.n, B, "int", seed=B, lo=-10**6, hi=10**6)
    perm = torch.from_numpy(P.rows()).to(dev())
    res = {}
    for o32 in ("1", "0"):
        monkeypatch.setenv("POSETX_O32", o32)
        for flat in ("1", "0"):
            monkeypatch.setenv("POSETX_SCAN_FLAT", flat)
            P.set_layout("nodes")
            g, a = px.zeta(P, T(f)), px.zeta_adjoint(P, T(f))
            P.set_layout("rows")
            fr = torch.empty_like(T(f))
            fr[perm] = T(f)
            gr, ar = px.zeta(P, fr), px.zeta_adjoint(P, fr)
            P.set_layout("nodes")
            assert torch.equal(gr[perm], g) and torch.equal(ar[perm], a)
            res[o32 + flat] = (H(g), H(a))
    for key, (g, a) in res.items():
        assert np.array_equal(g, O.zeta(R, f)), key
        assert np.array_equal(a, O.zeta_adjoint(R, f)), key


def test_table_builders_thread_count_independent(px, monkeypatch):
    """The walk, compact and run tables (built on host threads) are the same for one
    thread and for several: equal table statistics and bit-equal int64 zeta, adjoint and
    Möbius results, which also match the oracle on sampled elements."""
    import torch
    p = W.chain_poset(1 << 16, 24, 3, seed=31)
    f = W.functions(p.n, 8, "int", seed=32, lo=-1000, hi=1000)
    keys = ("walk_runs", "walk_events", "walk_snapshots", "walk_rows_distinct", "walk_row_loads", "run_chunks",
            "run_events")
    res = {}
    for thr in ("1", "5"):
        monkeypatch.setenv("POSETX_PREP_THREADS", thr)
        P = build(px, p)
        info = P.info_dict()
        res[thr] = ({k: info[k] for k in keys}, H(px.zeta(P, T(f))), H(px.zeta_adjoint(P, T(f))),
                    H(px.mobius(P, px.zeta(P, T(f)))))
    assert res["1"][0] == res["5"][0]
    for a, b in zip(res["1"][1:], res["5"][1:]):
        assert np.array_equal(a, b)
    assert np.array_equal(res["5"][3], f)
    nodes = np.random.default_rng(33).choice(p.n, 8, replace=False)
    assert np.array_equal(res["5"][1][nodes], O.zeta_at(p.n, p.indptr, p.indices, f, nodes))


# ------------------------------------------------------------ error handling
def test_argument_errors_and_nonfinite(px, cfg0):
    import torch
    p, _ = cfg0
    P = build(px, p)
    f = T(W.functions(p.n, 4, "normal", seed=1))
    with pytest.raises(px.PosetxError) as e:
        px.mobius(P, f, out=f)
    assert e.value.name == "PX_EINVAL"
    with pytest.raises(ValueError):
        px.zeta(P, f[:10])
    c = W.chain_only(4)
    Pc = build(px, c)
    g = T(np.array([[3e38], [-3e38], [3e38], [-3e38]], np.float32))
    with pytest.raises(px.PosetxError) as e:
        px.mobius(Pc, g, max_refine=2, tol=1e-6)
    assert e.value.name == "PX_ENONFINITE"
    # the default call (tol = 0) checks the result once it has run; float64 too
    for kw in ({}, {"max_refine": 0}):
        with pytest.raises(px.PosetxError) as e:
            px.mobius(Pc, g, **kw)
        assert e.value.name == "PX_ENONFINITE"
    g64 = T(np.array([[1e308], [-1e308], [1e308], [-1e308]]))
    with pytest.raises(px.PosetxError) as e:
        px.mobius(Pc, g64)
    assert e.value.name == "PX_ENONFINITE"
    with pytest.raises(px.PosetxError) as e:
        px.mobius_adjoint(Pc, g64)
    assert e.value.name == "PX_ENONFINITE"
    # tol < 0: asynchronous, no value checks; the overflow is in the result
    out = px.mobius(Pc, g64, tol=-1.0)
    assert not np.isfinite(H(out)).all()
    # the autograd backward through Möbius raises instead of returning Inf
    from paper_2211_13706_amd.autograd import mobius_fn
    x = T(np.array([[1.0], [2.0], [3.0], [4.0]])).requires_grad_(True)
    with pytest.raises(px.PosetxError):
        (mobius_fn(Pc, x) * g64).sum().backward()
    torch.cuda.synchronize()


def test_broadcast_inputs_and_checked_outputs(px, cfg0):
    """Inputs whose rows overlap in memory (a broadcast row, stride 0) are copied before the
    library reads n rows at the leading dimension; outputs of the wrong shape, dtype or
    layout are rejected for every transform, single and batched."""
    import torch
    p, R = cfg0
    P = build(px, p)
    row = W.functions(1, 64, "int", seed=90, lo=-100, hi=100)
    fb = T(row).expand(p.n, 64)
    assert fb.stride(0) == 0
    full = np.repeat(row, p.n, axis=0)
    assert np.array_equal(H(px.zeta(P, fb)), O.zeta(R, full))
    assert np.array_equal(H(px.mobius(P, fb)), O.mobius_by_substitution(R, full))
    assert np.array_equal(H(px.zeta_adjoint(P, T(row[:, :5]).expand(p.n, 5))), O.zeta_adjoint(R, full[:, :5]))
    f = T(full)
    bad_outs = [torch.empty(p.n, 32, dtype=torch.int64, device=dev()),
                torch.empty(p.n, 64, dtype=torch.float32, device=dev()),
                torch.empty(p.n - 1, 64, dtype=torch.int64, device=dev()),
                torch.empty(1, 64, dtype=torch.int64, device=dev()).expand(p.n, 64),
                torch.empty(64, p.n, dtype=torch.int64, device=dev()).t()]
    for o in bad_outs:
        for fn in (px.zeta, px.zeta_adjoint, px.mobius, px.mobius_adjoint):
            with pytest.raises(ValueError):
                fn(P, f, out=o)
    posets = W.batched_posets(3, seed=91, nmin=50, nmax=200)
    b = px.batch_build([build(px, q) for q in posets])
    fbat = T(row).expand(b.rows, 64)
    g = H(px.zeta_batched(b, fbat))
    fullb = np.repeat(row, b.rows, axis=0)
    for i, q in enumerate(posets):
        s0, e0 = b.offsets[i], b.offsets[i + 1]
        assert np.array_equal(g[s0:e0], O.zeta(O.reachability(q.n, q.indptr, q.indices), fullb[s0:e0]))
    for o in (torch.empty(b.rows, 63, dtype=torch.int64, device=dev()),
              torch.empty(1, 64, dtype=torch.int64, device=dev()).expand(b.rows, 64)):
        for fn in (px.zeta_batched, px.zeta_adjoint_batched):
            with pytest.raises(ValueError):
                fn(b, T(fullb), out=o)


# --------------------------------------------------------------- autotuner
def test_autotune_keeps_results_exact(px, cfg0):
    p, R = cfg0
    f = W.functions(p.n, 64, "int", seed=50, lo=-100, hi=100)
    want = O.zeta(R, f)
    for B in (64, 16):
        P = build(px, p)
        rep = P.autotune(__import__("torch").int64, B)
        assert rep["walk_T"] in (64, 128, 256) and rep["walk_emax"] in (48, 96, 192)
        assert rep["ms_best"] > 0
        assert P.info["walk_T"] == rep["walk_T"]
        fb = f[:, :B]
        assert np.array_equal(H(px.zeta(P, T(fb))), want[:, :B])
        assert np.array_equal(H(px.mobius(P, px.zeta(P, T(fb)))), fb)
        assert np.array_equal(H(px.zeta_adjoint(P, T(fb))), O.zeta_adjoint(R, fb))
        again = build(px, p).autotune(__import__("torch").int64, B)
        assert again["from_cache"] == 1 and again["walk_T"] == rep["walk_T"]
    posets = W.batched_posets(6, seed=51, nmin=100, nmax=800)
    b = px.batch_build([build(px, q) for q in posets])
    rb = b.autotune(__import__("torch").int64, 8)
    assert rb["rhs_tile"] in (0, 16, 32, 64)
    fx = W.functions(b.rows, 8, "int", seed=52, lo=-100, hi=100)
    g = H(px.zeta_batched(b, T(fx)))
    for i, q in enumerate(posets):
        s, e = b.offsets[i], b.offsets[i + 1]
        Rq = O.reachability(q.n, q.indptr, q.indices)
        assert np.array_equal(g[s:e], O.zeta(Rq, fx[s:e]))


# ------------------------------------------------------ sparse niv rows (CSR)
@pytest.fixture(scope="module")
def er2k():
    """Erdős–Rényi DAGs of average degree 4 and 6 (the workload of §5), n = 2000:
    widths 300-400, so the niv maps are kept as rows of their finite entries."""
    out = {}
    for deg in (4, 6):
        p = W.er_dag(2000, deg, seed=5)
        out[deg] = (p, O.reachability(p.n, p.indptr, p.indices))
    return out


@pytest.mark.parametrize("deg", [4, 6])
@pytest.mark.parametrize("B", [1, 8, 64, 100])
def test_er_dag_sparse_niv_int64_exact(px, er2k, deg, B):
    p, R = er2k[deg]
    P = build(px, p, planted=False)
    assert P.info_dict()["niv_sparse"] == 1 and P.k > 256
    f = W.functions(p.n, B, "int", seed=20 + B, lo=-100, hi=100)
    ft = T(f)
    g = H(px.zeta(P, ft))
    assert np.array_equal(g, O.zeta(R, f))
    assert np.array_equal(H(px.zeta_adjoint(P, ft)), O.zeta_adjoint(R, f))
    assert np.array_equal(H(px.mobius(P, T(g))), f)
    gr = W.functions(p.n, B, "int", seed=40 + B, lo=-1000, hi=1000)
    assert np.array_equal(H(px.mobius(P, T(gr))), O.mobius_by_substitution(R, gr))
    assert np.array_equal(H(px.mobius_adjoint(P, T(gr))), O.mobius_adjoint_by_substitution(R, gr))


@pytest.mark.parametrize("deg", [4, 6])
@pytest.mark.parametrize("B", [1, 33, 64])
def test_er_dag_sparse_niv_float(px, er2k, deg, B):
    """float32 zeta within the compensated-scan bound, float64 to 1e-12, and the refined
    float32 Möbius to 1e-5 (max|M r|/max|r| is 41 and 196 on these DAGs: well-posed)."""
    p, R = er2k[deg]
    P = build(px, p, planted=False)
    f = W.functions(p.n, B, "normal", seed=60 + B)
    fa = np.abs(f).astype(np.float64)
    check_f32_zeta(H(px.zeta(P, T(f))), O.zeta(R, f, exact=False), O.zeta(R, fa, exact=False))
    check_f32_zeta(H(px.zeta_adjoint(P, T(f))), O.zeta_adjoint(R, f, exact=False),
                   O.zeta_adjoint(R, fa, exact=False))
    f64 = f.astype(np.float64)
    assert rel(H(px.zeta(P, T(f64))), O.zeta(R, f64, exact=False)) <= 1e-12
    g64 = O.zeta(R, f64, exact=False)
    assert rel(H(px.mobius(P, T(g64))), f64) <= 1e-12
    g = W.functions(p.n, B, "uniform", seed=80 + B, lo=-1, hi=1)
    want = O.mobius(R, g.astype(np.float64), exact=False)
    got = H(px.mobius(P, T(g), max_refine=3))
    assert rel(got, want) <= 1e-5
    wantT = O.mobius_adjoint(R, g.astype(np.float64), exact=False)
    assert rel(H(px.mobius_adjoint(P, T(g), max_refine=3)), wantT) <= 1e-5


@pytest.mark.parametrize("case", ["cfg0", "lattice"])
@pytest.mark.parametrize("B", [5, 64])
def test_forced_sparse_niv_matches_dense(px, cfg0, case, B):
    """PX_BUILD_SPARSE_NIV on posets that default to dense rows: the same int64 results,
    and the same float64 Möbius bit for bit (both solves subtract the same terms in
    chain order, one at a time)."""
    p = cfg0[0] if case == "cfg0" else W.boolean_lattice(8)
    planted = case == "cfg0"
    A = build(px, p, planted=planted)
    S = build(px, p, planted=planted, flags=px.PX_BUILD_SPARSE_NIV)
    assert A.info_dict()["niv_sparse"] == 0 and S.info_dict()["niv_sparse"] == 1
    f = W.functions(p.n, B, "int", seed=90 + B, lo=-1000, hi=1000)
    ft = T(f)
    for fn in (px.zeta, px.zeta_adjoint, px.mobius, px.mobius_adjoint):
        assert np.array_equal(H(fn(A, ft)), H(fn(S, ft)))
    g = T(W.functions(p.n, B, "normal", seed=95 + B).astype(np.float64))
    assert np.array_equal(H(px.mobius(A, g)), H(px.mobius(S, g)))
    assert np.array_equal(H(px.mobius_adjoint(A, g)), H(px.mobius_adjoint(S, g)))


def test_sparse_niv_poset_not_batchable(px, er2k):
    p, _ = er2k[4]
    P = build(px, p, planted=False)
    with pytest.raises(px.PosetxError) as ei:
        px.batch_build([P])
    assert ei.value.name == "PX_EUNSUPPORTED"


def test_er_dag_sparse_niv_n65536_sampled(px):
    """n = 2^16, average degree 4 (k ~ 13,000, 14M niv entries; dense rows would take
    3.5 GB): float32 zeta at sampled nodes against down-set sums, int64 round trip exact."""
    p = W.er_dag(1 << 16, 4, seed=1)
    P = build(px, p, planted=False)
    assert P.info_dict()["niv_sparse"] == 1
    rng = np.random.default_rng(3)
    nodes = rng.choice(p.n, 8, replace=False)
    f = W.functions(p.n, 64, "normal", seed=5)
    g = H(px.zeta(P, T(f)))[nodes]
    check_f32_zeta(g, O.zeta_at(p.n, p.indptr, p.indices, f, nodes),
                   O.zeta_at(p.n, p.indptr, p.indices, np.abs(f), nodes))
    wT = H(px.zeta_adjoint(P, T(f)))[nodes]
    check_f32_zeta(wT, O.zeta_adjoint_at(p.n, p.indptr, p.indices, f, nodes),
                   O.zeta_adjoint_at(p.n, p.indptr, p.indices, np.abs(f), nodes))
    fi = W.functions(p.n, 16, "int", seed=6, lo=-(2**40), hi=2**40)
    gi = px.zeta(P, T(fi))
    assert np.array_equal(H(px.mobius(P, gi)), fi)
    assert np.array_equal(H(px.mobius_adjoint(P, px.zeta_adjoint(P, T(fi)))), fi)


# ------------------------------------------- niv maps computed on the device
def _host_only(px, p, planted):
    return px.poset_build(p.n, p.indptr, p.indices, p.chain_of if planted else None,
                          p.chain_pos if planted else None, flags=px.PX_BUILD_HOST_ONLY)


@pytest.mark.parametrize("case", ["example", "cfg0", "cfg0_matching", "grid", "lattice", "random", "antichain",
                                  "chain", "batched_small"])
def test_device_niv_equals_host_recursion(px, case, monkeypatch):
    """The device fixed point of the chain recursion gives the host recursion's maps
    (Theorem 5), for both directions, and the same level schedules."""
    monkeypatch.setenv("POSETX_PREP", "device")
    p, planted = {
        "example": (W.worked_example(), True), "cfg0": (W.chain_poset(2000, 16, 4, seed=0), True),
        "cfg0_matching": (W.chain_poset(2000, 16, 4, seed=0), False), "grid": (W.grid_poset(150, 20), True),
        "lattice": (W.boolean_lattice(8), False), "random": (W.random_small_dag(400, 0.02, 5), False),
        "antichain": (W.antichain(100), False), "chain": (W.chain_only(500, seed=2), True),
        "batched_small": (W.batched_posets(1, seed=4, nmin=3000, nmax=3000)[0], True)}[case]
    if planted and p.chain_of is None:
        planted = False
    Hh = _host_only(px, p, planted)
    D = build(px, p, planted=planted)
    info = D.info_dict()
    assert info["niv_sparse"] == 0 and info["niv_device_rounds"] >= 1
    # against the oracle: niv_j(x) read off the closure by its definition (§2.4); the dual
    # map is the same definition on the reversed order, with chain positions reversed
    R = O.reachability(p.n, p.indptr, p.indices)
    co, cp = D.chains()
    lens = np.bincount(co, minlength=D.k)
    want = {False: O.niv_from_closure(R, co, cp, D.k),
            True: O.niv_from_closure(np.ascontiguousarray(R.T), co, lens[co] - 1 - cp, D.k)}
    for up in (False, True):
        got = D.niv(up)
        assert np.array_equal(got, want[up])
        assert np.array_equal(got, Hh.niv(up))
        # the Möbius schedule respects every dependency of the U-solve: each other-chain
        # entry of a row lies on an earlier level
        lev = D.levels(up)
        x, j = np.nonzero(got >= 0)
        other = co[got[x, j]] != co[x]
        assert (lev[got[x, j]][other] < lev[x][other]).all()
        assert np.array_equal(lev, Hh.levels(up))
    assert info["nnz_niv"] == int((want[False] >= 0).sum()) and info["nnz_niv_up"] == int((want[True] >= 0).sum())


@pytest.mark.parametrize("case", ["cfg0", "grid", "er_d4"])
def test_device_levels_persistent_and_by_height(px, case, monkeypatch):
    """The U-dependency levels computed on the device in one persistent launch (the
    default), height by height (POSETX_UDEP=heights), and height by height after every
    wait of the persistent launch gave up (a spin limit of 0) all equal the host's, for
    dense rows and for sparse rows, both maps."""
    monkeypatch.setenv("POSETX_PREP", "device")
    p, flags = {"cfg0": (W.chain_poset(3000, 16, 4, seed=8), 0), "grid": (W.grid_poset(120, 24), 0),
                "er_d4": (W.er_dag(2000, 4, seed=9), px.PX_BUILD_SPARSE_NIV)}[case]
    planted = p.chain_of is not None
    co = p.chain_of if planted else None
    cp = p.chain_pos if planted else None
    Hh = px.poset_build(p.n, p.indptr, p.indices, co, cp, flags=flags | px.PX_BUILD_HOST_ONLY)
    for env in ({}, {"POSETX_UDEP": "heights"}, {"POSETX_FLOW_SPIN": "0"}):
        for key in ("POSETX_UDEP", "POSETX_FLOW_SPIN"):
            monkeypatch.delenv(key, raising=False)
        for key, val in env.items():
            monkeypatch.setenv(key, val)
        D = px.poset_build(p.n, p.indptr, p.indices, co, cp, flags=flags, device=0)
        assert D.info_dict()["niv_device_rounds"] >= 1
        for up in (False, True):
            assert np.array_equal(D.levels(up), Hh.levels(up)), (case, env, up)


@pytest.mark.parametrize("case", ["er_d4", "er_d6", "example", "lattice", "cfg0", "random", "antichain", "chain"])
def test_device_sparse_niv_rows_match_oracle(px, case, monkeypatch):
    """The sparse niv rows merged on the device, height after height (both maps),
    against the closure oracle's niv (§2.4) and the host recursion's rows; the
    transforms on those rows are exact (int64, against the oracle)."""
    monkeypatch.setenv("POSETX_PREP", "device")
    p, planted = {
        "er_d4": (W.er_dag(2000, 4, seed=2), False), "er_d6": (W.er_dag(1500, 6, seed=7), False),
        "example": (W.worked_example(), True), "lattice": (W.boolean_lattice(8), False),
        "cfg0": (W.chain_poset(2000, 16, 4, seed=0), True), "random": (W.random_small_dag(400, 0.02, 5), False),
        "antichain": (W.antichain(100), False), "chain": (W.chain_only(500, seed=2), True)}[case]
    D = build(px, p, planted=planted, flags=px.PX_BUILD_SPARSE_NIV)
    info = D.info_dict()
    assert info["niv_sparse"] == 1 and info["niv_device_rounds"] >= 1
    Hh = px.poset_build(p.n, p.indptr, p.indices, p.chain_of if planted else None, p.chain_pos if planted else None,
                        flags=px.PX_BUILD_HOST_ONLY | px.PX_BUILD_SPARSE_NIV)
    R = O.reachability(p.n, p.indptr, p.indices)
    co, cp = D.chains()
    lens = np.bincount(co, minlength=D.k)
    want = {False: O.niv_from_closure(R, co, cp, D.k),
            True: O.niv_from_closure(np.ascontiguousarray(R.T), co, lens[co] - 1 - cp, D.k)}
    for up in (False, True):
        ptr, nodes = D.niv_csr(up)
        hptr, hnodes = Hh.niv_csr(up)
        assert np.array_equal(ptr, hptr) and np.array_equal(nodes, hnodes)
        assert np.array_equal(D.niv(up), want[up])
        assert np.array_equal(D.levels(up), Hh.levels(up))
    f = W.functions(p.n, 8, "int", seed=3, lo=-1000, hi=1000)
    assert np.array_equal(H(px.zeta(D, T(f))), O.zeta(R, f))
    assert np.array_equal(H(px.zeta_adjoint(D, T(f))), O.zeta_adjoint(R, f))
    assert np.array_equal(H(px.mobius(D, T(f))), O.mobius_by_substitution(R, f))


def test_device_sparse_niv_rejects_unordered_chains(px, monkeypatch):
    """The device merge checks planted chains as the host recursion does."""
    monkeypatch.setenv("POSETX_PREP", "device")
    p = W.worked_example()
    co, cp = p.chain_of.copy(), p.chain_pos.copy()
    co[[4, 5]] = co[[5, 4]]; cp[[4, 5]] = cp[[5, 4]]     # x5 and x6 are incomparable
    with pytest.raises(px.PosetxError) as ei:
        px.poset_build(p.n, p.indptr, p.indices, co, cp, flags=px.PX_BUILD_SPARSE_NIV, device=0)
    assert ei.value.name == "PX_ECHAIN"
    cp2 = p.chain_pos.copy()
    c0 = np.nonzero(p.chain_of == 0)[0]; cp2[c0] = cp2[c0].max() - cp2[c0]
    with pytest.raises(px.PosetxError) as ei:
        px.poset_build(p.n, p.indptr, p.indices, p.chain_of, cp2, flags=px.PX_BUILD_SPARSE_NIV, device=0)
    assert ei.value.name == "PX_ECHAIN"


def test_device_sparse_niv_er_n64k_matches_host(px, monkeypatch):
    """ER n = 2^16, degree 4 (k = 13,243 chains, 13.8 M entries per map): the default
    build merges the rows on the device (n >= 2^16); they equal the host recursion's
    (POSETX_PREP=host), both maps, and the transforms agree bit for bit."""
    p = W.er_dag(1 << 16, 4, seed=1)
    D = px.poset_build(p.n, p.indptr, p.indices, device=0)
    assert D.info["niv_sparse"] == 1 and D.info["niv_device_rounds"] >= 1
    monkeypatch.setenv("POSETX_PREP", "host")
    Hh = px.poset_build(p.n, p.indptr, p.indices, device=0)
    assert Hh.info["niv_device_rounds"] == 0
    for up in (False, True):
        a, b = D.niv_csr(up), Hh.niv_csr(up)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    f = T(W.functions(p.n, 16, "int", seed=4, lo=-1000, hi=1000))
    assert np.array_equal(H(px.zeta(D, f)), H(px.zeta(Hh, f)))
    assert np.array_equal(H(px.mobius(D, f)), H(px.mobius(Hh, f)))


def test_device_niv_config1_and_host_switch(px, cfg1, monkeypatch):
    """n = 2^20, k = 64: the device maps equal the host's; POSETX_PREP=host selects the host recursion."""
    p, _ = cfg1
    D = build(px, p)
    rounds = D.info_dict()["niv_device_rounds"]
    assert 2 <= rounds <= 64
    Hh = _host_only(px, p, True)
    assert np.array_equal(D.niv(), Hh.niv())
    assert np.array_equal(D.niv(True), Hh.niv(True))
    # finite entries counted on host threads from the device maps
    di, hi = D.info_dict(), Hh.info_dict()
    assert di["nnz_niv"] == hi["nnz_niv"] == int((Hh.niv() >= 0).sum())
    assert di["nnz_niv_up"] == hi["nnz_niv_up"]
    monkeypatch.setenv("POSETX_PREP", "host")
    assert build(px, W.chain_poset(2000, 16, 4, seed=0)).info_dict()["niv_device_rounds"] == 0
    monkeypatch.delenv("POSETX_PREP")
    # below 2^24 entries the host recursion is the default
    assert build(px, W.chain_poset(2000, 16, 4, seed=0)).info_dict()["niv_device_rounds"] == 0


def test_device_niv_rejects_unordered_chains(px, monkeypatch):
    """Planted chains that the DAG does not order are rejected by the device check too."""
    monkeypatch.setenv("POSETX_PREP", "device")
    p = W.worked_example()
    co, cp = p.chain_of.copy(), p.chain_pos.copy()
    co[[4, 5]] = co[[5, 4]]; cp[[4, 5]] = cp[[5, 4]]     # x5 and x6 are incomparable
    cp2 = p.chain_pos.copy()
    c0 = np.nonzero(p.chain_of == 0)[0]; cp2[c0] = cp2[c0].max() - cp2[c0]
    q = W.chain_poset(2000, 16, 4, seed=0)
    cq = q.chain_pos.copy()
    c3 = np.nonzero(q.chain_of == 3)[0]
    i, j = c3[np.argsort(cq[c3])][[500 // 16, 500 // 16 + 7]]
    cq[[i, j]] = cq[[j, i]]                               # two elements of one chain swapped
    for (n, indptr, indices, cof, cpos) in ((12, p.indptr, p.indices, co, cp), (12, p.indptr, p.indices, p.chain_of, cp2),
                                            (q.n, q.indptr, q.indices, q.chain_of, cq)):
        with pytest.raises(px.PosetxError) as ei:
            px.poset_build(n, indptr, indices, cof, cpos, device=0)
        assert ei.value.name == "PX_ECHAIN"


@pytest.mark.parametrize("B", [1, 5, 64, 100])
def test_refine_report_residual_matches_host(px, B):
    """The report's backward error max_col ||g - zeta(f)||_inf / ||g||_inf (zeta in float64 of
    the returned float32 f) equals the same quantity from the oracle's exact zeta.  An unrefined
    solve on a 64 x 16 grid keeps the residual (~1e-7) far above float64 rounding (~1e-14)."""
    p = W.grid_poset(64, 16)
    R = O.reachability(p.n, p.indptr, p.indices)
    P = build(px, p)
    g = W.functions(p.n, B, "uniform", seed=120 + B, lo=-1, hi=1)
    got, rep = px.mobius(P, T(g), max_refine=0, report=True)
    fh = H(got).astype(np.float64)
    r = g.astype(np.float64) - O.zeta(R, fh)
    want = float((np.abs(r).max(axis=0) / np.abs(g).astype(np.float64).max(axis=0)).max())
    assert want > 0 and abs(rep["residual"] - want) <= 1e-4 * want, (rep, want)
    assert not rep["nonfinite"] and rep["iterations"] == 0


@pytest.mark.parametrize("case", ["example", "chain", "antichain", "grid"])
def test_forced_sparse_niv_small_posets_exact(px, case):
    """Sparse rows on degenerate shapes (one chain, no relations, the worked example, a grid):
    int64 zeta, Möbius and both adjoints bit-exact against the closure."""
    p, planted = {"example": (W.worked_example(), True), "chain": (W.chain_only(300, seed=1), True),
                  "antichain": (W.antichain(77), False), "grid": (W.grid_poset(40, 9), True)}[case]
    R = O.reachability(p.n, p.indptr, p.indices)
    S = build(px, p, planted=planted, flags=px.PX_BUILD_SPARSE_NIV)
    assert S.info_dict()["niv_sparse"] == 1
    for B in (1, 64):
        f = W.functions(p.n, B, "int", seed=7 + B, lo=-(2**40), hi=2**40)
        ft = T(f)
        assert np.array_equal(H(px.zeta(S, ft)), O.zeta(R, f))
        assert np.array_equal(H(px.zeta_adjoint(S, ft)), O.zeta_adjoint(R, f))
        assert np.array_equal(H(px.mobius(S, ft)), O.mobius_by_substitution(R, f))
        assert np.array_equal(H(px.mobius_adjoint(S, ft)), O.mobius_adjoint_by_substitution(R, f))


@pytest.mark.parametrize("case", ["cfg0", "er"])
def test_saved_poset_loads_on_device(px, case, tmp_path):
    """A handle loaded from a saved file (no preprocessing) gives the oracle's transforms."""
    p, planted = {"cfg0": (W.chain_poset(2000, 16, 4, seed=0), True), "er": (W.er_dag(2000, 4, seed=5), False)}[case]
    A = build(px, p, planted=planted)
    path = tmp_path / "p.pxposet"
    A.save(path)
    del A
    L = px.poset_load(path, device=0)
    assert L.info_dict()["niv_sparse"] == (1 if case == "er" else 0)
    R = O.reachability(p.n, p.indptr, p.indices)
    for B in (1, 64):
        f = W.functions(p.n, B, "int", seed=3 + B, lo=-1000, hi=1000)
        ft = T(f)
        assert np.array_equal(H(px.zeta(L, ft)), O.zeta(R, f))
        assert np.array_equal(H(px.zeta_adjoint(L, ft)), O.zeta_adjoint(R, f))
        assert np.array_equal(H(px.mobius(L, ft)), O.mobius_by_substitution(R, f))
        assert np.array_equal(H(px.mobius_adjoint(L, ft)), O.mobius_adjoint_by_substitution(R, f))


def test_poset_methods_match_functions(px, cfg0):
    """Poset.zeta / zeta_T / mobius / mobius_T are the module functions."""
    p, R = cfg0
    P = build(px, p)
    f = W.functions(p.n, 3, "int", seed=200, lo=-100, hi=100)
    ft = T(f)
    assert np.array_equal(H(P.zeta(ft)), O.zeta(R, f))
    assert np.array_equal(H(P.zeta_T(ft)), O.zeta_adjoint(R, f))
    assert np.array_equal(H(P.mobius(ft)), O.mobius_by_substitution(R, f))
    assert np.array_equal(H(P.mobius_T(ft)), O.mobius_adjoint_by_substitution(R, f))


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("sparse", [False, True])
def test_random_dags_int64_exact(px, seed, sparse):
    """Random DAGs of varied size and density (chains from the matching), dense and sparse
    rows, narrow and wide RHS: every transform bit-exact against the closure."""
    n, prob = [(60, 0.2), (200, 0.05), (333, 0.02), (128, 0.5), (500, 0.01), (257, 0.08)][seed]
    p = W.random_small_dag(n, prob, 100 + seed)
    R = O.reachability(p.n, p.indptr, p.indices)
    P = build(px, p, planted=False, flags=px.PX_BUILD_SPARSE_NIV if sparse else 0)
    for B in (1, 65):
        f = W.functions(p.n, B, "int", seed=300 + seed, lo=-(2**50), hi=2**50)
        ft = T(f)
        assert np.array_equal(H(px.zeta(P, ft)), O.zeta(R, f))
        assert np.array_equal(H(px.zeta_adjoint(P, ft)), O.zeta_adjoint(R, f))
        assert np.array_equal(H(px.mobius(P, ft)), O.mobius_by_substitution(R, f))
        assert np.array_equal(H(px.mobius_adjoint(P, ft)), O.mobius_adjoint_by_substitution(R, f))


@pytest.mark.parametrize("sparse", [False, True])
def test_empty_and_single_element_posets(px, sparse):
    """Degenerate sizes: no elements (every call succeeds and touches nothing), one element
    (zeta and Möbius are the identity), two comparable elements."""
    import torch
    flags = px.PX_BUILD_SPARSE_NIV if sparse else 0
    E = px.poset_build(0, np.zeros(1, np.int64), np.zeros(0, np.int32), flags=flags, device=0)
    z = torch.zeros((0, 3), dtype=torch.int64, device=dev())
    for fn in (px.zeta, px.zeta_adjoint, px.mobius, px.mobius_adjoint):
        assert fn(E, z).shape == (0, 3)
    one = W.antichain(1)
    S = build(px, one, planted=False, flags=flags)
    f = W.functions(1, 5, "int", seed=1, lo=-9, hi=9)
    for fn in (px.zeta, px.zeta_adjoint, px.mobius, px.mobius_adjoint):
        assert np.array_equal(H(fn(S, T(f))), f)
    two = W.chain_only(2)
    R = O.reachability(two.n, two.indptr, two.indices)
    C = build(px, two, flags=flags)
    f2 = W.functions(2, 70, "int", seed=2, lo=-9, hi=9)
    assert np.array_equal(H(px.zeta(C, T(f2))), O.zeta(R, f2))
    assert np.array_equal(H(px.mobius(C, T(f2))), O.mobius_by_substitution(R, f2))
