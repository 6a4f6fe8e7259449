"""Pins of the CPU oracle against facts the paper and mathematics fix.

Each test ties an oracle function to something other than itself: the
printed matrices of the paper's worked example, closed forms (chain,
antichain, Boolean lattice, grid), an independent algorithm (Yates' subset
sum), or brute-force invariants on small random DAGs.  A dropped term, a
wrong sign or index, or a transposed operand in the oracle fails at least
one of these.
"""

import itertools
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


# ---------------------------------------------------------------- helpers
def _rows_to_dense(rows, n=12, signed=False):
    M = np.zeros((n, n), dtype=np.int64)
    for r, cols in rows.items():
        for c in cols:
            if signed:
                M[int(r) - 1, c[0] - 1] = c[1]
            else:
                M[int(r) - 1, c - 1] = 1
    return M


@pytest.fixture(scope="module")
def ex():
    p = W.worked_example()
    R = O.reachability(p.n, p.indptr, p.indices)
    return p, R


# ------------------------------------------------------- worked example
def test_example_cover_graph_matches_print(ex, golden_example):
    p, _ = ex
    A = np.zeros((12, 12), np.int64)
    src, dst = p.edges()
    A[src, dst] = 1
    assert np.array_equal(A, _rows_to_dense(golden_example["cover_graph_A"]["rows"]))


def test_example_closure_is_printed_Z(ex, golden_example):
    _, R = ex
    assert np.array_equal(R.astype(np.int64), _rows_to_dense(golden_example["zeta_Z"]["rows"]))
    assert O.is_acyclic(R)


def test_example_mobius_matrix_is_printed_M(ex, golden_example):
    _, R = ex
    M = O.mobius_matrix(R)
    assert np.array_equal(M, _rows_to_dense(golden_example["mobius_M"]["rows"], signed=True))
    assert np.array_equal(M @ R.astype(np.int64), np.eye(12, dtype=np.int64))


def test_example_niv_is_printed_N(ex, golden_example):
    p, R = ex
    niv = O.niv_from_closure(R, p.chain_of, p.chain_pos, 4)
    want = np.array([golden_example["niv_N"]["rows"][str(i)] for i in range(1, 13)]) - 1
    assert np.array_equal(niv, want)
    assert int((niv >= 0).sum()) == golden_example["niv_N"]["nnz"]
    assert list(niv[3] + 1) == golden_example["niv_of_4"]["values"]
    assert list(np.nonzero(R[3])[0] + 1) == golden_example["out_of_4"]["values"]


def test_example_factorisation_Z_equals_UV(ex, golden_example):
    """Z = U V (Eq. zfac) with U from niv and V from the chains, as printed."""
    p, R = ex
    niv = O.niv_from_closure(R, p.chain_of, p.chain_pos, 4)
    U = np.zeros((12, 12), np.int64)
    for x in range(12):
        for y in niv[x]:
            if y >= 0:
                U[x, y] = 1
    V = np.zeros((12, 12), np.int64)
    for x in range(12):
        for y in range(12):
            if p.chain_of[x] == p.chain_of[y] and p.chain_pos[y] <= p.chain_pos[x]:
                V[x, y] = 1
    assert np.array_equal(U, _rows_to_dense(golden_example["factor_U"]["rows"]))
    assert np.array_equal(V, _rows_to_dense(golden_example["factor_V"]["rows"]))
    assert np.array_equal(U @ V, R.astype(np.int64))
    Vinv = np.rint(np.linalg.inv(V)).astype(np.int64)
    want = np.eye(12, dtype=np.int64)
    for r, c in golden_example["inverse_Vinv"]["minus_one_at"].items():
        want[int(r) - 1, c - 1] = -1
    assert np.array_equal(Vinv, want)


def test_example_permutation_blocks_V(ex, golden_example):
    """P maps block position -> element; P V P^-1 is block upper-triangular ones (Eq. exb)."""
    p, R = ex
    perm = list(range(1, 13))
    for cyc in golden_example["permutation_P"]["cycles"]:
        for a, b in zip(cyc, cyc[1:] + cyc[:1]):
            perm[a - 1] = b
    elem = np.array(perm) - 1                      # elem[position] = element
    V = np.array([[1 if (p.chain_of[x] == p.chain_of[y] and p.chain_pos[y] <= p.chain_pos[x]) else 0
                   for y in range(12)] for x in range(12)])
    Bm = V[np.ix_(elem, elem)]
    want = np.zeros((12, 12), np.int64)
    o = 0
    for s in golden_example["permutation_P"]["block_sizes"]:
        want[o:o + s, o:o + s] = np.triu(np.ones((s, s), np.int64))
        o += s
    assert np.array_equal(Bm, want)
    tops = [[c - 1 for c in ch] for ch in golden_example["chains"]["top_first"]]
    assert [list(elem[o:o + len(ch)]) for o, ch in zip(np.cumsum([0, 4, 3, 2]), tops)] == tops


def test_example_operation_counts(ex, golden_example):
    p, R = ex
    niv = O.niv_from_closure(R, p.chain_of, p.chain_pos, 4)
    n, k = 12, 4
    oc = golden_example["op_counts"]
    assert n - k == oc["V_adds"]
    assert int((niv >= 0).sum()) - n == oc["U_adds"]
    assert oc["V_adds"] + oc["U_adds"] == oc["total"]
    # the printed direct count (39) disagrees with nnz(Z) - n; the count is 40
    assert int(R.sum()) - n == oc["direct_counted_nnzZ_minus_n"] == oc["direct_printed"] + 1


def test_example_mirsky_levels(ex, golden_example):
    _, R = ex
    lev = O.mirsky_levels(R)
    assert lev.max() + 1 == golden_example["longest_chain"]["levels"]
    chain = [c - 1 for c in golden_example["longest_chain"]["chain"]]
    assert list(lev[chain]) == [4, 3, 2, 1, 0]
    # the alternative partition printed in §4 is valid too: every element strictly
    # above another sits on a strictly higher level
    alt = lev.copy()
    for x in golden_example["levels_alternative"]["L3"]:
        alt[x - 1] = 2
    for x in golden_example["levels_alternative"]["L4"]:
        alt[x - 1] = 3
    for x, y in itertools.product(range(12), range(12)):
        if x != y and R[x, y]:
            assert alt[x] > alt[y] and lev[x] > lev[y]


def test_example_zeta_first_entry(ex):
    """g(x_1) = f(x_1) + f(x_3) + f(x_4) + f(x_6) + ... + f(x_12) (§2.2)."""
    _, R = ex
    f = (np.arange(12, dtype=np.int64) + 1)[:, None] ** 3
    g = O.zeta(R, f)
    assert g[0, 0] == sum(int(f[i - 1, 0]) for i in [1, 3, 4, 6, 7, 8, 9, 10, 11, 12])
    assert np.array_equal(O.mobius(R, g), f)
    assert np.array_equal(O.mobius_by_substitution(R, g), f)


# ---------------------------------------------------------- closed forms
@pytest.mark.parametrize("seed", [None, 3])
def test_chain_is_prefix_sum_and_first_difference(seed):
    p = W.chain_only(40, seed)
    R = O.reachability(p.n, p.indptr, p.indices)
    f = W.functions(p.n, 3, "int", seed=1, lo=-50, hi=50)
    order = np.argsort(p.chain_pos)                 # bottom first
    g = O.zeta(R, f)
    assert np.array_equal(g[order], np.cumsum(f[order], axis=0))
    adj = O.zeta_adjoint(R, f)
    assert np.array_equal(adj[order], np.cumsum(f[order][::-1], axis=0)[::-1])
    fo = f[order]
    diff = fo - np.vstack([np.zeros((1, 3), np.int64), fo[:-1]])
    assert np.array_equal(O.mobius(R, f)[order], diff)
    assert np.array_equal(O.mobius_by_substitution(R, f)[order], diff)
    up = fo - np.vstack([fo[1:], np.zeros((1, 3), np.int64)])
    assert np.array_equal(O.mobius_adjoint(R, f)[order], up)


def test_antichain_is_identity():
    p = W.antichain(17)
    R = O.reachability(p.n, p.indptr, p.indices)
    f = W.functions(17, 2, "normal", seed=2)
    assert np.array_equal(O.zeta(R, f), f.astype(np.float64))
    assert np.array_equal(O.mobius(R, f), f.astype(np.float64))
    assert np.array_equal(O.zeta_adjoint(R, f), f.astype(np.float64))


def _yates_subset_sum(f, m):
    """Yates' fast subset-sum transform: g(T) = Σ_{S ⊆ T} f(S) (§1, related work)."""
    g = f.astype(np.int64).copy()
    for e in range(m):
        bit = 1 << e
        for s in range(1 << m):
            if s & bit:
                g[s] += g[s ^ bit]
    return g


@pytest.mark.parametrize("m", [4, 6, 10])
def test_boolean_lattice_mu_closed_form_and_yates(m):
    p = W.boolean_lattice(m)
    R = O.reachability(p.n, p.indptr, p.indices)
    s = np.arange(p.n)
    sub = (s[:, None] & s[None, :]) == s[None, :]        # sub[T, S]: S ⊆ T
    assert np.array_equal(R, sub)
    if m <= 6:
        mu = O.mobius_function(R)
        pc = np.array([bin(v).count("1") for v in range(p.n)])
        # μ(S, T) = (-1)^{|T \ S|} for S ⊆ T, else 0
        want = np.where(sub.T, 1 - 2 * ((pc[None, :] - pc[:, None]) % 2), 0)
        assert np.array_equal(mu, want)
    f = W.functions(p.n, 2, "int", seed=m, lo=-9, hi=9)
    g = O.zeta(R, f)
    assert np.array_equal(g, _yates_subset_sum(f, m))
    assert np.array_equal(O.mobius_by_substitution(R, g), f)


def test_grid_is_2d_prefix_sum_and_finite_difference():
    h, w = 9, 6
    p = W.grid_poset(h, w)
    R = O.reachability(p.n, p.indptr, p.indices)
    f = W.functions(p.n, 2, "int", seed=5, lo=-20, hi=20)
    g = O.zeta(R, f)
    f3 = f.reshape(h, w, 2)
    assert np.array_equal(g.reshape(h, w, 2), f3.cumsum(0).cumsum(1))
    g3 = g.reshape(h, w, 2)
    pad = np.zeros((h + 1, w + 1, 2), np.int64); pad[1:, 1:] = g3
    fd = pad[1:, 1:] - pad[:-1, 1:] - pad[1:, :-1] + pad[:-1, :-1]
    assert np.array_equal(O.mobius(R, g).reshape(h, w, 2), fd)
    ff = W.functions(p.n, 2, "uniform", seed=6, lo=-1, hi=1)
    gf = O.zeta(R, ff)
    exp = ff.astype(np.float64).reshape(h, w, 2).cumsum(0).cumsum(1)
    assert np.allclose(gf.reshape(h, w, 2), exp, rtol=0, atol=1e-12)


# ------------------------------------------------- brute-force invariants
def _greedy_chains(R):
    """Any partition into chains: each element joins the first chain whose top is below it."""
    n = R.shape[0]
    tops, chain_of, chain_pos = [], np.empty(n, np.int32), np.empty(n, np.int32)
    for x in O.linear_extension(R):
        for c, t in enumerate(tops):
            if R[x, t[-1]]:
                t.append(x); chain_of[x] = c; chain_pos[x] = len(t) - 1
                break
        else:
            tops.append([x]); chain_of[x] = len(tops) - 1; chain_pos[x] = 0
    return chain_of, chain_pos, len(tops)


@pytest.mark.parametrize("seed", range(6))
def test_random_dag_invariants(seed):
    n = 24 + 7 * seed
    p = W.random_small_dag(n, 0.12, seed)
    R = O.reachability(p.n, p.indptr, p.indices)
    assert O.is_acyclic(R)
    # the closure is transitive and contains every edge
    assert np.array_equal(R, R | ((R.astype(int) @ R.astype(int)) > 0))
    src, dst = p.edges()
    assert R[src, dst].all()
    mu = O.mobius_function(R)
    assert np.array_equal(O.mobius_matrix(R, mu) @ R.astype(np.int64), np.eye(n, dtype=np.int64))
    f = W.functions(n, 3, "int", seed=seed, lo=-1000, hi=1000)
    g = O.zeta(R, f)
    assert np.array_equal(O.mobius(R, g, mu), f)
    assert np.array_equal(O.mobius_by_substitution(R, g), f)
    # adjoints are the transforms of the dual order (reversed edges)
    Rd = O.reachability(p.n, *_reverse_csr(p))
    assert np.array_equal(Rd, R.T)
    assert np.array_equal(O.zeta_adjoint(R, f), O.zeta(Rd, f))
    assert np.array_equal(O.mobius_adjoint(R, f, mu), O.mobius_by_substitution(Rd, f))
    assert np.array_equal(O.mobius_adjoint_by_substitution(R, O.zeta_adjoint(R, f)), f)
    # Theorem 4: out(x) is the disjoint union of the chain segments below niv_j(x)
    chain_of, chain_pos, k = _greedy_chains(R)
    niv = O.niv_from_closure(R, chain_of, chain_pos, k)
    for x in range(n):
        union = np.zeros(n, bool)
        for j in range(k):
            if niv[x, j] >= 0:
                seg = (chain_of == j) & (chain_pos <= chain_pos[niv[x, j]])
                assert not (union & seg).any()
                union |= seg
        assert np.array_equal(union, R[x])
        # Theorem 5: niv_j(x) is the highest niv_j over the children (own chain: x)
        kids = p.indices[p.indptr[x]:p.indptr[x + 1]]
        for j in range(k):
            if j == chain_of[x]:
                assert niv[x, j] == x
            else:
                vals = [niv[z, j] for z in kids if niv[z, j] >= 0]
                best = -1 if not vals else max(vals, key=lambda v: chain_pos[v])
                assert niv[x, j] == best


def _reverse_csr(p):
    src, dst = p.edges()
    order = np.argsort(dst, kind="stable")
    indptr = np.zeros(p.n + 1, np.int64)
    np.cumsum(np.bincount(dst, minlength=p.n), out=indptr[1:])
    return indptr, src[order].astype(np.int32)


@pytest.mark.parametrize("edges", [[(0, 1), (1, 0)], [(0, 1), (1, 2), (2, 0)], [(0, 1), (1, 2), (2, 3), (3, 1), (0, 4)]])
def test_is_acyclic_rejects_cycles(edges):
    """A directed cycle makes the reachability relation symmetric on its nodes (x ⪯ y and
    y ⪯ x with x != y), so it is not a partial order (§2.1); removing one edge of the
    cycle restores antisymmetry."""
    n = 1 + max(max(e) for e in edges)

    def csr(es):
        order = sorted(es)
        indptr = np.zeros(n + 1, np.int64)
        for u, _ in order:
            indptr[u + 1] += 1
        return np.cumsum(indptr), np.array([v for _, v in order], np.int32)

    R = O.reachability(n, *csr(edges))
    assert not O.is_acyclic(R)
    cyc = [e for e in edges if e != (0, 4)]
    assert O.is_acyclic(O.reachability(n, *csr([e for e in edges if e != cyc[-1]])))


def test_int64_wraps_modulo_2_64():
    p = W.chain_only(5)
    R = O.reachability(p.n, p.indptr, p.indices)
    big = 2**62 + 12345
    f = np.array([[big], [big], [-7], [big], [3]], dtype=np.int64)
    g = O.zeta(R, f)
    exact = np.cumsum([int(v) for v in f[:, 0]])
    want = [((int(v) + 2**63) % 2**64) - 2**63 for v in exact]
    assert list(g[:, 0]) == want
    assert np.array_equal(O.mobius_by_substitution(R, g), f)
    assert np.array_equal(O.mobius(R, g), f)


def test_fsum_exactness():
    p = W.antichain(1)
    # one element, three right-hand sides: trivial; exactness is exercised on a chain
    c = W.chain_only(3)
    R = O.reachability(c.n, c.indptr, c.indices)
    f = np.array([[1e16], [1.0], [-1e16]])
    g = O.zeta(R, f)
    assert g[2, 0] == 1.0 and math.fsum([1e16, 1.0, -1e16]) == 1.0
    assert p.n == 1


# ------------------------------------------------------------ generators
def test_chain_poset_planted_chains_are_chains():
    p = W.chain_poset(300, 8, 4, seed=11)
    R = O.reachability(p.n, p.indptr, p.indices)
    assert O.is_acyclic(R)
    for c in range(8):
        nodes = np.nonzero(p.chain_of == c)[0]
        nodes = nodes[np.argsort(p.chain_pos[nodes])]
        assert R[nodes[1:], nodes[:-1]].all()
    # cross edges go to other chains, and lower heights
    src, dst = p.edges()
    cross = p.chain_of[src] != p.chain_of[dst]
    assert (np.bincount(src[cross], minlength=p.n) <= 4).all()
    assert len(set(zip(src.tolist(), dst.tolist()))) == src.size


# --------------------------------------------------------- sampled oracle
@pytest.mark.parametrize("kind", ["int", "normal"])
def test_sampled_oracle_matches_closure(kind):
    p = W.chain_poset(400, 8, 3, seed=4)
    R = O.reachability(p.n, p.indptr, p.indices)
    f = W.functions(p.n, 4, kind, seed=9, lo=-1000, hi=1000)
    nodes = np.arange(0, 400, 7)
    a = O.zeta_at(p.n, p.indptr, p.indices, f, nodes)
    b = O.zeta(R, f, exact=(kind == "int"))[nodes]
    aa = O.zeta_adjoint_at(p.n, p.indptr, p.indices, f, nodes)
    bb = O.zeta_adjoint(R, f, exact=(kind == "int"))[nodes]
    if kind == "int":
        assert np.array_equal(a, b) and np.array_equal(aa, bb)
    else:
        assert np.allclose(a, b, rtol=1e-12, atol=1e-9) and np.allclose(aa, bb, rtol=1e-12, atol=1e-9)


# ------------------------------------------------------------------ width
def _max_antichain_brute(R):
    """Largest set of pairwise incomparable elements, by trying every subset."""
    n = R.shape[0]
    comp = R | R.T
    best = 0
    for mask in range(1 << n):
        idx = [i for i in range(n) if mask >> i & 1]
        if len(idx) <= best:
            continue
        if not comp[np.ix_(idx, idx)][~np.eye(len(idx), dtype=bool)].any():
            best = len(idx)
    return best


@pytest.mark.parametrize("seed", range(8))
def test_width_is_the_largest_antichain_brute_force(seed):
    """Theorem 2 / Dilworth: the fewest chains equal the largest antichain, found
    here by brute force over all subsets of a small random DAG."""
    p = W.random_small_dag(11, 0.25 + 0.05 * (seed % 3), seed=seed)
    R = O.reachability(p.n, p.indptr, p.indices)
    assert O.width(R) == _max_antichain_brute(R)


def test_width_closed_forms():
    """Chain 1, antichain n, a w x h grid min(w, h), the Boolean lattice of
    subsets of m elements C(m, floor(m/2)) (Sperner), the worked example 4."""
    def w(p):
        return O.width(O.reachability(p.n, p.indptr, p.indices))
    assert w(W.chain_only(40, seed=3)) == 1
    assert w(W.antichain(13)) == 13
    assert w(W.grid_poset(7, 5)) == 5 and w(W.grid_poset(3, 9)) == 3
    for m in (4, 5, 6, 7):
        assert w(W.boolean_lattice(m)) == math.comb(m, m // 2)
    assert w(W.worked_example()) == 4
