"""CPU tests of the C-ABI library: it loads, exports what include/posetx.h declares,
and its host preprocessing (chains, niv, up-niv, levels, validation) matches the
oracle's definitions.  No compute calls: these run without a GPU."""

import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def px():
    import paper_2211_13706_amd as px
    from paper_2211_13706_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2211_13706_amd.build import build
        build()
    px.lib()
    return px


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "posetx.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(px_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol(px):
    from paper_2211_13706_amd import _lib
    declared = _declared_functions()
    assert len(declared) >= 20
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in declared:
        assert hasattr(lib, name), f"{name} declared in posetx.h but not exported"
    assert sorted(_lib.EXPORTS) == declared


def _host(px, p, **kw):
    return px.poset_build(p.n, p.indptr, p.indices, p.chain_of if kw.get("planted", True) else None,
                          p.chain_pos if kw.get("planted", True) else None,
                          flags=px.PX_BUILD_HOST_ONLY | kw.get("flags", 0))


def _check_against_closure(px, P, p, R):
    co, cp = P.chains()
    k = P.k
    # chain-major numbering: chains in order, bottom first
    rows = P.rows()
    off = np.concatenate([[0], np.cumsum(np.bincount(co, minlength=k))])
    assert np.array_equal(rows, off[co] + cp) and np.array_equal(np.sort(rows), np.arange(p.n))
    # chains are totally ordered, positions 0..len-1
    for c in range(k):
        nodes = np.nonzero(co == c)[0]
        nodes = nodes[np.argsort(cp[nodes])]
        assert list(cp[nodes]) == list(range(nodes.size))
        assert R[nodes[1:], nodes[:-1]].all()
    niv = P.niv()
    assert np.array_equal(niv, O.niv_from_closure(R, co, cp, k))
    # up-niv is niv of the dual order, lowest element above: read it off R^T
    RT = np.ascontiguousarray(R.T)
    up = P.niv(up=True)
    want = np.full_like(up, -1)
    for x in range(p.n):
        above = np.nonzero(RT[x])[0]
        for j in range(k):
            cand = above[co[above] == j]
            if cand.size:
                want[x, j] = cand[np.argmin(cp[cand])]
    assert np.array_equal(up, want)
    # schedules: every U-solve dependency lies on a strictly lower level
    for upflag, nv in ((False, niv), (True, up)):
        lev = P.levels(up=upflag)
        for x in range(p.n):
            deps = [t for j, t in enumerate(nv[x]) if t >= 0 and j != co[x]]
            assert all(lev[t] < lev[x] for t in deps)
    info = P.info
    assert info["nnz_niv"] == int((niv >= 0).sum())
    assert info["mirsky_levels"] == O.mirsky_levels(R).max() + 1


@pytest.mark.parametrize("case", ["example", "cfg0", "lattice6", "grid", "random"])
@pytest.mark.parametrize("planted", [True, False])
@pytest.mark.parametrize("sparse", [False, True])
def test_preprocessing_matches_closure(px, case, planted, sparse):
    p = {"example": W.worked_example, "cfg0": lambda: W.chain_poset(600, 16, 4, seed=0),
         "lattice6": lambda: W.boolean_lattice(6), "grid": lambda: W.grid_poset(20, 7),
         "random": lambda: W.random_small_dag(90, 0.08, 3)}[case]()
    if planted and p.chain_of is None:
        pytest.skip("no planted chains for this poset")
    R = O.reachability(p.n, p.indptr, p.indices)
    P = _host(px, p, planted=planted, flags=px.PX_BUILD_SPARSE_NIV if sparse else 0)
    assert P.info["niv_sparse"] == int(sparse)
    if planted:
        assert P.k == p.k_planted
    _check_against_closure(px, P, p, R)
    _check_csr(P)


def _check_csr(P):
    """px_poset_niv_csr lists exactly the finite entries of px_poset_niv, in chain order."""
    co, _ = P.chains()
    for up in (False, True):
        niv = P.niv(up)
        ptr, nodes = P.niv_csr(up)
        assert ptr[0] == 0 and ptr[-1] == int((niv >= 0).sum())
        for x in range(P.n):
            row = niv[x][niv[x] >= 0]
            assert np.array_equal(nodes[ptr[x]:ptr[x + 1]], row)
            assert (np.diff(co[row]) > 0).all()


@pytest.mark.parametrize("n,deg", [(1500, 4), (2000, 6)])
def test_er_dag_sparse_niv_matches_closure(px, n, deg):
    """Erdős–Rényi DAGs of average degree 4 and 6 (§5) are wide (k > 256 here): the
    niv maps are kept sparse automatically and agree with the closure."""
    p = W.er_dag(n, deg, seed=2)
    R = O.reachability(p.n, p.indptr, p.indices)
    P = _host(px, p, planted=False)
    assert P.k > 256 and P.info["niv_sparse"] == 1
    _check_against_closure(px, P, p, R)
    _check_csr(P)


def test_matching_chains_reach_width(px):
    """Alg. 1 on the cover graph of the worked example and a Boolean lattice gives the width."""
    P = _host(px, W.worked_example(), planted=False)
    assert P.k == 4
    P = _host(px, W.boolean_lattice(10), planted=False)
    assert P.k == 252            # C(10, 5), Sperner / Dilworth


@pytest.mark.parametrize("case", ["er300", "er2000", "er2000d6", "small0", "small1", "lattice", "grid", "example"])
def test_min_chains_reach_width(px, case):
    """PX_BUILD_MIN_CHAINS refines the matching's path cover (Alg. 1, edges only)
    to as many chains as the width (Theorem 2), here the oracle's matching on the
    closure; the chains partition the elements and are totally ordered, and the
    niv maps read off the closure for those chains agree."""
    p = {"er300": lambda: W.er_dag(300, 2, seed=1), "er2000": lambda: W.er_dag(2000, 4, seed=2),
         "er2000d6": lambda: W.er_dag(2000, 6, seed=3), "small0": lambda: W.random_small_dag(60, 0.08, seed=5),
         "small1": lambda: W.random_small_dag(120, 0.03, seed=6), "lattice": lambda: W.boolean_lattice(6),
         "grid": lambda: W.grid_poset(12, 9), "example": W.worked_example}[case]()
    R = O.reachability(p.n, p.indptr, p.indices)
    P0 = _host(px, p, planted=False)
    P = _host(px, p, planted=False, flags=px.PX_BUILD_MIN_CHAINS)
    assert P.k == O.width(R) <= P0.k
    assert P.info["path_cover"] == P0.k
    _check_against_closure(px, P, p, R)


def test_mirsky_schedule_flag(px):
    p = W.worked_example()
    P = _host(px, p, flags=px.PX_BUILD_LEVELS_MIRSKY)
    R = O.reachability(p.n, p.indptr, p.indices)
    assert np.array_equal(P.levels(), O.mirsky_levels(R))
    assert P.info["levels_down"] == 5


def _err(px, fn):
    with pytest.raises(px.PosetxError) as ei:
        fn()
    return ei.value.name


def test_rejects_bad_input(px):
    p = W.worked_example()
    # cycle: add an edge from a minimal element back up to the top
    src, dst = p.edges()
    src2 = np.concatenate([src, [11]]); dst2 = np.concatenate([dst, [0]])
    order = np.argsort(src2, kind="stable")
    indptr = np.zeros(13, np.int64); np.cumsum(np.bincount(src2, minlength=12), out=indptr[1:])
    assert _err(px, lambda: px.poset_build(12, indptr, dst2[order], flags=px.PX_BUILD_HOST_ONLY)) == "PX_ECYCLE"
    # self-loop
    ind = p.indices.copy(); ind[0] = 0
    assert _err(px, lambda: px.poset_build(12, p.indptr, ind, flags=px.PX_BUILD_HOST_ONLY)) == "PX_EINVAL"
    # out-of-range target
    ind = p.indices.copy(); ind[1] = 99
    assert _err(px, lambda: px.poset_build(12, p.indptr, ind, flags=px.PX_BUILD_HOST_ONLY)) == "PX_EINVAL"
    # planted chain that is not totally ordered: swap two incomparable elements' chains
    co, cp = p.chain_of.copy(), p.chain_pos.copy()
    co[[4, 5]] = co[[5, 4]]; cp[[4, 5]] = cp[[5, 4]]     # x5 and x6 are incomparable
    assert _err(px, lambda: px.poset_build(12, p.indptr, p.indices, co, cp,
                                           flags=px.PX_BUILD_HOST_ONLY)) == "PX_ECHAIN"
    # reversed chain order
    cp2 = p.chain_pos.copy()
    c0 = np.nonzero(p.chain_of == 0)[0]; cp2[c0] = cp2[c0].max() - cp2[c0]
    assert _err(px, lambda: px.poset_build(12, p.indptr, p.indices, p.chain_of, cp2,
                                           flags=px.PX_BUILD_HOST_ONLY)) == "PX_ECHAIN"
    # the sparse recursion checks the chains the same way
    for cpos, cof in ((cp, co), (cp2, p.chain_of)):
        assert _err(px, lambda: px.poset_build(12, p.indptr, p.indices, cof, cpos,
                                               flags=px.PX_BUILD_HOST_ONLY | px.PX_BUILD_SPARSE_NIV)) == "PX_ECHAIN"
    # duplicate chain position
    cp3 = p.chain_pos.copy(); cp3[c0[0]] = cp3[c0[1]]
    assert _err(px, lambda: px.poset_build(12, p.indptr, p.indices, p.chain_of, cp3,
                                           flags=px.PX_BUILD_HOST_ONLY)) == "PX_EINVAL"


def test_empty_and_trivial_posets(px):
    P = px.poset_build(0, np.zeros(1, np.int64), np.zeros(0, np.int32), flags=px.PX_BUILD_HOST_ONLY)
    assert P.k == 0 and P.n == 0
    P = _host(px, W.antichain(7), planted=False)
    assert P.k == 7 and P.info["levels_down"] == 1
    assert (P.niv() == np.where(np.eye(7, dtype=bool), np.arange(7)[:, None], -1)).all()


def test_duplicate_and_transitive_edges(px):
    p = W.worked_example()
    src, dst = p.edges()
    # add duplicates and the transitive edge x1 -> x12
    src2 = np.concatenate([src, src[:5], [0]]); dst2 = np.concatenate([dst, dst[:5], [11]])
    order = np.argsort(src2, kind="stable")
    indptr = np.zeros(13, np.int64); np.cumsum(np.bincount(src2, minlength=12), out=indptr[1:])
    P = px.poset_build(12, indptr, dst2[order], p.chain_of, p.chain_pos, flags=px.PX_BUILD_HOST_ONLY)
    R = O.reachability(p.n, p.indptr, p.indices)
    assert np.array_equal(P.niv(), O.niv_from_closure(R, p.chain_of, p.chain_pos, 4))


def test_config1_preprocessing_scale(px):
    """The n = 2^20, k = 64 poset preprocesses on the host in seconds; niv invariants hold."""
    p = W.chain_poset(1 << 16, 64, 3, seed=1)
    P = _host(px, p)
    info = P.info
    assert info["k"] == 64 and info["max_chain"] == 1024
    niv = P.niv()
    co, cp = P.chains()
    # own chain entry is the element itself (Theorem 5, second case)
    assert (niv[np.arange(p.n), co] == np.arange(p.n)).all()
    # niv is monotone along every chain: x below y implies out(x) ⊆ out(y)
    for c in range(0, 64, 16):
        nodes = np.nonzero(co == c)[0]
        nodes = nodes[np.argsort(cp[nodes])]
        pos = np.where(niv[nodes] >= 0, cp[np.maximum(niv[nodes], 0)], -1)
        assert (np.diff(pos, axis=0) >= 0).all()
    assert info["udep_levels"] < info["mirsky_levels"]


def test_threaded_recursion_matches_serial(px, monkeypatch):
    """The host recursion merges the rows of one height on several threads, and the parent
    lists are built on several threads; the maps and level schedules do not depend on the
    thread count (sparse rows of a wide ER DAG, and dense rows with the chain check)."""
    for p, planted in ((W.er_dag(1 << 15, 4, seed=9), False), (W.chain_poset(1 << 15, 16, 3, seed=9), True)):
        got = []
        for t in ("1", "6"):
            monkeypatch.setenv("POSETX_PREP_THREADS", t)
            P = _host(px, p, planted=planted)
            got.append((P.niv_csr(), P.niv_csr(True), P.levels(), P.levels(True)))
        (a, b) = got
        for x, y in zip(a[:2], b[:2]):
            assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1])
        assert np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3])


@pytest.mark.parametrize("case", ["cfg0", "er", "lattice", "antichain"])
def test_save_load_roundtrip(px, case, tmp_path):
    """A saved handle loads back with the same chains, maps, schedules and counts."""
    p, planted = {"cfg0": (W.chain_poset(2000, 16, 4, seed=0), True), "er": (W.er_dag(1500, 4, seed=2), False),
                  "lattice": (W.boolean_lattice(6), False), "antichain": (W.antichain(9), False)}[case]
    A = _host(px, p, planted=planted)
    path = tmp_path / "p.pxposet"
    A.save(path)
    Bq = px.poset_load(path, flags=px.PX_BUILD_HOST_ONLY)
    for a, b in zip(A.chains(), Bq.chains()):
        assert np.array_equal(a, b)
    assert np.array_equal(A.rows(), Bq.rows())
    for up in (False, True):
        for a, b in zip(A.niv_csr(up), Bq.niv_csr(up)):
            assert np.array_equal(a, b)
        assert np.array_equal(A.levels(up), Bq.levels(up))
    ia, ib = A.info_dict(), Bq.info_dict()
    for key in ("n", "k", "edges", "nnz_niv", "nnz_niv_up", "max_chain", "levels_down", "levels_up",
                "mirsky_levels", "udep_levels", "niv_sparse", "chains_planted"):
        assert ia[key] == ib[key], key


def test_load_rejects_bad_files(px, tmp_path):
    """Truncated, foreign and index-corrupted files are refused with PX_EINVAL."""
    p = W.chain_poset(300, 8, 3, seed=1)
    A = _host(px, p)
    good = tmp_path / "good.pxposet"
    A.save(good)
    data = bytearray(good.read_bytes())
    cases = {"truncated": data[: len(data) // 2], "foreign": b"not a poset file at all" + bytes(64),
             "empty": b""}
    # corrupt one node_of_row entry: the arrays follow the header (8 magic + 4 + 4 + 8 * 8 + 4 + 4 * 8);
    # chain_of, chain_pos, chain_off, row_of_node, then node_of_row
    hdr = 8 + 4 + 4 + 64 + 4 + 32
    n, k = p.n, 8
    off = hdr
    for cnt in (n, n, k + 1, n):
        off += 8 + 4 * cnt
    bad = bytearray(data)
    bad[off + 8: off + 12] = (10 ** 6).to_bytes(4, "little")
    cases["index"] = bad
    for name, blob in cases.items():
        f = tmp_path / f"{name}.pxposet"
        f.write_bytes(bytes(blob))
        with pytest.raises(px.PosetxError) as ei:
            px.poset_load(f, flags=px.PX_BUILD_HOST_ONLY)
        assert ei.value.name == "PX_EINVAL", name
    with pytest.raises(px.PosetxError):
        px.poset_load(tmp_path / "missing.pxposet", flags=px.PX_BUILD_HOST_ONLY)


def test_save_load_keeps_build_choices(px, tmp_path):
    """No-adjoint and Mirsky-schedule handles keep those choices through a file."""
    p = W.chain_poset(500, 8, 3, seed=3)
    for flags in (px.PX_BUILD_NO_ADJOINT, px.PX_BUILD_LEVELS_MIRSKY, px.PX_BUILD_SPARSE_NIV):
        A = _host(px, p, flags=flags)
        path = tmp_path / f"p{flags}.pxposet"
        A.save(path)
        Bq = px.poset_load(path, flags=px.PX_BUILD_HOST_ONLY)
        assert np.array_equal(A.levels(), Bq.levels())
        assert A.info_dict()["levels_down"] == Bq.info_dict()["levels_down"]
        assert A.info_dict()["niv_sparse"] == Bq.info_dict()["niv_sparse"]
        if flags == px.PX_BUILD_NO_ADJOINT:
            with pytest.raises(px.PosetxError) as ei:
                Bq.niv(up=True)
            assert ei.value.name == "PX_EUNSUPPORTED"
        else:
            for a, b in zip(A.niv_csr(True), Bq.niv_csr(True)):
                assert np.array_equal(a, b)


def test_load_recounts_sizes(px, tmp_path):
    """The entry counts that size device work are recounted from the arrays on load, not read
    from the file's header."""
    p = W.er_dag(600, 4, seed=4)
    A = _host(px, p, planted=False)
    path = tmp_path / "p.pxposet"
    A.save(path)
    data = bytearray(path.read_bytes())
    data[40:48] = (3).to_bytes(8, "little", signed=True)      # nnz_niv
    data[48:56] = (2 ** 40).to_bytes(8, "little", signed=True)  # nnz_niv_up
    path.write_bytes(bytes(data))
    Bq = px.poset_load(path, flags=px.PX_BUILD_HOST_ONLY)
    assert Bq.info_dict()["nnz_niv"] == A.info_dict()["nnz_niv"]
    assert Bq.info_dict()["nnz_niv_up"] == A.info_dict()["nnz_niv_up"]


def test_concurrent_builds_match_serial(px):
    """px_poset_build calls on several threads at once (poset_build_many) give the same
    chains, niv maps and level schedules as one build after another."""
    posets = W.batched_posets(24, seed=61, nmin=200, nmax=3000)
    specs = [(q.n, q.indptr, q.indices, None if i % 2 else q.chain_of, None if i % 2 else q.chain_pos)
             for i, q in enumerate(posets)]
    many = px.poset_build_many(specs, flags=px.PX_BUILD_HOST_ONLY, threads=6)
    for (n, ip, ix, co, cp), P in zip(specs, many):
        S = px.poset_build(n, ip, ix, co, cp, flags=px.PX_BUILD_HOST_ONLY)
        assert P.k == S.k
        for a, b in zip(P.chains(), S.chains()):
            assert np.array_equal(a, b)
        for up in (False, True):
            assert np.array_equal(P.niv(up), S.niv(up))
            assert np.array_equal(P.levels(up), S.levels(up))


def test_concurrent_builds_report_a_failing_spec(px):
    """A spec that cannot be built (here a 2-cycle) among concurrent builds raises its own
    error (PX_ECYCLE) from poset_build_many; the other specs build as usual alone."""
    posets = W.batched_posets(6, seed=62, nmin=200, nmax=800)
    specs = [(q.n, q.indptr, q.indices, None, None) for q in posets]
    specs.insert(3, (2, np.array([0, 1, 2], dtype=np.int64), np.array([1, 0], dtype=np.int32), None, None))
    assert _err(px, lambda: px.poset_build_many(specs, flags=px.PX_BUILD_HOST_ONLY, threads=4)) == "PX_ECYCLE"
    good = specs[:3] + specs[4:]
    assert [P.n for P in px.poset_build_many(good, flags=px.PX_BUILD_HOST_ONLY, threads=4)] == [q.n for q in posets]
    assert px.poset_build_many([], flags=px.PX_BUILD_HOST_ONLY) == []
