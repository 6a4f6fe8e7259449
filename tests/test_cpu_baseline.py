"""The O(n·k) CPU baseline (baseline/nk_cpu.cpp) against the oracle: it is a reported
baseline, so it must compute the same transforms (int64 exactly)."""

import numpy as np
import pytest

import oracle as O
import workloads as W


@pytest.fixture(scope="module")
def nk():
    import baseline
    baseline.build()
    return baseline


@pytest.mark.parametrize("case", ["cfg0", "grid", "matching"])
def test_nk_cpu_matches_oracle(nk, case):
    import paper_2211_13706_amd as px
    p, planted = {"cfg0": (W.chain_poset(2000, 16, 4, seed=0), True), "grid": (W.grid_poset(60, 7), True),
                  "matching": (W.random_small_dag(300, 0.03, 7), False)}[case]
    P = px.poset_build(p.n, p.indptr, p.indices, p.chain_of if planted else None,
                       p.chain_pos if planted else None, flags=px.PX_BUILD_HOST_ONLY)
    R = O.reachability(p.n, p.indptr, p.indices)
    cpu = nk.NkCpu(P, threads=4)
    assert cpu.threads == 4
    for B in (1, 17, 64):
        f = W.functions(p.n, B, "int", seed=B, lo=-(2**40), hi=2**40)
        g = cpu.zeta(f)
        assert np.array_equal(g, O.zeta(R, f))
        assert np.array_equal(cpu.mobius(g), f)
        assert np.array_equal(cpu.mobius(f), O.mobius_by_substitution(R, f))
        ff = W.functions(p.n, B, "normal", seed=B + 1)
        gf = cpu.zeta(ff).astype(np.float64)
        want = O.zeta(R, ff, exact=False)
        assert (np.abs(gf - want) <= 2.0 ** -23 * (R.astype(np.float64) @ np.abs(ff)) + 1e-30).all()
    assert cpu.time_zeta(W.functions(p.n, 8, "normal", seed=3), reps=3) > 0


def test_nk_cpu_model_and_threads(nk):
    t, aff = nk.host_threads()
    assert 1 <= t <= aff
    assert isinstance(nk.cpu_model(), str)
