"""Benchmark of the fast zeta transform on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
                    [--legs none|default|all|sparse|batched|chains|large]

Workload (the headline configuration): a random-height poset with
n = 2^20 elements, k = 64 planted chains of 16,384 elements, 3 cross edges
per element, and B = 64 float32 right-hand sides f ~ N(0, 1).  One step is
one batched zeta transform g = Z f (chain scan + niv gather) with the inputs
resident in HBM.  Host preprocessing is timed separately and reported under
"preprocess_s".

Printed: ONE JSON line with the metric (node·RHS/s), the roofline of the
dominant kernel (algorithmic bytes per launch / its average HIP-event
duration on the launch stream), the same steps over four rotating input
buffers (no input left in the cache by the step before), the CPU oracle timed
on a bounded sample of the same workload on the host, and the straightforward
O(n·k) C++/OpenMP transforms on all the host cores the process may use.  "legs" adds measurements of the other
rows: by default the int64 zeta and Möbius, the adjoint, the B = 8 share,
the preprocessing and the grid Möbius; "all" also the batched posets, the
n = 2^23 poset and the Erdős–Rényi DAGs with sparse niv rows.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "zeta/Möbius node·RHS per sec at 1 GPU + achieved HBM GB/s vs peak"
HBM_PEAK_GBS = 8000.0
N, K, CROSS, B, SEED = 1 << 20, 64, 3, 64, 1


def kernel_hash() -> str:
    h = hashlib.sha256()
    for name in ("kernels.hip", "kernels.h"):
        with open(os.path.join(ROOT, "paper_2211_13706_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(phase: str, n: int, k: int, B: int, s: int, compact: bool = False) -> int:
    """Compulsory bytes of one launch: the factored method Z = U V reads f, writes the chain
    prefixes P, reads P once, reads the niv map and writes g, each array once per step
    (20 B per node·RHS at k = B = 64 in float32).  A kernel is charged the arrays of that
    list which it reads or writes; tile states, snapshots, index arrays and the compact
    walk's gathered prefixes are implementation traffic (``moved_bytes``).

    compact walk (P never exists): scan_reduce reads f; apply_combine reads f and writes g.
    walk over P: scan_apply reads f and writes P; walk_combine reads P and writes g.
    gather (one thread per row): reads P and niv, writes g."""
    f = g = p_ = n * B * s
    niv = n * k * 4
    return {"scan_reduce": f, "scan_carry": 0, "walk_events": 0,
            "apply_combine": f + g,
            "scan_apply": f + p_, "scan_onepass": f + p_,
            "walk_combine": p_ + g,
            "gather": p_ + niv + g}.get(phase, 0)


def moved_bytes(phase: str, n: int, k: int, B: int, s: int, info: dict, compact: bool = False) -> int:
    """Bytes a kernel of this implementation moves: every array it touches, once.

    Tile states (the scan's per-tile totals and carries, n/64 tiles of 64 rows
    for 64-column blocks, 2s bytes per column) count where they are read or
    written.  The compact walk (the default at B = 64) records P only at the
    walk's gathered rows (walk_rows_distinct slots): the reduce also writes their
    tile-local prefixes L, the carry reads L and writes Q, the walk reads Q
    instead of P, and apply_combine writes g = P + snapshot without writing P.
    walk_events: the change events (16 B each) and the run table (16 B per run),
    the first-row entries of every run (4k B), every gathered row counted once
    and the snapshots it stores.
    walk_combine: P, the snapshots, node_of_row and snap_of_row, and g.
    """
    runs, ev, snaps = info.get("walk_runs", 0), info.get("walk_events", 0), info.get("walk_snapshots", 0)
    slots = info.get("walk_rows_distinct", 0)
    states = -(-n // 64) * B * 2 * s
    if phase == "walk_events":
        return ev * 16 + runs * (k * 4 + 16) + slots * B * s + snaps * B * s
    if phase == "walk_combine":
        return n * B * s + snaps * B * s + 8 * n + n * B * s
    if phase == "apply_combine":  # read f, C, snapshots, node_of_row, snap_of_row; write g
        return n * B * s + states + snaps * B * s + 8 * n + n * B * s
    if phase == "gather":        # one thread per row: read P, niv, node_of_row, write g
        return n * B * s + n * k * 4 + n * 4 + n * B * s
    if phase == "scan_apply":    # read f, C, node_of_row, write P
        return n * B * s + states + n * 4 + n * B * s
    if phase == "scan_reduce":   # read f, node_of_row, write tile totals (and L)
        return n * B * s + n * 4 + states + (slots * B * s if compact else 0)
    if phase == "scan_carry":    # read tile totals, write carries (and read L, write Q)
        return 2 * states + (2 * slots * B * s if compact else 0)
    if phase == "scan_onepass":  # read f, read node_of_row, write P
        return n * B * s + n * 4 + n * B * s
    return 0


def gathered_bytes(phase: str, k: int, B: int, s: int, info: dict) -> int:
    """Bytes a kernel moves through the memory hierarchy, re-reads included: for
    walk_events every P-row load (first rows' gathers, both rows of each event)."""
    if phase != "walk_events":
        return 0
    runs, ev, snaps = info.get("walk_runs", 0), info.get("walk_events", 0), info.get("walk_snapshots", 0)
    return ev * 16 + runs * (k * 4 + 16) + info.get("walk_row_loads", 0) * B * s + snaps * B * s


def profile_read(lib, nph=11):
    import ctypes
    ms = (ctypes.c_double * nph)()
    cnt = (ctypes.c_int64 * nph)()
    lib.px_profile_read(ms, cnt, nph)
    return {lib.px_profile_phase_name(i).decode(): (ms[i], cnt[i]) for i in range(nph)}


def traffic_for(phase: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they match this kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            t = json.load(fh)
    except OSError:
        return None
    if t.get("kernel_hash") != kernel_hash():
        return None
    return t.get("per_launch_bytes", {}).get(phase)


def measured_copy_gbps(dev, mib: int = 256, reps: int = 10) -> float:
    """Read + write bandwidth of a plain device-to-device copy of `mib` MiB (torch), timed with
    HIP events: the practical streaming rate that the roofline is also compared against."""
    import torch
    a = torch.empty(mib << 18, dtype=torch.float32, device=dev).normal_()
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) * 1e-3 / reps
    del a, b
    return round(2 * (mib << 20) / t / 1e9, 1)


def cpu_baseline(p, f, budget_s: float):
    """The oracle as it stands (BFS over each sampled element's down-set, float64 sums),
    on a bounded sample of elements of the same workload."""
    import oracle as O
    rng = np.random.default_rng(12345)
    order = rng.permutation(p.n)
    t0 = time.perf_counter()
    done = 0
    while done < len(order) and time.perf_counter() - t0 < budget_s:
        O.zeta_at(p.n, p.indptr, p.indices, f, order[done:done + 1])
        done += 1
    dt = time.perf_counter() - t0
    return {"value": done * f.shape[1] / dt, "unit": "node·RHS/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} random elements of the same n=2^20 poset, all {f.shape[1]} RHS "
                      f"(down-set by BFS, float64 pairwise sums), {dt:.1f} s single-threaded"}


def cpu_nk_baseline(P, p, f_host, gpu_rate):
    """The straightforward O(n·k) CPU transforms (C++17 + OpenMP: Alg. 3 zeta, Alg. 4 Möbius
    over the level schedule of Alg. 5) on the same dense niv map, on the host's cores: the
    float32 zeta of the whole workload and the exact int64 Möbius of an int64 copy, each
    the steady_clock median of 5 calls after one warm-up."""
    import baseline
    import workloads as W
    cpu = baseline.NkCpu(P)
    tz = cpu.time_zeta(f_host, reps=5)
    fi = W.functions(p.n, f_host.shape[1], "int", seed=3, lo=-1000, hi=1000)
    gi = cpu.zeta(fi)
    tm = cpu.time_mobius(gi, reps=5)
    exact = bool(np.array_equal(cpu.mobius(gi), fi))
    nb = p.n * f_host.shape[1]
    return {"value": nb / tz, "unit": "node·RHS/s", "cores": cpu.threads, "affinity_cpus": cpu.affinity,
            "cpu_model": baseline.cpu_model(), "build": baseline.lib().variant,
            "kind": "O(n·k) C++17/OpenMP (Alg. 3 zeta, Alg. 4 + Alg. 5 level-parallel Möbius)",
            "timing": "std::chrono::steady_clock, median of 5 after 1 warm-up",
            "zeta_f32_s": tz, "mobius_int64_s": tm, "mobius_int64_node_rhs_per_s": nb / tm,
            "mobius_roundtrip_exact": exact, "levels": cpu.nlev,
            "gpu_over_cpu_zeta": round(gpu_rate / (nb / tz), 1)}


def _time(fn, steps, sync):
    for _ in range(2):
        fn()
    sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    sync()
    return (time.perf_counter() - t0) / steps


def f64_growth(px, P, n, dev, B_: int = 4):
    """max|M r| / max|r| for r ~ U(-1, 1) in float64: how far the Möbius transform of this poset
    amplifies data (an infinite or NaN result means float64 overflows)."""
    import torch
    import workloads as W
    r = torch.from_numpy(W.functions(n, B_, "uniform", seed=12, lo=-1.0, hi=1.0).astype("float64")).to(dev)
    m = px.mobius(P, r, tol=-1.0)  # no value check: an overflow is the answer here
    g = (m.abs().amax() / r.abs().amax()).item()
    return g if g == g and g != float("inf") else str(g)


def legs_config1(px, P, p, dev, steps):
    """int64 zeta and the exact Möbius round trip, and the float32 adjoint, on the headline poset."""
    import torch
    import workloads as W
    sync = torch.cuda.synchronize
    out = {}
    fi = torch.from_numpy(W.functions(p.n, B, "int", seed=3, lo=-1000, hi=1000)).to(dev)
    gi = torch.empty_like(fi)
    fb = torch.empty_like(fi)
    P.reserve(torch.int64, B)
    t = _time(lambda: px.zeta(P, fi, out=gi), steps, sync)
    out["zeta_int64"] = {"ms": round(t * 1e3, 4), "node_rhs_per_s": p.n * B / t}
    t = _time(lambda: px.mobius(P, gi, out=fb), max(2, steps // 4), sync)
    out["mobius_int64"] = {"ms": round(t * 1e3, 4), "node_rhs_per_s": p.n * B / t,
                           "levels": P.info["levels_down"],
                           "us_per_level": round(t * 1e6 / max(1, P.info["levels_down"]), 2),
                           "roundtrip_exact": bool(torch.equal(fb, fi))}
    del fi, gi, fb
    out["mobius_f64_growth"] = f64_growth(px, P, p.n, dev)
    ff = torch.from_numpy(W.functions(p.n, B, "normal", seed=4)).to(dev)
    ga = torch.empty_like(ff)
    t = _time(lambda: px.zeta_adjoint(P, ff, out=ga), steps, sync)
    out["zeta_adjoint_f32"] = {"ms": round(t * 1e3, 4), "node_rhs_per_s": p.n * B / t}
    del ff, ga
    # one GPU's share of an 8-way split of the right-hand sides (the sharding that needs no
    # exchange): the same poset at B = 8, and its rate against B = 64
    f8 = torch.from_numpy(W.functions(p.n, 8, "normal", seed=4)).to(dev)
    g8 = torch.empty_like(f8)
    P.reserve(torch.float32, 8)
    tune8 = P.autotune(torch.float32, 8)  # the tile shapes for this width (the headline's were for 64)
    t8 = _time(lambda: px.zeta(P, f8, out=g8), steps, sync)
    P.set_layout("rows")  # the same share with the matrices in chain-major row order
    f8r = f8[torch.from_numpy(np.argsort(P.rows())).to(dev)].contiguous()
    g8r = torch.empty_like(f8r)
    t8r = _time(lambda: px.zeta(P, f8r, out=g8r), steps, sync)
    eq8 = bool(torch.equal(g8r[torch.from_numpy(P.rows()).to(dev)], g8))
    P.set_layout("nodes")
    out["zeta_f32_B8_share"] = {"ms": round(t8 * 1e3, 4), "node_rhs_per_s": p.n * 8 / t8,
                                "rows_layout_ms": round(t8r * 1e3, 4), "rows_layout_equal": eq8,
                                "autotune": {k: tune8[k] for k in ("walk_T", "walk_emax", "rhs_tile")}}
    del f8r, g8r
    del f8, g8
    out["preprocess"] = leg_preprocess(px, P, p)
    return out


def leg_preprocess(px, P, p):
    """The niv maps of the headline poset: device fixed point (as built) against the host
    recursion (POSETX_PREP=host), seconds of each and whether the maps agree."""
    os.environ["POSETX_PREP"] = "host"
    try:
        t0 = time.perf_counter()
        Q = px.poset_build(p.n, p.indptr, p.indices, p.chain_of, p.chain_pos, device=0)
        t_host = time.perf_counter() - t0
    finally:
        del os.environ["POSETX_PREP"]
    same = bool(np.array_equal(P.niv(), Q.niv()) and np.array_equal(P.niv(True), Q.niv(True)))
    return {"niv_device_s": round(P.info["t_niv"], 3), "niv_device_rounds": P.info["niv_device_rounds"],
            "niv_host_s": round(Q.info["t_niv"], 3), "build_host_niv_s": round(t_host, 3),
            "maps_equal": same}


def leg_grid(px, dev, steps, refine=3):
    """Config 2: the 4096 x 64 grid, B = 16 float32 g ~ U(-1, 1).  Batched float32 Möbius with
    float64-residual refinement against B single-RHS float64 Möbius calls."""
    import torch
    import workloads as W
    sync = torch.cuda.synchronize
    q = W.grid_poset(4096, 64)
    G = px.poset_build(q.n, q.indptr, q.indices, q.chain_of, q.chain_pos, device=0)
    Bg = 16
    g = torch.from_numpy(W.functions(q.n, Bg, "uniform", seed=10, lo=-1.0, hi=1.0)).to(dev)
    f = torch.empty_like(g)
    G.reserve(torch.float32, Bg)
    # asynchronous calls (tol < 0: no value check, no host synchronisation) on both sides
    t32 = _time(lambda: px.mobius(G, g, out=f, max_refine=refine, tol=-1.0), steps, sync)
    _, rep = px.mobius(G, g, out=f, max_refine=refine, report=True)
    g64 = g.double()
    cols = [g64[:, b:b + 1].contiguous() for b in range(Bg)]
    f64 = [torch.empty_like(c) for c in cols]
    G.reserve(torch.float64, 1)
    t64 = _time(lambda: [px.mobius(G, c, out=o, tol=-1.0) for c, o in zip(cols, f64)], max(2, steps // 4), sync)
    # agreement of the refined float32 result with the float64 solve, normwise per column
    f64m = torch.cat(f64, dim=1)
    err = ((f.double() - f64m).abs().amax(0) / f64m.abs().amax(0)).max().item()
    # one exact int64 solve: the time per level of the schedule
    gi = torch.from_numpy(W.functions(q.n, Bg, "int", seed=11, lo=-1000, hi=1000)).to(dev)
    fi = torch.empty_like(gi)
    G.reserve(torch.int64, Bg)
    ti = _time(lambda: px.mobius(G, gi, out=fi), steps, sync)
    # both forms again with one launch per level instead of the persistent level solve
    prev = os.environ.get("POSETX_LEVEL_POLL")
    os.environ["POSETX_LEVEL_POLL"] = "0"
    try:
        t32l = _time(lambda: px.mobius(G, g, out=f, max_refine=refine, tol=-1.0), steps, sync)
        t64l = _time(lambda: [px.mobius(G, c, out=o, tol=-1.0) for c, o in zip(cols, f64)], max(2, steps // 4), sync)
    finally:
        if prev is None:
            os.environ.pop("POSETX_LEVEL_POLL", None)
        else:
            os.environ["POSETX_LEVEL_POLL"] = prev
    return {"workload": "grid 4096x64 (n=262144, k=64), B=16 float32 U(-1,1)",
            "levels": G.info["levels_down"], "mirsky_levels": G.info["mirsky_levels"],
            "int64_mobius_ms": round(ti * 1e3, 4),
            "us_per_level": round(ti * 1e6 / max(1, G.info["levels_down"]), 2),
            "f32_refined_ms": round(t32 * 1e3, 4), "refine_steps": refine,
            "f64_single_rhs_x16_ms": round(t64 * 1e3, 4), "speedup": round(t64 / t32, 2),
            "rel_err_vs_f64": err, "report": rep,
            "launch_per_level": {"f32_refined_ms": round(t32l * 1e3, 4),
                                 "f64_single_rhs_x16_ms": round(t64l * 1e3, 4),
                                 "speedup": round(t64l / t32l, 2)}}


def leg_batched(px, dev, steps, count=512):
    """Config 3: uneven posets, forward zeta + adjoint per step, replayed from a HIP graph."""
    import torch
    import workloads as W
    from paper_2211_13706_amd.autograd import batch_zeta_fn
    sync = torch.cuda.synchronize
    t0 = time.perf_counter()
    posets = W.batched_posets(count, seed=40)
    # the posets are independent: built on several host threads at once
    Ps = px.poset_build_many([(q.n, q.indptr, q.indices, q.chain_of, q.chain_pos) for q in posets], device=0)
    bt = px.batch_build(Ps)
    t_prep = time.perf_counter() - t0
    Bb = 8
    f = torch.randn(bt.rows, Bb, device=dev, requires_grad=True)
    w = torch.randn(bt.rows, Bb, device=dev)
    bt.reserve(torch.float32, Bb)

    def step():
        f.grad = None
        (batch_zeta_fn(bt, f) * w).sum().backward()
    t_eager = _time(step, steps, sync)
    g = torch.empty(bt.rows, Bb, device=dev)
    gw = torch.empty(bt.rows, Bb, device=dev)
    fd = f.detach()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        px.zeta_batched(bt, fd, out=g)
        px.zeta_adjoint_batched(bt, w, out=gw)
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        px.zeta_batched(bt, fd, out=g)
        px.zeta_adjoint_batched(bt, w, out=gw)
    t_graph = _time(graph.replay, steps, sync)
    ok = bool(torch.allclose(gw, f.grad, rtol=0, atol=0))
    # the same graph with the matrices in the kernels' row order (px_batch_set_layout)
    perm = torch.from_numpy(bt.row_order()).to(dev)
    fr = torch.empty_like(fd)
    fr[perm] = fd
    wr = torch.empty_like(w)
    wr[perm] = w
    gr = torch.empty_like(g)
    gwr = torch.empty_like(gw)
    bt.set_layout("rows")
    with torch.cuda.stream(s):
        px.zeta_batched(bt, fr, out=gr)
        px.zeta_adjoint_batched(bt, wr, out=gwr)
    torch.cuda.current_stream().wait_stream(s)
    graph_r = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph_r):
        px.zeta_batched(bt, fr, out=gr)
        px.zeta_adjoint_batched(bt, wr, out=gwr)
    t_graph_r = _time(graph_r.replay, steps, sync)
    rows_equal = bool(torch.equal(gr[perm], g) and torch.equal(gwr[perm], gw))
    bt.set_layout("nodes")
    # load balance of the walk (its dominant kernel): workgroups take the runs in 8
    # contiguous slices, one per XCD, poset after poset; events per slice, from each
    # poset's run and event counts (events spread evenly over a poset's runs)
    infos = [P.info_dict() for P in Ps]
    runs = np.array([i["walk_runs"] for i in infos], np.float64)
    evs = np.array([i["walk_events"] for i in infos], np.float64)
    edges = np.linspace(0, runs.sum(), 9)
    cum = np.concatenate([[0], np.cumsum(runs)])
    per_xcd = []
    for a, b in zip(edges[:-1], edges[1:]):
        lo = np.clip(np.minimum(cum[1:], b) - np.maximum(cum[:-1], a), 0, None)
        per_xcd.append(float((lo / np.maximum(runs, 1) * evs).sum()))
    balance = {"walk_events_per_xcd_max_over_mean": round(max(per_xcd) / (sum(per_xcd) / 8), 3),
               "walk_runs": int(runs.sum()), "walk_events": int(evs.sum())}
    # compulsory bytes of forward + adjoint: per direction the niv map (4k B per row)
    # and f, P written, P read and g (4 B per row and RHS each)
    nk = sum(int(P.n) * int(P.k) for P in Ps)
    alg = 2 * (4 * nk + 4 * 4 * int(bt.rows) * Bb)
    floor_ms = alg / (HBM_PEAK_GBS * 1e9) * 1e3
    return {"workload": f"{count} posets, n log-uniform in [1000, 65536], k in 4..128, B=8 float32",
            "rows": int(bt.rows), "preprocess_s": round(t_prep, 2),
            "autograd_fwd_bwd_ms": round(t_eager * 1e3, 4), "graph_fwd_adj_ms": round(t_graph * 1e3, 4),
            "node_rhs_per_s_graph": 2 * bt.rows * Bb / t_graph, "graph_grad_equal_eager": ok,
            "alg_bytes": alg, "hbm_floor_ms": round(floor_ms, 4),
            "frac_of_floor": round(floor_ms / (t_graph * 1e3), 4),
            "graph_fwd_adj_rows_layout_ms": round(t_graph_r * 1e3, 4), "rows_layout_equal": rows_equal,
            "frac_of_floor_rows_layout": round(floor_ms / (t_graph_r * 1e3), 4), "load_balance": balance}


def leg_large(px, dev, steps):
    """Config 4: n = 2^23, k = 32, B = 16 float32: zeta, float32 Möbius(zeta(f)) with refinement,
    and the exact int64 round trip."""
    import torch
    import workloads as W
    sync = torch.cuda.synchronize
    t0 = time.perf_counter()
    q = W.chain_poset(1 << 23, 32, 3, seed=4)
    L = px.poset_build(q.n, q.indptr, q.indices, q.chain_of, q.chain_pos, device=0)
    t_prep = time.perf_counter() - t0
    Bl = 16
    f = torch.from_numpy(W.functions(q.n, Bl, "normal", seed=5)).to(dev)
    g = torch.empty_like(f)
    L.reserve(torch.float32, Bl)
    tz = _time(lambda: px.zeta(L, f, out=g), steps, sync)
    # the same transform with the matrices kept in chain-major row order (px_poset_set_layout):
    # the chain scans and the combine then stream f and g instead of visiting them in node order
    L.set_layout("rows")
    fr = f[torch.from_numpy(np.argsort(L.rows())).to(dev)].contiguous()
    gr = torch.empty_like(fr)
    tz_rows = _time(lambda: px.zeta(L, fr, out=gr), steps, sync)
    rows_equal = bool(torch.equal(gr[torch.from_numpy(L.rows()).to(dev)], g))
    L.set_layout("nodes")
    del fr, gr
    try:
        f2, rep = px.mobius(L, g, max_refine=2, report=True)
        err = ((f2 - f).abs().amax(0) / f.abs().amax(0)).max().item()
    except px.PosetxError as e:  # the float Möbius of this poset is ill-conditioned
        rep, err = {"status": e.name}, None
    fi = torch.from_numpy(W.functions(q.n, Bl, "int", seed=6, lo=-1000, hi=1000)).to(dev)
    gi = px.zeta(L, fi)
    tm = _time(lambda: px.mobius(L, gi), 2, sync)
    exact = bool(torch.equal(px.mobius(L, gi), fi))
    exact_adj = bool(torch.equal(px.mobius_adjoint(L, px.zeta_adjoint(L, fi)), fi))
    growth = f64_growth(px, L, q.n, dev)
    # autograd through both transforms, loss = Σ w·T(x): zeta's backward is the adjoint walk;
    # Möbius's backward is M^T w, which overflows float32 here like M itself
    from paper_2211_13706_amd.autograd import mobius_fn, zeta_fn
    fa = f.clone().requires_grad_(True)
    wz = torch.randn_like(f)

    def zstep():
        fa.grad = None
        (zeta_fn(L, fa) * wz).sum().backward()
    t_ag = _time(zstep, steps, sync)
    ga = g.clone().requires_grad_(True)
    try:
        (mobius_fn(L, ga) * wz).sum().backward()
        mob_bwd = "finite" if bool(torch.isfinite(ga.grad).all()) else "nonfinite"
    except px.PosetxError as e:
        mob_bwd = e.name
    return {"workload": "n=8388608, k=32, 3 cross edges, B=16", "preprocess_s": round(t_prep, 2),
            "levels": L.info["levels_down"], "zeta_f32_ms": round(tz * 1e3, 4),
            "zeta_node_rhs_per_s": q.n * Bl / tz,
            "zeta_f32_rows_layout_ms": round(tz_rows * 1e3, 4), "rows_layout_equal": rows_equal,
            "mobius_int64_ms": round(tm * 1e3, 4),
            "us_per_level": round(tm * 1e6 / max(1, L.info["levels_down"]), 2),
            "int64_roundtrip_exact": exact, "int64_adjoint_roundtrip_exact": exact_adj,
            "mobius_f64_growth": growth,
            "autograd_zeta_fwd_bwd_ms": round(t_ag * 1e3, 4), "autograd_mobius_bwd": mob_bwd,
            "f32_roundtrip_rel_err": err, "f32_refine_report": rep}


def leg_min_chains(px, dev, steps, n_log2=18, deg=4):
    """The same Erdős–Rényi DAG with a minimum chain decomposition (PX_BUILD_MIN_CHAINS, as many
    chains as the width) against the matching's path cover: k, nnz(N), the decomposition time and
    the float32 zeta / int64 Möbius times at B = 64."""
    import torch
    import workloads as W
    sync = torch.cuda.synchronize
    q = W.er_dag(1 << n_log2, deg, seed=1)
    out = {"workload": f"Erdős–Rényi DAG, n={q.n}, average degree {deg}, B=64"}
    for name, flags in (("path_cover", 0), ("min_chains", px.PX_BUILD_MIN_CHAINS)):
        t0 = time.perf_counter()
        P = px.poset_build(q.n, q.indptr, q.indices, None, None, flags=flags | px.PX_BUILD_NO_ADJOINT, device=0)
        t_build = time.perf_counter() - t0
        f = torch.from_numpy(W.functions(q.n, 64, "normal", seed=5)).to(dev)
        g = torch.empty_like(f)
        P.reserve(torch.float32, 64)
        tz = _time(lambda: px.zeta(P, f, out=g), steps, sync)
        fi = torch.from_numpy(W.functions(q.n, 64, "int", seed=6, lo=-1000, hi=1000)).to(dev)
        gi = px.zeta(P, fi)
        tm = _time(lambda: px.mobius(P, gi), max(2, steps // 4), sync)
        out[name] = {"k": P.info["k"], "nnz_niv": P.info["nnz_niv"], "chains_s": round(P.info["t_chains"], 2),
                     "build_s": round(t_build, 2), "zeta_f32_ms": round(tz * 1e3, 4),
                     "mobius_int64_ms": round(tm * 1e3, 4),
                     "int64_roundtrip_exact": bool(torch.equal(px.mobius(P, gi), fi))}
        del P, f, g, fi, gi
        torch.cuda.empty_cache()
    return out


def leg_er_sparse(px, dev, steps, n_log2=18, deg=4, refine=True):
    """The workload class of the paper's experiments (§5): an Erdős–Rényi DAG of average degree
    `deg`, n = 2^n_log2, chains from the maximum matching.  At n = 2^18, degree 4 its width (about
    53,000) keeps the niv map as rows of its finite entries (about 61M; dense rows would need
    55 GB).  float32 zeta and adjoint at B = 64, the int64 Möbius round trip, the refined float32
    Möbius, and the rate of the sparse gather: its compulsory bytes (the niv rows, P read once, g)
    and the P rows it gathers."""
    import torch
    import workloads as W
    sync = torch.cuda.synchronize
    t0 = time.perf_counter()
    q = W.er_dag(1 << n_log2, deg, seed=1)
    P = px.poset_build(q.n, q.indptr, q.indices, None, None, device=0)
    t_prep = time.perf_counter() - t0
    info = P.info
    n, Bl, nnz = q.n, 64, info["nnz_niv"]
    f = torch.from_numpy(W.functions(n, Bl, "normal", seed=5)).to(dev)
    g = torch.empty_like(f)
    w = torch.empty_like(f)
    P.reserve(torch.float32, Bl)
    tz = _time(lambda: px.zeta(P, f, out=g), steps, sync)
    ta = _time(lambda: px.zeta_adjoint(P, f, out=w), steps, sync)
    lib = px.lib()
    lib.px_profile(1)
    for _ in range(steps):
        px.zeta(P, f, out=g)
    sync()
    ph = profile_read(lib)
    lib.px_profile(0)
    gms, gcnt = ph["gather"]
    t_gather = gms / max(1, gcnt) / 1e3
    gather_bytes = nnz * 4 + (n + 1) * 8 + 2 * n * Bl * 4 + n * 4   # niv rows, P once, g, node ids
    fi = torch.from_numpy(W.functions(n, Bl, "int", seed=6, lo=-1000, hi=1000)).to(dev)
    gi = px.zeta(P, fi)
    tm = _time(lambda: px.mobius(P, gi), steps, sync)
    exact = bool(torch.equal(px.mobius(P, gi), fi))
    exact_adj = bool(torch.equal(px.mobius_adjoint(P, px.zeta_adjoint(P, fi)), fi))
    rep, err, tr = None, None, float("nan")
    if refine:
        try:
            f2, rep = px.mobius(P, g, max_refine=3, report=True)
            err = ((f2 - f).abs().amax(0) / f.abs().amax(0)).max().item()
        except px.PosetxError as e:
            rep, err = {"status": e.name}, None
        tr = _time(lambda: px.mobius(P, g, max_refine=3, tol=-1.0), max(2, steps // 4), sync)
    return {"workload": f"Erdős–Rényi DAG, n={n}, average degree {deg}, matching chains, B=64 float32",
            "k": info["k"], "nnz_niv": nnz, "niv_sparse": info["niv_sparse"], "levels": info["levels_down"],
            "preprocess_s": round(t_prep, 2),
            "zeta_f32_ms": round(tz * 1e3, 4), "zeta_node_rhs_per_s": n * Bl / tz,
            "adjoint_f32_ms": round(ta * 1e3, 4),
            "gather_ms": round(t_gather * 1e3, 4), "gather_alg_GBps": round(gather_bytes / t_gather / 1e9, 1),
            "gathered_row_GBps": round(nnz * Bl * 4 / t_gather / 1e9, 1),
            "mobius_int64_ms": round(tm * 1e3, 4), "int64_roundtrip_exact": exact,
            "int64_adjoint_roundtrip_exact": exact_adj,
            "mobius_f32_refined_ms": round(tr * 1e3, 4) if refine else None, "f32_roundtrip_rel_err": err,
            "f32_refine_report": rep,
            "mobius_f64_growth": f64_growth(px, P, n, dev)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--legs", default="default", choices=["none", "default", "all", "sparse", "batched", "chains",
                                                          "large"],
                    help="extra measurements of the other hot-path rows (all: also the batched, n=2^23 and "
                         "Erdős–Rényi configs; sparse / batched / large: that config alone)")
    ap.add_argument("--copy-ref", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; multi-GPU sharding is a design "
                          "(RHS or poset sharding, no collective), not measured here", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import paper_2211_13706_amd as px
    import workloads as W
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    lib = px.lib()

    t0 = time.perf_counter()
    p = W.chain_poset(N, K, CROSS, seed=SEED)
    t_gen = time.perf_counter() - t0
    t0 = time.perf_counter()
    P = px.poset_build(p.n, p.indptr, p.indices, p.chain_of, p.chain_pos, device=0)
    t_prep = time.perf_counter() - t0
    f_host = W.functions(p.n, B, "normal", seed=2)
    f = torch.from_numpy(f_host).to(dev)
    g = torch.empty_like(f)
    t0 = time.perf_counter()
    tune = P.autotune(torch.float32, B)
    t_tune = time.perf_counter() - t0
    P.reserve(torch.float32, B)
    if args.copy_ref:
        a = torch.empty(64 << 20, dtype=torch.float32, device=dev).normal_()
        bcopy = torch.empty_like(a)
        bcopy.copy_(a)
        torch.cuda.synchronize()

    for _ in range(args.warmup):
        px.zeta(P, f, out=g)
    torch.cuda.synchronize()
    # timed region: K steps with nothing else on the stream
    t0 = time.perf_counter()
    for _ in range(args.steps):
        px.zeta(P, f, out=g)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # the same K steps again with a HIP event pair around every kernel on its
    # launch stream (the per-kernel durations of the roofline); the event
    # markers themselves add time, so this pass does not set `value`
    lib.px_profile(1)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        px.zeta(P, f, out=g)
    torch.cuda.synchronize()
    dt_prof = time.perf_counter() - t1
    prof = profile_read(lib)
    lib.px_profile(0)
    # the same K steps over NROT distinct input and output matrices in turn (1 GiB of
    # inputs at n = 2^20, B = 64, four times the 256 MB last-level cache), so that no
    # step finds its input left in the cache by the step before
    NROT = 4
    fs = [f] + [torch.from_numpy(W.functions(p.n, B, "normal", seed=200 + i)).to(dev) for i in range(NROT - 1)]
    gs = [g] + [torch.empty_like(f) for _ in range(NROT - 1)]
    for i in range(NROT):
        px.zeta(P, fs[i], out=gs[i])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for i in range(args.steps):
        px.zeta(P, fs[i % NROT], out=gs[i % NROT])
    torch.cuda.synchronize()
    dt_rot = time.perf_counter() - t1
    del fs, gs
    # the same K steps with the matrices in the kernels' chain-major row order
    # (px_poset_set_layout): same values bit for bit, permuted; node order stays `value`
    rows_np = P.rows()
    row_idx = torch.from_numpy(rows_np).to(dev)
    fr = torch.empty_like(f)
    fr[row_idx] = f
    gr = torch.empty_like(g)
    P.set_layout("rows")
    for _ in range(max(1, args.warmup)):
        px.zeta(P, fr, out=gr)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        px.zeta(P, fr, out=gr)
    torch.cuda.synchronize()
    dt_rows = time.perf_counter() - t1
    P.set_layout("nodes")
    px.zeta(P, f, out=g)
    rows_equal = bool(torch.equal(gr[row_idx], g))
    del fr, gr, row_idx
    copy_gbps = measured_copy_gbps(dev)

    ms_step = dt * 1e3 / args.steps
    value = p.n * B / (dt / args.steps)
    phases = {}
    compact = prof["apply_combine"][1] > 0
    for name in ("scan_reduce", "scan_carry", "scan_apply", "scan_onepass", "gather", "walk_events",
                 "walk_combine", "apply_combine"):
        ms, cnt = prof[name]
        if cnt:
            avg = ms / cnt
            byt = algorithmic_bytes(name, p.n, P.k, B, 4, compact)
            mv = moved_bytes(name, p.n, P.k, B, 4, P.info, compact)
            phases[name] = {"avg_ms": round(avg, 4), "launches": cnt, "alg_bytes": byt,
                            "GBps": round(byt / (avg * 1e-3) / 1e9, 1) if byt else None,
                            "moved_bytes": mv, "moved_GBps": round(mv / (avg * 1e-3) / 1e9, 1)}
            gb = gathered_bytes(name, P.k, B, 4, P.info)
            if gb:
                phases[name]["gathered_bytes"] = gb
                phases[name]["gathered_GBps"] = round(gb / (avg * 1e-3) / 1e9, 1)
    dom = max((k for k in phases if phases[k]["alg_bytes"]), key=lambda k: phases[k]["avg_ms"])
    ach = phases[dom]["GBps"]
    tr = traffic_for(dom)
    # whole-step bytes of the factored method Z = U V as stated: read f, write P,
    # read P, read niv, write g (20 B per node and right-hand side at k = B);
    # the compact walk moves fewer (the sum of the phases' moved bytes)
    step_bytes = 4 * p.n * B * 4 + p.n * P.k * 4
    moved = sum(ph["moved_bytes"] for ph in phases.values())
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "node·RHS/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "ms_per_step_with_kernel_events": dt_prof * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched zeta forward on a random-height poset, n=1048576, k=64 planted "
                               "chains of 16384, 3 cross edges per element, B=64 float32 RHS ~ N(0,1)",
                   "n": p.n, "k": P.k, "B": B, "edges": p.nedges},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": tr,
                     "alg_bytes_per_launch": phases[dom]["alg_bytes"],
                     "avg_ms": phases[dom]["avg_ms"],
                     "moved_bytes_per_launch": phases[dom]["moved_bytes"],
                     "moved_GBps": phases[dom]["moved_GBps"],
                     "gathered_GBps": phases[dom].get("gathered_GBps"),
                     "copy_GBps": copy_gbps, "frac_of_copy": round(ach / copy_gbps, 4),
                     "traffic_GBps": round(tr / (phases[dom]["avg_ms"] * 1e-3) / 1e9, 1) if tr else None},
        "step_roofline": {"alg_bytes": step_bytes, "GBps": round(step_bytes / (ms_step * 1e-3) / 1e9, 1),
                          "frac": round(step_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                          "path": "compact walk" if compact else "scan + walk over P",
                          "phase_moved_bytes": moved,
                          "phase_moved_GBps": round(moved / (ms_step * 1e-3) / 1e9, 1)},
        "rotating_inputs": {"buffers": NROT, "ms_per_step": dt_rot * 1e3 / args.steps,
                            "node_rhs_per_s": p.n * B / (dt_rot / args.steps),
                            "step_frac": round(step_bytes / (dt_rot / args.steps) / 1e9 / HBM_PEAK_GBS, 4)},
        "rows_layout": {"ms_per_step": dt_rows * 1e3 / args.steps,
                        "node_rhs_per_s": p.n * B / (dt_rows / args.steps),
                        "step_frac": round(step_bytes / (dt_rows / args.steps) / 1e9 / HBM_PEAK_GBS, 4),
                        "equal_to_node_order": rows_equal},
        "phases": phases,
        "preprocess_s": {"total": round(t_prep, 3), **{k: round(v, 3) for k, v in P.info.items()
                                                      if k.startswith("t_")},
                         "niv_device_rounds": P.info["niv_device_rounds"]},
        "walk": {k: P.info[k] for k in ("walk_runs", "walk_events", "walk_snapshots", "walk_T", "walk_emax",
                                        "walk_rows_distinct", "walk_row_loads")},
        "autotune": {**tune, "seconds": round(t_tune, 2)},
        "generate_s": round(t_gen, 3),
        "kernel_hash": kernel_hash(),
    }
    # the host baselines first: the legs below free the headline poset
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(p, f_host, args.cpu_budget)
        cpu_nk = cpu_nk_baseline(P, p, f_host, value)
    if args.legs == "sparse":
        out["legs"] = {"er_sparse": leg_er_sparse(px, dev, max(2, args.steps // 4))}
    elif args.legs == "chains":
        out["legs"] = {"min_chains_n64k": leg_min_chains(px, dev, max(2, args.steps // 4), n_log2=16),
                       "min_chains_n256k": leg_min_chains(px, dev, max(2, args.steps // 4), n_log2=18)}
    elif args.legs == "batched":
        del P
        out["legs"] = {"batched": leg_batched(px, dev, args.steps)}
    elif args.legs == "large":
        del P
        out["legs"] = {"large": leg_large(px, dev, max(2, args.steps // 4))}
    elif args.legs != "none":
        def note(msg):
            print(f"[bench] {msg}", file=sys.stderr, flush=True)
        note("legs: config 1 int64 and adjoint")
        legs = legs_config1(px, P, p, dev, args.steps)
        note("legs: grid Möbius")
        legs["grid_mobius"] = leg_grid(px, dev, args.steps)
        if args.legs == "all":
            del P
            note("legs: batched posets")
            legs["batched"] = leg_batched(px, dev, args.steps)
            note("legs: n = 2^23")
            legs["large"] = leg_large(px, dev, max(2, args.steps // 4))
            note("legs: Erdős–Rényi DAG with sparse niv rows")
            legs["er_sparse"] = leg_er_sparse(px, dev, max(2, args.steps // 4))
            note("legs: Erdős–Rényi DAGs, degree 6 and n = 2^20")
            legs["er_sparse_deg6"] = leg_er_sparse(px, dev, max(2, args.steps // 4), n_log2=16, deg=6)
            legs["er_sparse_n1M"] = leg_er_sparse(px, dev, 3, n_log2=20, deg=4, refine=False)
            note("legs: minimum chain decompositions")
            legs["min_chains"] = leg_min_chains(px, dev, max(2, args.steps // 4))
        out["legs"] = legs
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu
        out["cpu_nk_baseline"] = cpu_nk
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
