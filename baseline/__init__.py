"""The straightforward O(n·k) CPU transforms (C++17 + OpenMP, ``nk_cpu.cpp``).

A reported baseline for the GPU library, timed on the host's own cores next to
it: Alg. 3 (chain prefix sums, then the niv gather) for zeta and Alg. 4 with
the level schedule of Alg. 5 for Möbius, on the same dense niv map and level
schedule as the GPU handle.  It is neither the oracle nor part of the GPU path.

    from baseline import build, NkCpu
    build()                          # g++ -O3 -fopenmp, two builds (AVX2 and generic x86-64)
    cpu = NkCpu(P)                   # P: a paper_2211_13706_amd.Poset with dense niv rows
    g = cpu.zeta(f)                  # numpy [n, B] float32 or int64, node order
    sec = cpu.time_zeta(f, reps=5)   # steady_clock median of 5 after one warm-up
"""

from __future__ import annotations

import ctypes
import os
import shutil
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "nk_cpu.cpp")
LIBS = {"v3": os.path.join(HERE, "libnkcpu_v3.so"), "generic": os.path.join(HERE, "libnkcpu.so")}
FLAGS = {"v3": ["-march=x86-64-v3"], "generic": []}


def build() -> None:
    """Compile both builds in-tree (every call)."""
    gxx = shutil.which("g++") or "g++"
    for key, out in LIBS.items():
        tmp = out + ".tmp"
        cmd = [gxx, "-O3", "-std=c++17", "-fopenmp", "-fPIC", "-shared", *FLAGS[key], SRC, "-o", tmp]
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        if r.returncode != 0:
            raise RuntimeError("command failed:\n" + " ".join(cmd) + "\n" + r.stdout)
        os.replace(tmp, out)


def _cpu_flags() -> set:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("flags"):
                    return set(line.split(":", 1)[1].split())
    except OSError:
        pass
    return set()


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads() -> tuple:
    """(threads to use, CPUs in this process's affinity mask): the affinity mask, capped by
    OMP_NUM_THREADS when the environment sets a share of the host."""
    aff = len(os.sched_getaffinity(0))
    cap = os.environ.get("OMP_NUM_THREADS", "")
    threads = min(aff, int(cap)) if cap.isdigit() and int(cap) > 0 else aff
    return threads, aff


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        key = "v3" if {"avx2", "fma", "bmi2"} <= _cpu_flags() else "generic"
        path = LIBS[key]
        if not os.path.exists(path):
            raise ImportError(f"{path} is not built; call baseline.build()")
        L = ctypes.CDLL(path)
        P, i32, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
        L.nk_set_threads.argtypes, L.nk_set_threads.restype = [i32], i32
        L.nk_zeta.argtypes, L.nk_zeta.restype = [i32, i64, i64, i64, P, P, P, P, P, P], i32
        L.nk_mobius.argtypes, L.nk_mobius.restype = [i32, i64, i64, i64, P, P, P, P, P, P, i64, P, P, P], i32
        L.nk_time_zeta.argtypes = [i32, i64, i64, i64, P, P, P, P, P, P, i32, P]
        L.nk_time_zeta.restype = ctypes.c_double
        L.nk_time_mobius.argtypes = [i32, i64, i64, i64, P, P, P, P, P, P, i64, P, P, P, i32, P]
        L.nk_time_mobius.restype = ctypes.c_double
        L.variant = key
        _LIB = L
    return _LIB


def _code(a):
    if a.dtype == np.int64:
        return 0
    if a.dtype == np.float32:
        return 1
    raise TypeError("int64 or float32 matrices")


class NkCpu:
    """The chain-major numbering, dense niv rows and level schedule of a GPU poset handle,
    laid out for the CPU transforms."""

    def __init__(self, P, threads: int | None = None):
        n, k = P.n, P.k
        row_of_node = P.rows()
        self.n, self.k = n, k
        self.node_of_row = np.empty(n, np.int32)
        self.node_of_row[row_of_node] = np.arange(n, dtype=np.int32)
        chain_of, _ = P.chains()
        self.chain_off = np.concatenate([[0], np.cumsum(np.bincount(chain_of, minlength=k))]).astype(np.int32)
        self.chain_of_row = np.ascontiguousarray(chain_of[self.node_of_row], dtype=np.int32)
        niv = P.niv()[self.node_of_row]                      # rows in chain-major order, entries node ids
        self.niv_rows = np.where(niv >= 0, row_of_node[np.maximum(niv, 0)], -1).astype(np.int32)
        lev = P.levels()[self.node_of_row]
        self.lev_rows = np.argsort(lev, kind="stable").astype(np.int32)
        self.lev_ptr = np.concatenate([[0], np.cumsum(np.bincount(lev))]).astype(np.int32)
        self.nlev = len(self.lev_ptr) - 1
        t, self.affinity = host_threads()
        self.threads = lib().nk_set_threads(int(threads or t))

    def _args(self, x):
        x = np.ascontiguousarray(x)
        if x.ndim != 2 or x.shape[0] != self.n:
            raise ValueError(f"[{self.n}, B] matrix expected")
        return x, np.empty_like(x), np.empty(x.shape, np.float64 if x.dtype == np.float32 else np.uint64)

    def zeta(self, f):
        f, g, w = self._args(f)
        st = lib().nk_zeta(_code(f), self.n, self.k, f.shape[1], self.chain_off.ctypes.data,
                           self.node_of_row.ctypes.data, self.niv_rows.ctypes.data, f.ctypes.data,
                           g.ctypes.data, w.ctypes.data)
        if st:
            raise ValueError("nk_zeta rejected its arguments")
        return g

    def mobius(self, g):
        g, f, w = self._args(g)
        st = lib().nk_mobius(_code(g), self.n, self.k, g.shape[1], self.chain_of_row.ctypes.data,
                             self.chain_off.ctypes.data, self.node_of_row.ctypes.data, self.niv_rows.ctypes.data,
                             self.lev_ptr.ctypes.data, self.lev_rows.ctypes.data, self.nlev, g.ctypes.data,
                             f.ctypes.data, w.ctypes.data)
        if st:
            raise ValueError("nk_mobius rejected its arguments")
        return f

    def time_zeta(self, f, reps: int = 5):
        f, g, w = self._args(f)
        return lib().nk_time_zeta(_code(f), self.n, self.k, f.shape[1], self.chain_off.ctypes.data,
                                  self.node_of_row.ctypes.data, self.niv_rows.ctypes.data, f.ctypes.data,
                                  g.ctypes.data, w.ctypes.data, int(reps), None)

    def time_mobius(self, g, reps: int = 5):
        g, f, w = self._args(g)
        return lib().nk_time_mobius(_code(g), self.n, self.k, g.shape[1], self.chain_of_row.ctypes.data,
                                    self.chain_off.ctypes.data, self.node_of_row.ctypes.data,
                                    self.niv_rows.ctypes.data, self.lev_ptr.ctypes.data, self.lev_rows.ctypes.data,
                                    self.nlev, g.ctypes.data, f.ctypes.data, w.ctypes.data, int(reps), None)
