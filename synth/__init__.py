"""Seeded synthetic inputs shared by the oracle and the GPU path.

Holds no traversal arithmetic: R-MAT edge lists and their undirected simple
CSR (the paper's preprocessing, Sec. VII-A), 2D grids, symmetric weights in
[1, 64], random nonzero-degree sources and random partition owners (Sec. V-C).
Random numbers are counter-based SplitMix64 outputs (see synth.c).

The C code is compiled to ``synth/libsynth.so`` by ``__graft_entry__.build()``.
"""
import ctypes
import os
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None

# Fixed seeds of the workloads (graph, weights, sources, partition are distinct).
SEED_GRAPH = 0x5EED0001
SEED_WEIGHT = 0x5EED0002
SEED_SOURCE = 0x5EED0003
SEED_OWNER = 0x5EED0004

RMAT_ABCD = (Fraction(57, 100), Fraction(19, 100), Fraction(19, 100), Fraction(5, 100))


def build_cmd():
    return ["gcc", "-O3", "-fPIC", "-shared", "-fopenmp", "-std=c11",
            os.path.join(_HERE, "synth.c"), "-o", _LIB_PATH]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    lib.syn_ctr_u64.restype = ctypes.c_uint64
    lib.syn_ctr_u64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    lib.syn_rmat_edges.restype = None
    lib.syn_rmat_edges.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                                   ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, P, P]
    lib.syn_csr_build.restype = ctypes.c_int64
    lib.syn_csr_build.argtypes = [ctypes.c_int32, ctypes.c_int64, P, P, P, P, P]
    lib.syn_grid_csr.restype = ctypes.c_int64
    lib.syn_grid_csr.argtypes = [ctypes.c_int32, ctypes.c_int32, P, P]
    lib.syn_weights.restype = None
    lib.syn_weights.argtypes = [ctypes.c_int32, P, P, ctypes.c_uint64, P]
    lib.syn_sources.restype = ctypes.c_int32
    lib.syn_sources.argtypes = [ctypes.c_int32, P, ctypes.c_uint64, ctypes.c_int32, P]
    lib.syn_owner.restype = None
    lib.syn_owner.argtypes = [ctypes.c_int32, ctypes.c_uint64, ctypes.c_int32, P]
    _lib = lib
    return lib


def _p(a):
    return ctypes.c_void_p(a.ctypes.data)


def ctr_u64(seed, i):
    """i-th SplitMix64 output for `seed` (counter-based)."""
    return int(_load().syn_ctr_u64(seed & (2**64 - 1), i))


def rmat_thresholds(abcd=RMAT_ABCD):
    a, b, c, _ = abcd
    t1 = int(a * 2**64)
    t2 = int((a + b) * 2**64)
    t3 = int((a + b + c) * 2**64)
    return t1, t2, t3


def rmat_edges(scale, edge_factor=16, seed=SEED_GRAPH, abcd=RMAT_ABCD):
    """Directed R-MAT edge list (eu, ev) of edge_factor * 2**scale edges."""
    ne = edge_factor * (1 << scale)
    eu = np.empty(ne, dtype=np.int32)
    ev = np.empty(ne, dtype=np.int32)
    t1, t2, t3 = rmat_thresholds(abcd)
    _load().syn_rmat_edges(scale, ne, seed, t1, t2, t3, _p(eu), _p(ev))
    return eu, ev


def csr_from_edges(n, eu, ev):
    """Undirected simple CSR (row_offsets int32[n+1], cols int32[m])."""
    lib = _load()
    eu = np.ascontiguousarray(eu, dtype=np.int32)
    ev = np.ascontiguousarray(ev, dtype=np.int32)
    tmp = np.empty(n + 1, dtype=np.int64)
    off = np.empty(n + 1, dtype=np.int32)
    slots = lib.syn_csr_build(n, len(eu), _p(eu), _p(ev), _p(tmp), _p(off), None)
    if slots >= 2**31:
        raise ValueError("graph too large for int32 CSR")
    cols = np.empty(max(slots, 1), dtype=np.int32)
    m = lib.syn_csr_build(n, len(eu), _p(eu), _p(ev), _p(tmp), _p(off), _p(cols))
    return off, (cols[:m].copy() if m != len(cols) else cols)


def rmat_csr(scale, edge_factor=16, seed=SEED_GRAPH):
    eu, ev = rmat_edges(scale, edge_factor, seed)
    return csr_from_edges(1 << scale, eu, ev)


def grid_csr(rows, cols):
    n = rows * cols
    m = 2 * (rows * (cols - 1) + (rows - 1) * cols)
    off = np.empty(n + 1, dtype=np.int32)
    col = np.empty(max(m, 1), dtype=np.int32)
    _load().syn_grid_csr(rows, cols, _p(off), _p(col))
    return off, col[:m]


def weights(off, cols, seed=SEED_WEIGHT):
    n = len(off) - 1
    w = np.empty(len(cols), dtype=np.uint32)
    _load().syn_weights(n, _p(off), _p(cols), seed, _p(w))
    return w


def sources(off, k, seed=SEED_SOURCE):
    n = len(off) - 1
    out = np.empty(k, dtype=np.int32)
    got = _load().syn_sources(n, _p(off), seed, k, _p(out))
    return out[:got]


def owners(n, parts=4, seed=SEED_OWNER):
    out = np.empty(n, dtype=np.uint8)
    _load().syn_owner(n, seed, parts, _p(out))
    return out


def from_edge_pairs(n, pairs):
    """Small helper for tests: CSR of an explicit undirected edge list."""
    if len(pairs) == 0:
        eu = np.zeros(0, np.int32)
        ev = np.zeros(0, np.int32)
    else:
        a = np.asarray(pairs, dtype=np.int32)
        eu, ev = a[:, 0].copy(), a[:, 1].copy()
    return csr_from_edges(n, eu, ev)
