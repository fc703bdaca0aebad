"""Seeded workload graphs shared by the config-scale tests (generator calls
only, no arithmetic of the method), cached for the pytest session, and a
thread pool for running many oracle queries side by side: the oracle is a
serial C library called through ctypes, which releases the GIL, so one
query per thread runs on its own core."""
import os
from concurrent.futures import ThreadPoolExecutor

import synth

EDGE_FACTOR = 16
_cache = {}


def graph(name):
    """(row_offsets, cols, weights) of a named workload graph:
    rmatS (R-MAT scale S, edge factor 16) or gridN (N x N grid); weights are
    the symmetric uint32 weights in [1, 64]."""
    if name not in _cache:
        if name.startswith("rmat"):
            off, col = synth.rmat_csr(int(name[4:]), EDGE_FACTOR)
        elif name.startswith("grid"):
            r = int(name[4:])
            off, col = synth.grid_csr(r, r)
        else:
            raise KeyError(name)
        _cache[name] = (off, col, synth.weights(off, col))
    return _cache[name]


def drop(name):
    _cache.pop(name, None)


def threads():
    # the GPU machines give each GPU a 16-core share, whatever os.cpu_count() says
    return max(1, min(16, os.cpu_count() or 1))


def pool():
    return ThreadPoolExecutor(max_workers=threads())
