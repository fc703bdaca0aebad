"""Pins of the oracle functions behind the widened rows: duplicate-all +
broadcast DOBFS (O11), connected components (O12) and PageRank (O13).

Each is checked against facts that do not come from the function itself:
a hand-worked example (tests/golden, with its citation), closed forms,
brute force on tiny inputs, an independent library routine
(scipy.sparse.csgraph) or an independent formulation (a dense linear
solve), so that a dropped term, a wrong index or a swapped operand fails.
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def csr_of(n, pairs, orc):
    a = np.asarray(pairs, np.int32).reshape(-1, 2)
    return orc.csr_from_edges(n, a[:, 0], a[:, 1])


def er_graph(n, p, seed):
    rng = np.random.default_rng(seed)
    iu = np.triu_indices(n, 1)
    keep = rng.random(len(iu[0])) < p
    return iu[0][keep].astype(np.int32), iu[1][keep].astype(np.int32)


# ------------------------------------------------ O11 duplicate-all DOBFS

def test_dupall_golden(orc):
    g = golden("dobfs_dupall.json")
    off, col = csr_of(g["n"], g["edges"], orc)
    depth, dirs, it = orc.dobfs_dupall(off, col, g["owner"], g["nparts"], g["src"],
                                       tuple(g["do_a"]), tuple(g["do_b"]))
    assert depth.tolist() == g["depth"]
    assert dirs.tolist() == g["dirs"]
    assert it == g["iterations"]


THRESH = [((1, 100), (1, 10)), ((1, 100000), (1, 1)), ((0, 1), (1, 1)), ((1 << 30, 1), (1, 1)),
          ((1, 2), (1, 1000))]


@pytest.mark.parametrize("nparts", [1, 2, 3, 4])
def test_dupall_equals_bfs_and_schedule(orc, nparts):
    """Global depths equal the FIFO BFS (O2) and the direction trace equals
    the single-graph prediction from the level sizes (O3): duplicate-all +
    broadcast leaves every partition with the whole level after each
    iteration, whatever the direction."""
    cases = [synth.rmat_csr(10), synth.rmat_csr(11), synth.grid_csr(9, 13)]
    eu, ev = er_graph(90, 0.04, 3)
    cases.append(orc.csr_from_edges(90, eu, ev))
    for ci, (off, col) in enumerate(cases):
        n = len(off) - 1
        owner = synth.owners(n, nparts, seed=ci + 7)
        for src in [0] + [int(s) for s in synth.sources(off, 3, seed=ci)]:
            want, _, cnt, _ = orc.bfs(off, col, src)
            for da, db in THRESH:
                depth, dirs, it = orc.dobfs_dupall(off, col, owner, nparts, src, da, db)
                assert np.array_equal(depth, want), (ci, src, da, db)
                assert it == len(cnt)
                sched = orc.do_schedule(cnt, n, len(col), da, db)
                assert dirs.tolist() == sched.tolist(), (ci, src, da, db)


def test_dupall_closed_forms(orc):
    # path 0-1-...-29 with alternating owners: depth |i - s|
    n = 30
    off, col = csr_of(n, [(i, i + 1) for i in range(n - 1)], orc)
    owner = np.arange(n) % 3
    for s in (0, 13, 29):
        for da, db in THRESH:
            d, _, it = orc.dobfs_dupall(off, col, owner, 3, s, da, db)
            assert d.tolist() == [abs(i - s) for i in range(n)]
            assert it == max(s, n - 1 - s) + 1
    # grid: Manhattan distance from the corner; a disconnected vertex stays -1
    off, col = synth.grid_csr(6, 7)
    owner = synth.owners(42, 4, seed=1)
    d, _, _ = orc.dobfs_dupall(off, col, owner, 4, 0, (1, 10), (1, 1))
    assert d.tolist() == [r + c for r in range(6) for c in range(7)]
    off, col = csr_of(5, [(0, 1), (1, 2)], orc)
    d, _, _ = orc.dobfs_dupall(off, col, [1, 0, 1, 0, 1], 2, 2, (0, 1), (1, 1))
    assert d.tolist() == [2, 1, 0, -1, -1]


# -------------------------------------------------------------- O12 CC

def test_cc_golden_and_isolated(orc):
    off, col = csr_of(7, [(1, 3), (3, 5), (2, 6)], orc)
    label, c = orc.cc(off, col)
    assert label.tolist() == [0, 1, 2, 1, 4, 1, 2]
    assert c == 4
    off, col = csr_of(5, [], orc)
    label, c = orc.cc(off, col)
    assert label.tolist() == list(range(5)) and c == 5


@pytest.mark.parametrize("seed", range(4))
def test_cc_matches_scipy_and_reachability(orc, seed):
    """Same partition as scipy's connected_components, every label the
    smallest id of its part; on tiny graphs, u and v share a label iff
    Floyd-Warshall finds a path."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(40, 400))
    eu, ev = er_graph(n, 1.2 / n, seed)
    off, col = orc.csr_from_edges(n, eu, ev)
    label, c = orc.cc(off, col)
    A = sp.csr_matrix((np.ones(len(col)), col, off), shape=(n, n))
    nc, comp = csg.connected_components(A, directed=False)
    assert c == nc
    mins = np.full(nc, n)
    np.minimum.at(mins, comp, np.arange(n))
    assert np.array_equal(label, mins[comp])
    small = 60
    eu, ev = er_graph(small, 0.03, seed + 10)
    off, col = orc.csr_from_edges(small, eu, ev)
    label, _ = orc.cc(off, col)
    D = orc.floyd_warshall(off, col)
    reach = D < np.iinfo(np.uint64).max
    same = label[:, None] == label[None, :]
    assert np.array_equal(same, reach | np.eye(small, dtype=bool))


def test_cc_rmat_and_grid(orc):
    off, col = synth.grid_csr(11, 3)
    label, c = orc.cc(off, col)
    assert c == 1 and not label.any()
    off, col = synth.rmat_csr(12)
    label, c = orc.cc(off, col)
    A = sp.csr_matrix((np.ones(len(col)), col, off), shape=(len(off) - 1, len(off) - 1))
    nc, comp = csg.connected_components(A, directed=False)
    assert c == nc
    # isolated vertices (R-MAT has many) are their own components
    iso = np.flatnonzero(np.diff(off) == 0)
    assert np.array_equal(label[iso], iso)


# ------------------------------------------------------- O13 PageRank

def test_pagerank_regular_graphs_stay_uniform(orc):
    """On a regular graph (complete, cycle) rank 1/n is the fixed point: the
    rank each vertex receives equals what it gives away."""
    n = 9
    off, col = csr_of(n, [(i, j) for i in range(n) for j in range(i + 1, n)], orc)
    r, it = orc.pagerank(off, col, 0.85, 0.0, 7)
    assert it == 7 and np.allclose(r, 1.0 / n, rtol=0, atol=1e-15)
    off, col = csr_of(12, [(i, (i + 1) % 12) for i in range(12)], orc)
    r, _ = orc.pagerank(off, col, 0.6, 0.0, 5)
    assert np.allclose(r, 1.0 / 12, rtol=0, atol=1e-15)


def test_pagerank_star_closed_form(orc):
    """Star with k leaves, n = k + 1: the fixed point solves
    c = (1-d)/n + d k l, l = (1-d)/n + d c / k, so c = (1 + d k) / (n (1 + d))."""
    k, d = 7, 0.85
    n = k + 1
    off, col = csr_of(n, [(0, i) for i in range(1, n)], orc)
    r, it = orc.pagerank(off, col, d, 1e-14, 2000)
    c = (1 + d * k) / (n * (1 + d))
    l = (1 - d) / n + d * c / k
    assert it < 2000
    assert abs(r[0] - c) < 1e-12 and np.allclose(r[1:], l, rtol=0, atol=1e-12)


@pytest.mark.parametrize("seed", range(3))
def test_pagerank_matches_dense_iteration_and_solve(orc, seed):
    """Against a dense formulation: r' = (1-d)/n + d A^T D^-1 r (zero
    columns for vertices of degree 0) iterated t times, and against the
    fixed point from a linear solve of (I - d A^T D^-1) r = (1-d)/n."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(30, 120))
    eu, ev = er_graph(n, 2.5 / n, seed)
    off, col = orc.csr_from_edges(n, eu, ev)
    d = 0.85
    A = sp.csr_matrix((np.ones(len(col)), col, off), shape=(n, n)).toarray()
    deg = A.sum(axis=1)
    W = np.where(deg[:, None] > 0, A / np.maximum(deg, 1)[:, None], 0.0)  # row u: 1/deg(u)
    r = np.full(n, 1.0 / n)
    for _ in range(13):
        r = (1 - d) / n + d * (W.T @ r)
    got, it = orc.pagerank(off, col, d, 0.0, 13)
    assert it == 13 and np.allclose(got, r, rtol=1e-13, atol=0)
    fixed = np.linalg.solve(np.eye(n) - d * W.T, np.full(n, (1 - d) / n))
    conv, it2 = orc.pagerank(off, col, d, 1e-13, 10000)
    assert it2 < 10000 and np.allclose(conv, fixed, rtol=1e-9, atol=0)


def test_pagerank_threshold_stops_when_all_updates_small(orc):
    """The threshold-ratio rule: the run stops after the first iteration in
    which no vertex's rank moved by more than tol times its old value."""
    off, col = synth.rmat_csr(9)
    tol = 1e-4
    r_stop, it = orc.pagerank(off, col, 0.85, tol, 500)
    prev, _ = orc.pagerank(off, col, 0.85, 0.0, it - 1)
    cur, _ = orc.pagerank(off, col, 0.85, 0.0, it)
    assert np.array_equal(cur, r_stop)
    assert np.all(np.abs(cur - prev) <= tol * prev)
    before, _ = orc.pagerank(off, col, 0.85, 0.0, it - 2)
    assert np.any(np.abs(prev - before) > tol * before)
