"""Parity of the HIP SSSP path with the oracle's Dijkstra: distances and the
canonical (smallest-id tight) parents must match bit-exactly."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import announce, gpu, need_gpu, to_np

pytestmark = gpu


@pytest.fixture(scope="module")
def fg():
    need_gpu()
    import paper_1504_04804_amd as fg
    fg.lib()
    return fg


def check(fg, orc, g, off, col, w, src, **kw):
    announce(f"sssp n={len(off)-1} m={len(col)} src={src} {kw}")
    dist, parent, st = fg.sssp(g, src, **kw)
    d = to_np(dist).astype(np.uint32)
    p = to_np(parent)
    wd, wp = orc.dijkstra(off, col, w, src)
    assert st.status == 0
    assert np.array_equal(d, wd), f"dist mismatch at {np.flatnonzero(d != wd)[:10]}"
    assert np.array_equal(p, wp), f"parent mismatch at {np.flatnonzero(p != wp)[:10]}"
    assert orc.check_sssp(off, col, w, src, d, p) is None
    assert st.reached == int((wd != 0xFFFFFFFF).sum())
    return st


@pytest.mark.parametrize("scale", [10, 12, 16])
def test_rmat_weighted(fg, orc, scale):
    off, col = synth.rmat_csr(scale)
    w = synth.weights(off, col)
    g = fg.Graph(off, col, weights=w)
    for s in [0] + list(synth.sources(off, 3, seed=scale)):
        check(fg, orc, g, off, col, w, int(s))
    check(fg, orc, g, off, col, w, 0, small_frontier=1, small_edges=1)
    check(fg, orc, g, off, col, w, 0, big_degree=2)
    # near-far steps: tiny (many splits, large piles split by the whole
    # grid), below and above the largest weight, and no threshold at all
    for delta in (1, 7, 64, 500, fg.SSSP_NO_THRESHOLD):
        check(fg, orc, g, off, col, w, 0, delta=delta)
    check(fg, orc, g, off, col, w, 0, delta=3, small_frontier=1, small_edges=1)


@pytest.mark.parametrize("delta", [0, 1, 33, 600, 0xFFFFFFFF])
def test_grid_near_far(fg, orc, delta):
    off, col = synth.grid_csr(300, 300)
    w = synth.weights(off, col)
    g = fg.Graph(off, col, weights=w)
    for s in (0, 300 * 150 + 150, 300 * 300 - 1):
        st = check(fg, orc, g, off, col, w, s, delta=delta)
        if delta == 1:
            assert st.iterations > 500  # about one split per distance value


@pytest.mark.parametrize("team,team_e,delta", [(2, 0, 0), (5, 0, 1), (32, 0, 0), (64, 0, 600),
                                               (32, 40, 0), (-1, 0, 0), (3, 0, 0xFFFFFFFF)])
def test_team_mode(fg, orc, team, team_e, delta):
    # small_frontier=1 sends every frontier of more than one vertex to the
    # team (or the full grid when its mean degree is too high)
    off, col = synth.grid_csr(200, 220)
    w = synth.weights(off, col)
    g = fg.Graph(off, col, weights=w)
    for s in (0, 200 * 110 + 37):
        check(fg, orc, g, off, col, w, s, small_frontier=1, small_edges=1, team_blocks=team,
              team_edges=team_e, delta=delta)
    off, col = synth.rmat_csr(13)
    w = synth.weights(off, col)
    g = fg.Graph(off, col, weights=w)
    check(fg, orc, g, off, col, w, 0, small_frontier=1, small_edges=1, team_blocks=team,
          team_edges=team_e, delta=delta)
    check(fg, orc, g, off, col, w, 77, team_blocks=team, team_edges=team_e, delta=delta)


def test_team_handoffs_repeated(fg, orc):
    # back-to-back launches with the team forced on R-MAT and the solo
    # threshold varied, so episodes hand off to each other in quick
    # succession; every run must finish with Dijkstra's distances
    off, col = synth.rmat_csr(14)
    w = synth.weights(off, col)
    g = fg.Graph(off, col, weights=w)
    srcs = [int(s) for s in synth.sources(off, 4, seed=7)]
    want = {s: orc.dijkstra(off, col, w, s)[0] for s in srcs}
    announce("sssp team hand-offs: 60 runs on rmat14")
    for r in range(60):
        s = srcs[r % 4]
        dist, _, st = fg.sssp(g, s, team_blocks=32, small_frontier=(r % 3) * 300 + 1)
        assert st.status == 0, f"run {r}: status {st.status}"
        assert np.array_equal(to_np(dist).astype(np.uint32), want[s]), f"run {r} src {s}"


def test_near_far_gaps(fg, orc):
    # weights far above the step: each split first finds no vertex below the
    # new threshold and jumps to the smallest distance in the pile
    n = 50
    off, col = synth.from_edge_pairs(n, [(i, i + 1) for i in range(n - 1)] + [(0, 25)])
    w = np.full(len(col), 1000, np.uint32)
    g = fg.Graph(off, col, weights=w)
    for delta in (1, 999, 1000, 1001):
        check(fg, orc, g, off, col, w, 0, delta=delta)
        check(fg, orc, g, off, col, w, 0, delta=delta, small_frontier=1, small_edges=1)


def test_closed_forms(fg, orc):
    n = 200
    off, col = synth.from_edge_pairs(n, [(i, i + 1) for i in range(n - 1)])
    wt = np.arange(1, n, dtype=np.uint32)
    w = np.array([wt[min(u, col[k])] for u in range(n) for k in range(off[u], off[u + 1])], np.uint32)
    g = fg.Graph(off, col, weights=w)
    st = check(fg, orc, g, off, col, w, 0)
    R, C = 40, 50
    off, col = synth.grid_csr(R, C)
    w = np.full(len(col), 7, np.uint32)
    g = fg.Graph(off, col, weights=w)
    for delta in (0, 1, 7, 50, fg.SSSP_NO_THRESHOLD):
        dist, parent, st = fg.sssp(g, 0, delta=delta)
        d = to_np(dist)
        assert d.tolist() == [7 * (r + c) for r in range(R) for c in range(C)]
    check(fg, orc, g, off, col, w, R * C // 2 + 7)


def test_zero_weights_and_isolated(fg, orc):
    off, col = synth.rmat_csr(11)
    w = synth.weights(off, col) % 3  # many zero weights (symmetric)
    g = fg.Graph(off, col, weights=w)
    for s in (0, 17):
        check(fg, orc, g, off, col, w, s)
    off, col = synth.from_edge_pairs(6, [(0, 1), (1, 2)])
    w = np.ones(len(col), np.uint32)
    g = fg.Graph(off, col, weights=w)
    check(fg, orc, g, off, col, w, 5)  # isolated source


def test_directed_graph(fg, orc):
    rng = np.random.default_rng(3)
    n = 3000
    eu = rng.integers(0, n, 20000)
    ev = rng.integers(0, n, 20000)
    keep = eu != ev
    pairs = np.unique(np.stack([eu[keep], ev[keep]], 1), axis=0)
    order = np.lexsort((pairs[:, 1], pairs[:, 0]))
    pairs = pairs[order]
    off = np.zeros(n + 1, np.int32)
    np.add.at(off, pairs[:, 0] + 1, 1)
    off = np.cumsum(off).astype(np.int32)
    col = pairs[:, 1].astype(np.int32)
    w = rng.integers(1, 65, len(col)).astype(np.uint32)
    g = fg.Graph(off, col, weights=w, symmetric=False)
    for s in (0, 1, 2):
        check(fg, orc, g, off, col, w, s)


def test_overflow_reported(fg):
    off, col = synth.from_edge_pairs(3, [(0, 1), (1, 2)])
    w = np.full(len(col), 0x90000000, np.uint32)
    g = fg.Graph(off, col, weights=w)
    dist, parent, st = fg.sssp(g, 0)
    assert st.status == fg.FG_EOVERFLOW


def test_sssp_needs_weights(fg):
    off, col = synth.from_edge_pairs(3, [(0, 1)])
    g = fg.Graph(off, col)
    with pytest.raises(fg.FGError) as e:
        fg.sssp(g, 0)
    assert e.value.status == fg.FG_EINVAL


@pytest.mark.slow
def test_config_rmat22_sssp_sampled(fg, orc):
    off, col = synth.rmat_csr(22)
    w = synth.weights(off, col)
    g = fg.Graph(off, col, weights=w)
    for s in synth.sources(off, 64)[:2]:
        check(fg, orc, g, off, col, w, int(s))
