"""Asynchronous push BFS (fg_bfs with FG_MODE_PUSH and async_levels > 1:
a team that synchronises every K levels, label-correcting keys) against
the oracle, through the C ABI: depths bit-exact (closed forms on grids,
FIFO BFS elsewhere), every parent the smallest-id neighbour one level
closer (the key's tie-break), the record's level sizes and per-level
entries equal to the oracle's, and the level-synchronous kernel taking
over when a member's frontier outgrows its LDS room."""
import numpy as np
import pytest
import torch

import synth
import workloads
from gpu_util import announce, gpu, need_gpu, to_np

pytestmark = gpu


@pytest.fixture(scope="module")
def fg():
    need_gpu()
    import paper_1504_04804_amd as fg
    fg.lib()
    return fg


def canonical_parents(off, col, depth, src):
    """min{u in N(v) : depth[u] = depth[v] - 1} for reached v != src."""
    n = len(off) - 1
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(off))
    ok = (depth[rows] > 0) & (depth[col] == depth[rows] - 1)
    best = np.full(n, np.iinfo(np.int64).max)
    np.minimum.at(best, rows[ok], col[ok].astype(np.int64))
    out = np.where(depth >= 0, best, -1)
    out[src] = src
    return out.astype(np.int64)


def run(fg, orc, g, off, col, src, K, T, what, expect_fallback=False):
    announce(f"async bfs {what} src={src} K={K} T={T}")
    o = fg.bfs_opts(mode=fg.FG_MODE_PUSH, async_levels=K, team_blocks=T)
    depth, parent, st = fg.bfs(g, src, opts=o)
    d, p = to_np(depth), to_np(parent)
    want, _, cnt, _ = orc.bfs(off, col, src)
    assert np.array_equal(d, want), (what, src, K, T, np.flatnonzero(d != want)[:8])
    assert orc.check_bfs(off, col, src, d, p) is None
    assert st.status == 0 and st.iterations == len(cnt)
    assert st.reached == int((want >= 0).sum())
    L = min(len(cnt), 64)
    dirs, front, insp = st.trace()
    assert dirs[:L] == [0] * L
    assert front[:L] == cnt[:L].tolist()
    assert insp[:L] == orc.edges_inspected(off, col, want, np.zeros(len(cnt), np.int8))[:L].tolist()
    if not expect_fallback:
        # the team's keys break ties towards the smaller parent id
        assert np.array_equal(p.astype(np.int64), canonical_parents(off, col, want, src))
    return st


@pytest.mark.parametrize("K", [2, 3, 8, 64])
def test_grids_closed_form(fg, orc, K):
    for R, C in ((1, 1), (1, 300), (40, 61), (257, 129)):
        off, col = synth.grid_csr(R, C)
        g = fg.Graph(off, col)
        for src in {0, (R // 2) * C + C // 2, R * C - 1}:
            for T in (1, 3, 24):
                run(fg, orc, g, off, col, src, K, T, f"grid{R}x{C}")
        g.close()


def test_general_graphs(fg, orc):
    """Higher degrees (the block scan-gather path) and graphs where members
    run ahead of each other (depth corrections)."""
    cases = [("rmat10", synth.rmat_csr(10)), ("rmat12", synth.rmat_csr(12))]
    rng = np.random.default_rng(5)
    n = 3000
    eu = rng.integers(0, n, 4000).astype(np.int32)
    ev = rng.integers(0, n, 4000).astype(np.int32)
    cases.append(("er3000", orc.csr_from_edges(n, eu, ev)))
    a = np.array([(0, 1), (1, 2), (5, 6)], np.int32)
    cases.append(("tiny", orc.csr_from_edges(9, a[:, 0], a[:, 1])))
    for what, (off, col) in cases:
        g = fg.Graph(off, col)
        srcs = {0, 3, int(g.n) - 1} | {int(s) for s in synth.sources(off, 2, seed=4)}
        for src in srcs:
            for K, T in ((2, 2), (8, 24), (5, 7)):
                # a member's frontier may outgrow its room on these graphs:
                # the level-synchronous kernel then answers (parents valid,
                # not necessarily the smallest)
                run(fg, orc, g, off, col, src, K, T, what, expect_fallback=True)
        g.close()


def test_overflow_hands_over(fg, orc):
    """A star of 5000 leaves on a team of one: the member's next queue
    outgrows its LDS room after one level, and the level-synchronous
    kernel behind the team runs the traversal."""
    leaves = np.arange(1, 5001, dtype=np.int32)
    off, col = orc.csr_from_edges(5001, np.zeros_like(leaves), leaves)
    g = fg.Graph(off, col)
    for src in (0, 17):
        st = run(fg, orc, g, off, col, src, 8, 1, "star5000", expect_fallback=True)
        assert st.grid_blocks > 1  # the record comes from the full-grid kernel
    g.close()


def test_repeated_calls_and_modes_interleaved(fg, orc):
    """Asynchronous and level-synchronous traversals on one workspace, one
    after the other: each leaves the control block ready for the next."""
    off, col = synth.grid_csr(100, 90)
    g = fg.Graph(off, col)
    for i in range(6):
        src = (i * 977) % g.n
        run(fg, orc, g, off, col, src, 8, 24, "grid100x90")
        depth, parent, st = fg.bfs(g, src, opts=fg.bfs_opts(mode=fg.FG_MODE_PUSH))
        assert np.array_equal(to_np(depth), orc.bfs(off, col, src)[0])
        assert st.status == 0
    g.close()


@pytest.mark.slow
def test_grid4096_workload(fg, orc):
    off, col, _ = workloads.graph("grid4096")
    g = fg.Graph(off, col, symmetric=True, validate=False)
    R = 4096
    for src in (0, (R // 2) * R + R // 2):
        for K in (8, 16):
            announce(f"async grid4096 src={src} K={K}")
            o = fg.bfs_opts(mode=fg.FG_MODE_PUSH, async_levels=K)
            depth, parent, st = fg.bfs(g, src, opts=o)
            d = to_np(depth)
            r0, c0 = divmod(src, R)
            rr = np.abs(np.arange(R, dtype=np.int32) - r0)
            cc = np.abs(np.arange(R, dtype=np.int32) - c0)
            assert np.array_equal(d.reshape(R, R), rr[:, None] + cc[None, :])
            assert st.status == 0 and st.iterations == int(d.max()) + 1
            assert orc.check_bfs(off, col, src, d, to_np(parent)) is None
    g.close()
