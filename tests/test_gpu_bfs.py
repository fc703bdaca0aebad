"""Parity of the HIP BFS path with the serial oracle.

Depths are compared bit-exactly; parents are validated as a BFS tree (they
may legally differ); the per-iteration frontier sizes must equal the
oracle's level histogram; in direction-optimizing mode the direction trace
must equal the oracle's prediction from the level histogram (Sec. VI-A) and
the CSR entries read per iteration must equal the oracle's count for the
early-exit pull (which pins the early exit itself).
"""
import numpy as np
import pytest
import torch

import synth
from gpu_util import announce, gpu, need_gpu, to_np

pytestmark = gpu

MODES = {"do": 0, "push": 1, "unfused": 2}


@pytest.fixture(scope="module")
def fg():
    need_gpu()
    import paper_1504_04804_amd as fg
    fg.lib()
    return fg


def check_bfs(fg, orc, g, off, col, src, mode, do_a=(1, 100), do_b=(1, 10), **kw):
    announce(f"bfs n={len(off)-1} m={len(col)} src={src} mode={mode} {kw}")
    depth, parent, st = fg.bfs(g, src, mode=MODES[mode], do_a=do_a, do_b=do_b, **kw)
    d = to_np(depth)
    p = to_np(parent)
    want, _, cnt, mc = orc.bfs(off, col, src)
    assert st.status == 0
    assert np.array_equal(d, want), f"depth mismatch at {np.flatnonzero(d != want)[:10]}"
    err = orc.check_bfs(off, col, src, d, p)
    assert err is None, err
    L = len(cnt)
    assert st.iterations == L
    assert st.reached == cnt.sum()
    dirs, front, insp = st.trace()
    k = min(L, fg.FG_TRACE_MAX)
    assert front == cnt[:k].tolist()
    if mode == "do":
        want_dirs = orc.do_schedule(cnt, len(off) - 1, len(col), do_a, do_b)
        assert dirs == want_dirs[:k].tolist()
    else:
        want_dirs = np.zeros(L, np.int8)
        assert dirs == [0] * k
    want_insp = orc.edges_inspected(off, col, want, want_dirs)
    assert insp == want_insp[:k].tolist()
    if L <= fg.FG_TRACE_MAX:
        assert st.edges_inspected == want_insp.sum()
    return st


@pytest.fixture(scope="module")
def rmat12(fg):
    off, col = synth.rmat_csr(12)
    return off, col, fg.Graph(off, col)


@pytest.mark.parametrize("mode", ["do", "push", "unfused"])
def test_rmat12_from_vertex0(fg, orc, rmat12, mode):
    off, col, g = rmat12
    check_bfs(fg, orc, g, off, col, 0, mode)


@pytest.mark.parametrize("mode", ["do", "push"])
def test_rmat12_random_sources(fg, orc, rmat12, mode):
    off, col, g = rmat12
    for s in synth.sources(off, 6, seed=77):
        check_bfs(fg, orc, g, off, col, int(s), mode)


def test_rmat12_forced_paths(fg, orc, rmat12):
    """Full-grid iterations only, tiny big-degree cut (phase B on), and an
    always-pull / never-pull schedule: results must not change."""
    off, col, g = rmat12
    for s in (0, 5, 100):
        check_bfs(fg, orc, g, off, col, s, "do", small_frontier=1, small_edges=1)
        check_bfs(fg, orc, g, off, col, s, "push", small_frontier=1, small_edges=1, big_degree=2)
        check_bfs(fg, orc, g, off, col, s, "do", do_a=(0, 1), do_b=(0, 1))
        check_bfs(fg, orc, g, off, col, s, "do", do_a=(0, 1), do_b=(10**6, 1))
        check_bfs(fg, orc, g, off, col, s, "do", do_a=(10**6, 1))


def test_closed_form_graphs(fg, orc):
    # path, grid, star, isolated source, disconnected union, single vertex
    cases = []
    n = 300
    cases.append(("path", synth.from_edge_pairs(n, [(i, i + 1) for i in range(n - 1)]), [0, 150, 299]))
    cases.append(("grid", synth.grid_csr(33, 47), [0, 16 * 47 + 23, 33 * 47 - 1]))
    cases.append(("star", synth.from_edge_pairs(2000, [(0, i) for i in range(1, 2000)]), [0, 7]))
    cases.append(("iso", synth.from_edge_pairs(10, [(0, 1), (1, 2)]), [9, 0]))
    cases.append(("two", synth.from_edge_pairs(8, [(0, 1), (1, 2), (4, 5), (5, 6), (6, 7)]), [6, 1]))
    cases.append(("single", (np.zeros(2, np.int32), np.zeros(0, np.int32)), [0]))
    for name, (off, col), srcs in cases:
        g = fg.Graph(off, col)
        for s in srcs:
            for mode in ("do", "push"):
                check_bfs(fg, orc, g, off, col, s, mode)


@pytest.mark.parametrize("scale", [14, 16])
def test_rmat_medium(fg, orc, scale):
    off, col = synth.rmat_csr(scale)
    g = fg.Graph(off, col)
    for s in synth.sources(off, 3, seed=scale):
        for mode in ("do", "push"):
            check_bfs(fg, orc, g, off, col, int(s), mode)
    check_bfs(fg, orc, g, off, col, 0, "do", big_degree=64, small_frontier=1)


def test_grid_high_diameter(fg, orc):
    off, col = synth.grid_csr(256, 256)
    g = fg.Graph(off, col)
    for s in (0, 128 * 256 + 128):
        check_bfs(fg, orc, g, off, col, s, "push")
    check_bfs(fg, orc, g, off, col, 0, "push", small_frontier=1, small_edges=1)
    # full-grid levels only, every vertex cut into descriptors (phase B on
    # every level), the same workspace reused across the runs
    for src in (0, 255, 128 * 256 + 128):
        check_bfs(fg, orc, g, off, col, src, "push", small_frontier=1, small_edges=1,
                  team_blocks=-1, big_degree=2)
    # team levels whose shares drift apart (the frontier grows at its ends)
    check_bfs(fg, orc, g, off, col, 0, "push", small_edges=1, team_blocks=8)
    check_bfs(fg, orc, g, off, col, 128 * 256 + 128, "push", small_edges=1, team_blocks=64)


def test_lds_queue_modes(fg, orc, rmat12):
    """Levels run by one workgroup or a team from LDS queues: team widths
    from 2 to the whole grid, and a hub whose 3000 neighbours exceed one
    workgroup's LDS queue, so the overflow goes to the global queue."""
    n = 6001
    edges = [(0, i) for i in range(1, 3001)] + [(i, i + 3000) for i in range(1, 3001)]
    off, col = synth.from_edge_pairs(n, edges)
    g = fg.Graph(off, col)
    for mode in ("do", "push"):
        check_bfs(fg, orc, g, off, col, 0, mode)
        check_bfs(fg, orc, g, off, col, 0, mode, small_edges=1, team_blocks=2)
        check_bfs(fg, orc, g, off, col, 0, mode, small_edges=1, team_blocks=7, team_edges=1 << 20)
        check_bfs(fg, orc, g, off, col, 4000, mode, small_frontier=1, team_blocks=3)
    # 100 vertices of degree 51 (mean degree low enough for LDS levels)
    # discover 5000 leaves: more than one workgroup's LDS queue holds
    edges = [(0, i) for i in range(1, 101)]
    edges += [(i, 101 + 50 * (i - 1) + j) for i in range(1, 101) for j in range(50)]
    off, col = synth.from_edge_pairs(5101, edges)
    g = fg.Graph(off, col)
    for mode in ("do", "push"):
        check_bfs(fg, orc, g, off, col, 0, mode, small_edges=1 << 18)
        check_bfs(fg, orc, g, off, col, 0, mode, small_edges=1, team_blocks=2)
        check_bfs(fg, orc, g, off, col, 0, mode, small_edges=1, team_blocks=3, team_edges=1 << 18)
    off, col, g = rmat12
    for team in (-1, 2, 5, 64, 10**6):
        for s in (0, 5):
            check_bfs(fg, orc, g, off, col, s, "push", team_blocks=team)
            check_bfs(fg, orc, g, off, col, s, "push", team_blocks=team, small_edges=1,
                      team_edges=1 << 30)
            check_bfs(fg, orc, g, off, col, s, "do", team_blocks=team, small_edges=1,
                      team_edges=1 << 30)


def test_repeat_determinism(fg, orc, rmat12):
    """Atomic races must not change depths: 50 repeats, identical depths."""
    off, col, g = rmat12
    want = orc.bfs(off, col, 3)[0]
    for _ in range(50):
        d, p, st = fg.bfs(g, 3, mode=0)
        assert np.array_equal(to_np(d), want)


@pytest.mark.slow
def test_config_rmat22_dobfs_sampled(fg, orc):
    """Full-size RMAT scale 22 DOBFS in the benchmark's launch configuration."""
    off, col = synth.rmat_csr(22)
    g = fg.Graph(off, col)
    for s in synth.sources(off, 64)[:4]:
        check_bfs(fg, orc, g, off, col, int(s), "do")


@pytest.mark.slow
def test_config_grid4096_push(fg, orc):
    off, col = synth.grid_csr(4096, 4096)
    g = fg.Graph(off, col)
    announce("grid 4096x4096 push from 0")
    depth, parent, st = fg.bfs(g, 0, mode=1)
    d = to_np(depth)
    r = np.arange(4096, dtype=np.int32)
    assert np.array_equal(d.reshape(4096, 4096), r[:, None] + r[None, :])
    assert st.iterations == 8191
    assert orc.check_bfs(off, col, 0, d, to_np(parent)) is None


def test_workspace_alignment_checked(fg, orc):
    """A workspace whose start is not 256-byte aligned is refused with
    FG_EINVAL before anything runs (every primitive carves its workspace
    into 256-byte aligned pieces); the aligned one still works."""
    off, col = synth.rmat_csr(8)
    g = fg.Graph(off, col)
    need = g.workspace_bytes(fg.FG_PRIM_BFS)
    big = torch.zeros(need + 512, dtype=torch.uint8, device="cuda")
    depth = torch.empty(g.n, dtype=torch.int32, device="cuda")
    for shift in (16, 128):
        with pytest.raises(fg.FGError) as e:
            fg.bfs_into(g, 0, depth, None, fg.bfs_opts(), ws=big[shift:shift + need])
        assert e.value.status == fg.FG_EINVAL
        srcs = torch.zeros(2, dtype=torch.int32, device="cuda")
        with pytest.raises(fg.FGError) as e:
            fg.bfs_many_into(g, srcs, depth, None, fg.bfs_opts(), ws=big[shift:shift + need])
        assert e.value.status == fg.FG_EINVAL
        with pytest.raises(fg.FGError) as e:
            fg.cc_into(g, torch.empty(g.n, dtype=torch.int32, device="cuda"),
                       ws=big[shift:shift + 64])
        assert e.value.status == fg.FG_EINVAL
    fg.bfs_into(g, 0, depth, None, fg.bfs_opts(), ws=big[256:256 + need])
    assert np.array_equal(to_np(depth), orc.bfs(off, col, 0)[0])
    g.close()
