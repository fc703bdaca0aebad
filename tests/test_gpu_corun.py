"""fg_bfs_corun (a list of sources and one asynchronous push query side by
side in one launch) against the oracle, through the C ABI: each list
traversal's depths bit-exact with a valid parent tree and the record of
fg_bfs_many (level sizes, direction trace), the push query's depths the
oracle's with a valid parent tree, also when its team gives up and the
level-synchronous launch answers; shared outputs; no list; the argument
checks."""
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


def corun(fg, g, srcs, opts, stride, g2, src2, opts2):
    n = g.n
    rows = len(srcs) if stride else 1
    depth = torch.full((max(rows, 1) * n,), -7, dtype=torch.int32, device="cuda")
    parent = torch.full((max(rows, 1) * n,), -7, dtype=torch.int32, device="cuda")
    stats = fg.new_stats_many(max(len(srcs), 1))
    depth2 = torch.full((g2.n,), -7, dtype=torch.int32, device="cuda")
    parent2 = torch.full((g2.n,), -7, dtype=torch.int32, device="cuda")
    stats2 = fg.new_stats()
    s = torch.tensor(srcs, dtype=torch.int32, device="cuda")
    fg.bfs_corun_into(g, s, depth, parent, opts, None, stats, g2, src2, depth2, parent2, opts2,
                      stats2=stats2, out_stride=n if stride else 0)
    torch.cuda.synchronize()
    sts = fg.read_stats_many(stats, len(srcs)) if srcs else []
    return depth, parent, sts, depth2, parent2, fg.read_stats(stats2)


def check_list_record(orc, off, col, src, st, do_a, do_b):
    want, _, cnt, _ = orc.bfs(off, col, src)
    assert st.status == 0, (src, st.status)
    L = len(cnt)
    assert st.iterations == L and st.reached == int((want >= 0).sum())
    dirs, front, _ = st.trace()
    k = min(L, 64)
    assert front[:k] == cnt[:k].tolist()
    assert dirs[:k] == orc.do_schedule(cnt, len(off) - 1, len(col), do_a, do_b)[:k].tolist()
    return want


def grid_want(r, c):
    return np.add.outer(np.arange(r), np.arange(c)).astype(np.int32).ravel()


@pytest.mark.parametrize("mode,team2,blocks", [(0, 8, 0), (0, 64, 0), (0, 64, 50), (1, 32, 0)])
def test_list_beside_grid_query(fg, orc, mode, team2, blocks):
    """The list in either mode, on every workgroup the team leaves or on a
    narrower share (grid_blocks)."""
    off, col = synth.rmat_csr(14)
    g = fg.Graph(off, col)
    goff, gcol = synth.grid_csr(300, 200)
    g2 = fg.Graph(goff, gcol)
    srcs = [int(x) for x in synth.sources(off, 12, seed=21)]
    da, db = (1, 100), (1, 10)
    opts = fg.bfs_opts(mode=mode, do_a=da, do_b=db, grid_blocks=blocks)
    opts2 = fg.bfs_opts(mode=fg.FG_MODE_PUSH, async_levels=8, team_blocks=team2)
    announce(f"bfs_corun rmat14 x{len(srcs)} mode {mode} on {blocks or 'all'} workgroups "
             f"beside grid300x200 team {team2}")
    depth, parent, sts, d2, p2, st2 = corun(fg, g, srcs, opts, True, g2, 0, opts2)
    d = to_np(depth).reshape(len(srcs), g.n)
    p = to_np(parent).reshape(len(srcs), g.n)
    for j, s in enumerate(srcs):
        if mode == 0:
            want = check_list_record(orc, off, col, s, sts[j], da, db)
        else:
            want, _, cnt, _ = orc.bfs(off, col, s)
            assert sts[j].status == 0 and sts[j].iterations == len(cnt)
            assert sts[j].trace()[0] == [0] * min(len(cnt), 64)
        assert np.array_equal(d[j], want), j
        assert orc.check_bfs(off, col, s, d[j], p[j]) is None
        assert sts[j].grid_blocks == (blocks or 256 - team2)
    assert st2.status == 0 and st2.reached == g2.n
    assert np.array_equal(to_np(d2), grid_want(300, 200))
    assert orc.check_bfs(goff, gcol, 0, to_np(d2), to_np(p2)) is None
    g.close()
    g2.close()


def test_shared_outputs_beside_a_query_that_gives_up(fg, orc):
    """The push query from the largest hub of an R-MAT graph: its first
    level does not fit a member's LDS queue, the team gives up and the
    level-synchronous launch behind the co-run answers."""
    off, col = synth.rmat_csr(13)
    g = fg.Graph(off, col)
    off2, col2 = synth.rmat_csr(16)
    g2 = fg.Graph(off2, col2)
    hub = int(np.argmax(np.diff(off2)))
    assert off2[hub + 1] - off2[hub] > 2048
    srcs = [int(x) for x in synth.sources(off, 6, seed=4)]
    opts = fg.bfs_opts(mode=0)
    opts2 = fg.bfs_opts(mode=fg.FG_MODE_PUSH, async_levels=16, team_blocks=4)
    announce("bfs_corun rmat13 x6 shared outputs beside rmat16 push from its hub")
    depth, parent, sts, d2, p2, st2 = corun(fg, g, srcs, opts, False, g2, hub, opts2)
    for j, s in enumerate(srcs):
        check_list_record(orc, off, col, s, sts[j], (1, 100), (1, 10))
    want = orc.bfs(off, col, srcs[-1])[0]
    assert np.array_equal(to_np(depth), want)
    assert orc.check_bfs(off, col, srcs[-1], want, to_np(parent)) is None
    want2 = orc.bfs(off2, col2, hub)[0]
    assert st2.status == 0
    assert np.array_equal(to_np(d2), want2)
    assert orc.check_bfs(off2, col2, hub, want2, to_np(p2)) is None
    g.close()
    g2.close()


def test_no_list_invalid_sources_and_argument_checks(fg, orc):
    off, col = synth.rmat_csr(12)
    g = fg.Graph(off, col)
    goff, gcol = synth.grid_csr(64, 50)
    g2 = fg.Graph(goff, gcol)
    opts = fg.bfs_opts(mode=0)
    opts2 = fg.bfs_opts(mode=fg.FG_MODE_PUSH, async_levels=4, team_blocks=8)
    announce("bfs_corun no list; invalid list sources")
    _, _, sts, d2, p2, st2 = corun(fg, g, [], opts, False, g2, 7, opts2)
    assert st2.status == 0
    want2 = orc.bfs(goff, gcol, 7)[0]
    assert np.array_equal(to_np(d2), want2)
    assert orc.check_bfs(goff, gcol, 7, want2, to_np(p2)) is None
    n = g.n
    srcs = [3, n, -1, int(synth.sources(off, 1, seed=2)[0])]
    depth, parent, sts, d2, p2, st2 = corun(fg, g, srcs, opts, True, g2, 7, opts2)
    d = to_np(depth).reshape(len(srcs), n)
    for j, s in enumerate(srcs):
        if 0 <= s < n:
            assert np.array_equal(d[j], check_list_record(orc, off, col, s, sts[j], (1, 100),
                                                           (1, 10)))
        else:
            assert sts[j].status == fg.FG_EINVAL and sts[j].iterations == 0
    assert np.array_equal(to_np(d2), want2)

    s = torch.zeros(2, dtype=torch.int32, device="cuda")
    depth = torch.empty(2 * n, dtype=torch.int32, device="cuda")
    depth2 = torch.empty(g2.n, dtype=torch.int32, device="cuda")
    ws = g.workspace(fg.FG_PRIM_BFS)
    ws2 = g2.workspace(fg.FG_PRIM_BFS)

    def call(**kw):
        a = dict(g=g, srcs=s, depth=depth, parent=None, opts=opts, ws=ws, stats=None, g2=g2,
                 src2=0, depth2=depth2, parent2=None, opts2=opts2, ws2=ws2)
        a.update(kw)
        with pytest.raises(fg.FGError) as e:
            fg.bfs_corun_into(**a)
        return e.value.status

    # the second query must be an asynchronous push query
    assert call(opts2=fg.bfs_opts(mode=fg.FG_MODE_PUSH, async_levels=1)) == fg.FG_EINVAL
    assert call(opts2=fg.bfs_opts(mode=0, async_levels=8)) == fg.FG_EINVAL
    assert call(src2=g2.n) == fg.FG_EINVAL
    # one workspace for both, a bad stride, the unfused mode
    big = g.workspace(fg.FG_PRIM_BFS)
    assert call(ws2=big, ws=big) == fg.FG_EINVAL
    assert call(out_stride=n - 1) == fg.FG_EINVAL
    assert call(opts=fg.bfs_opts(mode=fg.FG_MODE_PUSH_UNFUSED)) == fg.FG_EUNSUPPORTED
    g.close()
    g2.close()
