"""fg_bfs_noalloc (workspace in the library's static device array) against
fg_bfs (caller workspace): two calls in a row, the second on a smaller
graph, then the larger again; depths bit-exact, parents a valid BFS tree
(they may legally differ), stats equal.  Called through the C ABI."""
import ctypes

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


def _pair(fg, orc, g, off, col, src, opts):
    n = g.n
    d0 = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    p0 = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    d1 = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    p1 = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    s0, s1 = fg.new_stats(), fg.new_stats()
    announce(f"noalloc n={n} src={src} mode={opts.mode}")
    fg.bfs_into(g, src, d0, p0, opts, stats=s0)
    fg.bfs_noalloc_into(g, src, d1, p1, opts, stats=s1)
    a, b = fg.read_stats(s0), fg.read_stats(s1)
    assert a.status == 0 and b.status == 0
    assert (a.iterations, a.reached, a.edges_inspected) == (b.iterations, b.reached, b.edges_inspected)
    assert a.trace() == b.trace()
    want = orc.bfs(off, col, src)[0]
    assert np.array_equal(to_np(d0), want)
    assert np.array_equal(to_np(d1), to_np(d0))
    assert orc.check_bfs(off, col, src, to_np(d1), to_np(p1)) is None


def test_noalloc_matches_fg_bfs(fg, orc):
    big = synth.rmat_csr(20)
    small = synth.rmat_csr(12)
    gb = fg.Graph(*big)
    gs = fg.Graph(*small)
    assert gb.workspace_bytes(fg.FG_PRIM_BFS) <= fg.FG_NOALLOC_SCRATCH_BYTES
    for mode in (fg.FG_MODE_DO, fg.FG_MODE_PUSH):
        o = fg.bfs_opts(mode=mode)
        sb = int(synth.sources(big[0], 1)[0])
        _pair(fg, orc, gb, *big, sb, o)
        _pair(fg, orc, gs, *small, 5, o)      # second call, smaller input
        _pair(fg, orc, gb, *big, 0, o)        # and the larger again
    # team and solo modes forced (they use the scratch's queues and records)
    _pair(fg, orc, gs, *small, 0, fg.bfs_opts(mode=fg.FG_MODE_DO, team_blocks=3, small_edges=1))
    _pair(fg, orc, gs, *small, 0, fg.bfs_opts(mode=fg.FG_MODE_PUSH, team_blocks=-1,
                                              small_edges=1 << 18))


def test_noalloc_rejects(fg):
    off, col = synth.grid_csr(2048, 2048)
    g = fg.Graph(off, col)
    assert g.workspace_bytes(fg.FG_PRIM_BFS) > fg.FG_NOALLOC_SCRATCH_BYTES
    d = torch.empty(g.n, dtype=torch.int32, device="cuda")
    with pytest.raises(fg.FGError) as e:
        fg.bfs_noalloc_into(g, 0, d)
    assert e.value.status == fg.FG_ENOMEM
    off, col = synth.rmat_csr(10)
    g2 = fg.Graph(off, col)
    d2 = torch.empty(g2.n, dtype=torch.int32, device="cuda")
    with pytest.raises(fg.FGError) as e:
        fg.bfs_noalloc_into(g2, 0, d2, opts=fg.bfs_opts(mode=fg.FG_MODE_PUSH_UNFUSED))
    assert e.value.status == fg.FG_EUNSUPPORTED
    with pytest.raises(fg.FGError) as e:
        fg.bfs_noalloc_into(g2, g2.n, d2)
    assert e.value.status == fg.FG_EINVAL
