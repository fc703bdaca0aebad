"""The autotuner: a reduced sweep on a small graph returns options that give
the oracle's depths, the JSON caches round-trip, and the committed
workload cache holds an entry for every timed workload."""
import json
import os

import numpy as np
import pytest
import torch

import synth
from gpu_util import announce, gpu, need_gpu, to_np

pytestmark = gpu


@pytest.fixture(scope="module")
def env():
    need_gpu()
    import paper_1504_04804_amd as fg
    from paper_1504_04804_amd import autotune
    fg.lib()
    return fg, autotune


def test_tune_bfs_small(env, orc, tmp_path):
    fg, at = env
    off, col = synth.rmat_csr(14)
    g = fg.Graph(off, col)
    srcs = [int(s) for s in synth.sources(off, 4, seed=5)]
    announce("autotune bfs rmat14")
    path = str(tmp_path / "cache.json")
    opts, kw = at.tuned_bfs_opts(g, srcs, path, log=print, do_a=[(1, 100), (1, 10000)],
                                 do_b=[(1, 10), (1, 1)], big_deg=[64], team=[-1, 16])
    assert kw["mode"] == fg.FG_MODE_DO
    assert kw["do_a"] in [(1, 100), (1, 10000)] and kw["do_b"] in [(1, 10), (1, 1)]
    # the cache round-trips: a second call reads the same options, no tuning
    with open(path) as f:
        cached = json.load(f)
    assert len(cached) == 1
    opts2, kw2 = at.tuned_bfs_opts(g, srcs, path, log=None, do_a=[(1, 2)])
    assert kw2 == kw
    for s in srcs:
        d, p, st = fg.bfs(g, s, opts=opts2)
        want = orc.bfs(off, col, s)[0]
        assert st.status == 0
        assert np.array_equal(to_np(d), want)
        assert orc.check_bfs(off, col, s, to_np(d), to_np(p)) is None


def test_tune_push_async_small(env, orc):
    """Push tuning includes the asynchronous team; the winner's options give
    the oracle's depths (Manhattan distances on a grid)."""
    fg, at = env
    off, col = synth.grid_csr(300, 200)
    g = fg.Graph(off, col)
    announce("autotune push grid300x200")
    kw, ms = at.tune_bfs(g, [0], fg.FG_MODE_PUSH, print, big_deg=[32], team=[16],
                         async_levels=[8, 32], async_team=[8, 16])
    assert kw["mode"] == fg.FG_MODE_PUSH and ms > 0
    d, p, st = fg.bfs(g, 0, opts=fg.bfs_opts(**kw))
    assert st.status == 0
    assert to_np(d).tolist() == [r + c for r in range(300) for c in range(200)]
    assert orc.check_bfs(off, col, 0, to_np(d), to_np(p)) is None
    g.close()


def test_tune_corun_small(env, orc):
    """The list's share of the workgroups beside an asynchronous query: the
    winner is one of the candidates, and a co-run with it gives the
    oracle's depths for every list source and the grid's closed form."""
    fg, at = env
    off, col = synth.rmat_csr(14)
    g = fg.Graph(off, col)
    goff, gcol = synth.grid_csr(300, 200)
    g2 = fg.Graph(goff, gcol)
    srcs = [int(s) for s in synth.sources(off, 8, seed=12)]
    opts2 = fg.bfs_opts(mode=fg.FG_MODE_PUSH, async_levels=8, team_blocks=16)
    announce("autotune corun rmat14 x8 beside grid300x200")
    kw, ms = at.tune_corun(g, srcs, dict(mode=fg.FG_MODE_DO), g2, 0, opts2, print,
                           widths=[0, 96, 24])
    assert kw["grid_blocks"] in (0, 96, 24) and ms > 0
    n = g.n
    depth = torch.empty(len(srcs) * n, dtype=torch.int32, device="cuda")
    parent = torch.empty(len(srcs) * n, dtype=torch.int32, device="cuda")
    d2 = torch.empty(g2.n, dtype=torch.int32, device="cuda")
    stats = fg.new_stats_many(len(srcs))
    fg.bfs_corun_into(g, torch.tensor(srcs, dtype=torch.int32, device="cuda"), depth, parent,
                      fg.bfs_opts(**kw), None, stats, g2, 0, d2, None, opts2, out_stride=n)
    torch.cuda.synchronize()
    d = to_np(depth).reshape(len(srcs), n)
    p = to_np(parent).reshape(len(srcs), n)
    for j, s in enumerate(srcs):
        assert np.array_equal(d[j], orc.bfs(off, col, s)[0])
        assert orc.check_bfs(off, col, s, d[j], p[j]) is None
    sts = fg.read_stats_many(stats, len(srcs))
    if kw["grid_blocks"]:
        assert all(st.grid_blocks == kw["grid_blocks"] for st in sts)
    assert to_np(d2).tolist() == [r + c for r in range(300) for c in range(200)]
    g.close()
    g2.close()


def test_tune_msbfs_small(env, orc):
    fg, at = env
    off, col = synth.rmat_csr(13)
    g = fg.Graph(off, col)
    srcs = [int(s) for s in synth.sources(off, 16, seed=6)]
    announce("autotune msbfs rmat13")
    kw, ms = at.tune_msbfs(g, srcs, pull_div=[8, 64], push_div=[64, 512], reps=1)
    assert ms > 0 and kw["pull_div"] in (8, 64) and kw["push_div"] in (64, 512)
    b = fg.MsBatch(g, 16, fg.msbfs_opts(**kw))
    for lane, s in enumerate(srcs):
        b.admit(lane, s)
    b.run(k_iters=8)
    for lane, s in enumerate(srcs):
        assert np.array_equal(to_np(b.read(lane)), orc.bfs(off, col, s)[0])


def test_workload_cache_entries(env):
    """Every workload the benchmark times has an entry, looked up by name
    and checked against the graph it was tuned on."""
    fg, at = env
    cache = at.load(at.TUNED_PATH)
    for name in ("rmat22_dobfs", "grid4096_push", "rmat23_msbfs", "grid2048_msbfs",
                 "rmat23_dobfs", "grid2048_push", "rmat22_dobfs_corun"):
        assert name in cache, name
        ent = cache[name]
        assert ent["kind"] in ("bfs", "msbfs") and "signature" in ent and "kwargs" in ent
    off, col = synth.grid_csr(2048, 2048)
    g = fg.Graph(off, col)
    opts, kw = at.workload_opts("grid2048_msbfs", g)
    assert isinstance(opts, fg.MsOpts) and set(kw) == {"pull_div", "push_div"}
    with pytest.raises(ValueError):
        at.workload_opts("rmat23_msbfs", g)  # tuned on another graph
    with pytest.raises(KeyError):
        at.workload_opts("no_such_workload", g)
