"""fg_bfs_many (several sources one after another in one launch) against
the oracle, through the C ABI: every traversal's depths bit-exact (with a
per-source output stride), parents a valid BFS tree, and each record's
level sizes, direction trace and entries read equal to the oracle's for
that source; invalid sources skipped with FG_EINVAL in their record; team
and single-workgroup episodes across traversal boundaries; the R-MAT 22
workload's 64 sources with its tuned options."""
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


def check_record(orc, off, col, src, st, opts_mode, do_a, do_b):
    want, _, cnt, _ = orc.bfs(off, col, src)
    assert st.status == 0, (src, st.status)
    L = len(cnt)
    assert st.iterations == L, (src, st.iterations, L)
    assert st.reached == int((want >= 0).sum())
    dirs, front, insp = st.trace()
    k = min(L, 64)
    assert front[:k] == cnt[:k].tolist()
    if opts_mode == 0:
        sched = orc.do_schedule(cnt, len(off) - 1, len(col), do_a, do_b)
    else:
        sched = np.zeros(L, np.int8)
    assert dirs[:k] == sched[:k].tolist()
    assert insp[:k] == orc.edges_inspected(off, col, want, sched)[:k].tolist()
    return want


def run_many(fg, g, srcs, opts, stride, parents=True):
    n = g.n
    rows = len(srcs) if stride else 1
    depth = torch.full((rows * n,), -7, dtype=torch.int32, device="cuda")
    parent = torch.full((rows * n,), -7, dtype=torch.int32, device="cuda") if parents else None
    stats = fg.new_stats_many(len(srcs))
    s = torch.tensor(srcs, dtype=torch.int32, device="cuda")
    fg.bfs_many_into(g, s, depth, parent, opts, stats=stats, out_stride=n if stride else 0)
    torch.cuda.synchronize()
    return depth, parent, fg.read_stats_many(stats, len(srcs))


@pytest.mark.parametrize("mode", [0, 1])
def test_many_retained_outputs(fg, orc, mode):
    off, col = synth.rmat_csr(14)
    g = fg.Graph(off, col)
    srcs = [0] + [int(x) for x in synth.sources(off, 11, seed=3)]
    da, db = (1, 100), (1, 10)
    opts = fg.bfs_opts(mode=mode, do_a=da, do_b=db)
    announce(f"bfs_many rmat14 mode={mode} {len(srcs)} sources, stride n")
    depth, parent, sts = run_many(fg, g, srcs, opts, stride=True)
    d = to_np(depth).reshape(len(srcs), g.n)
    p = to_np(parent).reshape(len(srcs), g.n)
    for j, s in enumerate(srcs):
        want = check_record(orc, off, col, s, sts[j], mode, da, db)
        assert np.array_equal(d[j], want), j
        assert orc.check_bfs(off, col, s, d[j], p[j]) is None
    g.close()


def test_many_shared_outputs_and_invalid_sources(fg, orc):
    off, col = synth.rmat_csr(13)
    g = fg.Graph(off, col)
    n = g.n
    srcs = [5, n, 17, -3, int(synth.sources(off, 1, seed=8)[0])]
    opts = fg.bfs_opts(mode=0)
    announce("bfs_many rmat13 shared outputs with invalid sources")
    depth, parent, sts = run_many(fg, g, srcs, opts, stride=False)
    for j, s in enumerate(srcs):
        if 0 <= s < n:
            check_record(orc, off, col, s, sts[j], 0, (1, 100), (1, 10))
        else:
            assert sts[j].status == fg.FG_EINVAL and sts[j].iterations == 0
    want = orc.bfs(off, col, srcs[-1])[0]
    assert np.array_equal(to_np(depth), want)
    assert orc.check_bfs(off, col, srcs[-1], want, to_np(parent)) is None
    # no sources: nothing happens; a bad stride is refused
    fg.bfs_many_into(g, torch.zeros(0, dtype=torch.int32, device="cuda"), depth)
    with pytest.raises(fg.FGError) as e:
        fg.bfs_many_into(g, torch.zeros(2, dtype=torch.int32, device="cuda"), depth,
                         out_stride=n - 1)
    assert e.value.status == fg.FG_EINVAL
    with pytest.raises(fg.FGError) as e:
        fg.bfs_many_into(g, torch.zeros(2, dtype=torch.int32, device="cuda"), depth,
                         opts=fg.bfs_opts(mode=fg.FG_MODE_PUSH_UNFUSED))
    assert e.value.status == fg.FG_EUNSUPPORTED
    g.close()


def test_many_shared_outputs_reset_between_components(fg, orc):
    """Shared outputs: a traversal after one that reached other vertices
    leaves exactly its own reach set non-negative (the vertices only the
    previous traversal reached go back to -1), whatever came before it,
    invalid sources and a first source that reaches little included."""
    # an R-MAT graph plus a disjoint grid and an isolated vertex
    ro, rc = synth.rmat_csr(12)
    go, gc = synth.grid_csr(30, 40)
    nr, ng = len(ro) - 1, len(go) - 1
    off = np.concatenate([ro, go[1:] + ro[-1], [ro[-1] + go[-1]]]).astype(np.int32)
    col = np.concatenate([rc, gc + nr]).astype(np.int32)
    n = nr + ng + 1
    g = fg.Graph(off, col)
    a = int(synth.sources(ro, 1, seed=5)[0])
    b = nr + 617
    iso = n - 1
    cases = ([a, b], [b, a], [a, b, a], [b, iso], [iso, a, b], [-1, b, a], [a, n, b],
             [b, a, b, a, iso, b])
    for mode in (0, 1):
        opts = fg.bfs_opts(mode=mode)
        for srcs in cases:
            announce(f"bfs_many shared outputs mode={mode} sources {srcs}")
            depth, parent, sts = run_many(fg, g, srcs, opts, stride=False)
            last = [s for s in srcs if 0 <= s < n][-1]
            want = orc.bfs(off, col, last)[0]
            assert np.array_equal(to_np(depth), want), (mode, srcs)
            assert orc.check_bfs(off, col, last, want, to_np(parent)) is None
            for j, s in enumerate(srcs):
                if 0 <= s < n:
                    assert sts[j].status == 0 and sts[j].reached == int((orc.bfs(off, col, s)[0] >= 0).sum())
    g.close()


def test_many_episodes_across_traversals(fg, orc):
    """Team and single-workgroup episodes forced, on a grid (long, thin
    frontiers) and R-MAT: the hand-off state is reset between traversals."""
    for off, col, mode in ((*synth.grid_csr(64, 70), 1), (*synth.rmat_csr(12), 0)):
        g = fg.Graph(off, col)
        srcs = [0, 17, int(g.n) - 1, 1000, 0]
        for kw in (dict(team_blocks=3, small_edges=1), dict(team_blocks=-1, small_edges=1 << 18),
                   dict(team_blocks=7)):
            opts = fg.bfs_opts(mode=mode, **kw)
            announce(f"bfs_many episodes n={g.n} mode={mode} {kw}")
            depth, parent, sts = run_many(fg, g, srcs, opts, stride=True)
            d = to_np(depth).reshape(len(srcs), g.n)
            p = to_np(parent).reshape(len(srcs), g.n)
            for j, s in enumerate(srcs):
                want = check_record(orc, off, col, s, sts[j], mode, (1, 100), (1, 10))
                assert np.array_equal(d[j], want), (kw, j)
                assert orc.check_bfs(off, col, s, d[j], p[j]) is None
        g.close()


@pytest.mark.slow
def test_many_rmat22_benchmark_sources(fg, orc):
    """The 64 R-MAT 22 sources of the DOBFS workload with its tuned options
    in one launch: every record equals the oracle's level sizes, directions
    and entries read; the first 8 with retained outputs, bit-exact."""
    from paper_1504_04804_amd import autotune
    off, col, _ = workloads.graph("rmat22")
    g = fg.Graph(off, col, symmetric=True, validate=False)
    opts, kw = autotune.workload_opts("rmat22_dobfs", g)
    srcs = [int(s) for s in synth.sources(off, 64)]
    announce("bfs_many rmat22 64 sources shared outputs")
    depth, parent, sts = run_many(fg, g, srcs, opts, stride=False, parents=True)
    last_d, last_p = to_np(depth), to_np(parent)

    def rec(j):
        check_record(orc, off, col, srcs[j], sts[j], 0, kw["do_a"], kw["do_b"])
        return None

    with workloads.pool() as ex:
        list(ex.map(rec, range(64)))
    want = orc.bfs(off, col, srcs[-1])[0]
    assert np.array_equal(last_d, want)
    assert orc.check_bfs(off, col, srcs[-1], want, last_p) is None
    announce("bfs_many rmat22 8 sources retained outputs")
    depth, parent, sts = run_many(fg, g, srcs[:8], opts, stride=True)
    d = to_np(depth).reshape(8, g.n)
    p = to_np(parent).reshape(8, g.n)

    def full(j):
        w = orc.bfs(off, col, srcs[j])[0]
        assert np.array_equal(d[j], w), j
        assert orc.check_bfs(off, col, srcs[j], d[j], p[j]) is None

    with workloads.pool() as ex:
        list(ex.map(full, range(8)))
    g.close()


@pytest.mark.parametrize("blocks", [1, 37, 100])
def test_many_narrowed_launch(fg, orc, blocks):
    """grid_blocks narrows the persistent launch (a team wider than it is
    narrowed too): every traversal's outputs and record as on the full
    device, and the record names the width."""
    off, col = synth.rmat_csr(13)
    g = fg.Graph(off, col)
    srcs = [int(x) for x in synth.sources(off, 6, seed=14)]
    for mode in (0, 1):
        opts = fg.bfs_opts(mode=mode, grid_blocks=blocks)
        announce(f"bfs_many rmat13 grid_blocks={blocks} mode={mode}")
        depth, parent, sts = run_many(fg, g, srcs, opts, stride=True)
        d = to_np(depth).reshape(len(srcs), g.n)
        p = to_np(parent).reshape(len(srcs), g.n)
        for j, s in enumerate(srcs):
            want = check_record(orc, off, col, s, sts[j], mode, (1, 100), (1, 10))
            assert np.array_equal(d[j], want), (mode, j)
            assert orc.check_bfs(off, col, s, d[j], p[j]) is None
            assert sts[j].grid_blocks == blocks
        dd, pp, st = fg.bfs(g, srcs[0], opts=opts)
        assert st.status == 0 and st.grid_blocks == blocks
        assert np.array_equal(to_np(dd), orc.bfs(off, col, srcs[0])[0])
    g.close()
