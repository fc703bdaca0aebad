"""Parity at the workloads' full sizes, in the launch configurations the
benchmark times, against the serial oracle on every query.

* R-MAT 22 direction-optimizing BFS from all 64 benchmark sources with the
  tuned thresholds the benchmark uses (and with the paper's example
  thresholds): depths bit-exact, parents a valid BFS tree, frontier sizes
  equal to the oracle's level histogram, the direction trace equal to the
  oracle's prediction from that histogram (Sec. VI-A) and the CSR entries
  read per iteration equal to the oracle's early-exit count.
* Push BFS on the 4096 x 4096 grid from the centre (the corner is covered
  by the closed-form test of test_gpu_bfs.py).
* The benchmark step as timed: the 64 R-MAT 22 sources beside the grid
  query from vertex 0 in one co-run launch, with per-source and with shared
  outputs.
* SSSP on R-MAT 22 with weights in [1, 64] from the first 16 sources:
  distances and canonical parents bit-exact against Dijkstra.
* 64-lane batched BFS on R-MAT 23 and on the 2048 x 2048 grid with the
  benchmark's sources and tuned switch points: all 64 lanes bit-exact.
* 64-lane batched SSSP on R-MAT 22 and on the 2048 x 2048 grid: all 64
  lanes bit-exact against Dijkstra.

The oracle queries run one per thread (see workloads.py), so these tests
take tens of seconds each rather than minutes.
"""
import numpy as np
import pytest
import torch

import synth
import workloads
from gpu_util import announce, gpu, need_gpu, to_np

pytestmark = [gpu, pytest.mark.slow]

U32_MAX = 0xFFFFFFFF


@pytest.fixture(scope="module")
def fg():
    need_gpu()
    import paper_1504_04804_amd as fg
    fg.lib()
    return fg


@pytest.fixture(scope="module")
def rmat22(fg):
    off, col, w = workloads.graph("rmat22")
    g = fg.Graph(off, col, weights=w, symmetric=True, validate=False)
    yield off, col, w, g
    g.close()


def _bfs_oracle_checks(orc, off, col, src, d, p, dirs, front, insp, iters, do_a, do_b, mode):
    """Everything the oracle fixes for one traversal; returns an error
    string or None (runs in a worker thread)."""
    want, _, cnt, _ = orc.bfs(off, col, src)
    if not np.array_equal(d, want):
        return f"src {src}: depth mismatch at {np.flatnonzero(d != want)[:8]}"
    err = orc.check_bfs(off, col, src, d, p)
    if err is not None:
        return f"src {src}: {err}"
    L = len(cnt)
    if iters != L:
        return f"src {src}: {iters} iterations, oracle {L}"
    k = min(L, 64)
    if front[:k] != cnt[:k].tolist():
        return f"src {src}: frontier sizes {front[:k]} != {cnt[:k].tolist()}"
    if mode == "do":
        want_dirs = orc.do_schedule(cnt, len(off) - 1, len(col), do_a, do_b)
    else:
        want_dirs = np.zeros(L, np.int8)
    if dirs[:k] != want_dirs[:k].tolist():
        return f"src {src}: directions {dirs[:k]} != {want_dirs[:k].tolist()}"
    want_insp = orc.edges_inspected(off, col, want, want_dirs)
    if insp[:k] != want_insp[:k].tolist():
        return f"src {src}: entries read {insp[:k]} != {want_insp[:k].tolist()}"
    return None


def _run_bfs_sources(fg, orc, g, off, col, srcs, opts, do_a, do_b, mode):
    depth = torch.empty(g.n, dtype=torch.int32, device="cuda")
    parent = torch.empty(g.n, dtype=torch.int32, device="cuda")
    stats = fg.new_stats()
    ws = g.workspace(fg.FG_PRIM_BFS)
    futs = []
    with workloads.pool() as ex:
        for s in srcs:
            announce(f"config bfs n={g.n} src={s} mode={mode} do_a={do_a} do_b={do_b}")
            fg.bfs_into(g, int(s), depth, parent, opts, ws=ws, stats=stats)
            st = fg.read_stats(stats)
            assert st.status == 0, (s, st.status)
            dirs, front, insp = st.trace()
            futs.append(ex.submit(_bfs_oracle_checks, orc, off, col, int(s), to_np(depth),
                                  to_np(parent), dirs, front, insp, st.iterations, do_a, do_b,
                                  mode))
        errs = [f.result() for f in futs]
    bad = [e for e in errs if e is not None]
    assert not bad, bad[:4]


def test_c2_rmat22_dobfs_all_sources_tuned(fg, orc, rmat22):
    """All 64 sources with the thresholds the benchmark times."""
    from paper_1504_04804_amd import autotune
    off, col, _, g = rmat22
    opts, kw = autotune.workload_opts("rmat22_dobfs", g)
    srcs = synth.sources(off, 64)
    assert len(srcs) == 64
    _run_bfs_sources(fg, orc, g, off, col, srcs, opts, kw["do_a"], kw["do_b"], "do")


def test_c2_rmat22_dobfs_paper_thresholds(fg, orc, rmat22):
    """The paper's example thresholds (do_a = 1/100, do_b = 1/10) on 16 sources."""
    off, col, _, g = rmat22
    opts = fg.bfs_opts(mode=fg.FG_MODE_DO, do_a=(1, 100), do_b=(1, 10))
    _run_bfs_sources(fg, orc, g, off, col, synth.sources(off, 64)[:16], opts, (1, 100),
                     (1, 10), "do")


def test_c2_rmat22_push_sources(fg, orc, rmat22):
    """Push-only BFS (fused advance + filter every level) from 8 sources."""
    off, col, _, g = rmat22
    opts = fg.bfs_opts(mode=fg.FG_MODE_PUSH)
    _run_bfs_sources(fg, orc, g, off, col, synth.sources(off, 64)[:8], opts, None, None, "push")


def test_c2_grid4096_push_centre_tuned(fg, orc):
    from paper_1504_04804_amd import autotune
    off, col, _ = workloads.graph("grid4096")
    g = fg.Graph(off, col, symmetric=True, validate=False)
    opts, _ = autotune.workload_opts("grid4096_push", g)
    R = 4096
    for src in (0, (R // 2) * R + R // 2, R * R - 1):
        announce(f"grid4096 push src={src}")
        depth, parent, st = fg.bfs(g, src, opts=opts)
        d = to_np(depth)
        r0, c0 = divmod(src, R)
        rr = np.abs(np.arange(R, dtype=np.int32) - r0)
        cc = np.abs(np.arange(R, dtype=np.int32) - c0)
        assert np.array_equal(d.reshape(R, R), rr[:, None] + cc[None, :])
        assert st.status == 0 and st.iterations == int(d.max()) + 1
        assert orc.check_bfs(off, col, src, d, to_np(parent)) is None
    g.close()


def test_c2_step_corun_as_benchmarked(fg, orc, rmat22):
    """The benchmark step itself: fg_bfs_corun with the 64 sources and the
    grid query from vertex 0, the tuned options of both.  Per-source outputs:
    every traversal's depths, parents and record against the oracle; shared
    outputs (the benchmark's launch): the last source's outputs; the grid's
    depths in closed form with a valid parent tree both times."""
    from paper_1504_04804_amd import autotune
    off, col, _, g = rmat22
    opts, kw = autotune.workload_opts("rmat22_dobfs_corun", g)
    goff, gcol, _ = workloads.graph("grid4096")
    gg = fg.Graph(goff, gcol, symmetric=True, validate=False)
    gopts, _ = autotune.workload_opts("grid4096_push", gg)
    R = 4096
    want_grid = (np.arange(R, dtype=np.int32)[:, None] + np.arange(R, dtype=np.int32)[None, :])
    srcs = [int(x) for x in synth.sources(off, 64)]
    n = g.n
    srcs_dev = torch.tensor(srcs, dtype=torch.int32, device="cuda")
    stats = fg.new_stats_many(64)
    gdepth = torch.empty(gg.n, dtype=torch.int32, device="cuda")
    gparent = torch.empty(gg.n, dtype=torch.int32, device="cuda")
    gst = fg.new_stats()
    for stride in (n, 0):
        rows = 64 if stride else 1
        depth = torch.full((rows * n,), -7, dtype=torch.int32, device="cuda")
        parent = torch.full((rows * n,), -7, dtype=torch.int32, device="cuda")
        announce(f"config step co-run rmat22 x64 beside grid4096, out_stride={stride}")
        fg.bfs_corun_into(g, srcs_dev, depth, parent, opts, None, stats, gg, 0, gdepth,
                          gparent, gopts, stats2=gst, out_stride=stride)
        torch.cuda.synchronize()
        sts = fg.read_stats_many(stats, 64)
        assert all(st.status == 0 for st in sts), [st.status for st in sts]
        sg = fg.read_stats(gst)
        assert sg.status == 0 and sg.iterations == 2 * R - 1
        d2 = to_np(gdepth)
        assert np.array_equal(d2.reshape(R, R), want_grid)
        assert orc.check_bfs(goff, gcol, 0, d2, to_np(gparent)) is None
        d = to_np(depth).reshape(rows, n)
        p = to_np(parent).reshape(rows, n)
        if stride:
            with workloads.pool() as ex:
                futs = []
                for j, s in enumerate(srcs):
                    dirs, front, insp = sts[j].trace()
                    futs.append(ex.submit(_bfs_oracle_checks, orc, off, col, s, d[j], p[j], dirs,
                                          front, insp, sts[j].iterations, kw["do_a"], kw["do_b"],
                                          "do"))
                bad = [e for e in (f.result() for f in futs) if e is not None]
            assert not bad, bad[:4]
        else:
            assert _bfs_oracle_checks(orc, off, col, srcs[-1], d[0], p[0], *sts[-1].trace(),
                                      sts[-1].iterations, kw["do_a"], kw["do_b"], "do") is None
        del depth, parent
    gg.close()


def test_c3a_sssp_rmat22_16_sources(fg, orc, rmat22):
    off, col, w, g = rmat22
    dist = torch.empty(g.n, dtype=torch.int32, device="cuda")
    par = torch.empty(g.n, dtype=torch.int32, device="cuda")
    ws = g.workspace(fg.FG_PRIM_SSSP)
    st = fg.new_stats()

    def check(src, d, p):
        want, wpar = orc.dijkstra(off, col, w, src)
        if not np.array_equal(d, want):
            return f"src {src}: dist mismatch at {np.flatnonzero(d != want)[:8]}"
        if not np.array_equal(p, wpar):
            return f"src {src}: parent mismatch at {np.flatnonzero(p != wpar)[:8]}"
        return None

    futs = []
    with workloads.pool() as ex:
        for s in synth.sources(off, 64)[:16]:
            announce(f"config sssp rmat22 src={s}")
            fg.sssp_into(g, int(s), dist, par, ws=ws, stats=st)
            r = fg.read_stats(st)
            assert r.status == 0, (s, r.status)
            futs.append(ex.submit(check, int(s), to_np(dist).view(np.uint32).copy(), to_np(par)))
        bad = [e for e in (f.result() for f in futs) if e is not None]
    assert not bad, bad[:4]


def _check_lanes_parallel(orc, reads, off, col, w=None):
    """reads: list of (lane, src, host result); BFS depths when w is None,
    else distances against Dijkstra."""
    def check(lane, src, got):
        if w is None:
            want = orc.bfs(off, col, src)[0]
        else:
            want = orc.dijkstra(off, col, w, src)[0]
            got = got.view(np.uint32)
        if not np.array_equal(got, want):
            return f"lane {lane} src {src}: mismatch at {np.flatnonzero(got != want)[:8]}"
        return None

    with workloads.pool() as ex:
        bad = [e for e in ex.map(lambda t: check(*t), reads) if e is not None]
    assert not bad, bad[:4]


@pytest.mark.parametrize("name", ["rmat23", "grid2048"])
def test_c4_msbfs_all_64_lanes(fg, orc, name):
    """The benchmark's 64-lane batches with its sources and tuned switch points."""
    from paper_1504_04804_amd import autotune
    off, col, _ = workloads.graph(name)
    g = fg.Graph(off, col, symmetric=True, validate=False)
    opts, _ = autotune.workload_opts(f"{name}_msbfs", g)
    srcs = [int(s) for s in synth.sources(off, 64)]
    announce(f"config msbfs {name} 64 lanes")
    b = fg.MsBatch(g, 64, opts)
    for lane, s in enumerate(srcs):
        b.admit(lane, s)
    b.step(1 << 30)
    done, _ = b.poll()
    assert done == (1 << 64) - 1
    reads = [(lane, s, to_np(b.read(lane))) for lane, s in enumerate(srcs)]
    b.close()
    g.close()
    _check_lanes_parallel(orc, reads, off, col)
    if name == "rmat23":
        workloads.drop(name)


@pytest.mark.parametrize("name", ["rmat22", "grid2048"])
def test_batched_sssp_all_64_lanes(fg, orc, name):
    """The benchmark's 64-lane SSSP batches (sources of seed 31)."""
    off, col, w = workloads.graph(name)
    g = fg.Graph(off, col, weights=w, symmetric=True, validate=False)
    srcs = [int(s) for s in synth.sources(off, 64, seed=31)]
    announce(f"config mssp {name} 64 lanes")
    b = fg.MsspBatch(g, 64)
    for lane, s in enumerate(srcs):
        b.admit(lane, s)
    b.step(1 << 30)
    done, _ = b.poll()
    assert done == (1 << 64) - 1
    reads = [(lane, s, to_np(b.read(lane))) for lane, s in enumerate(srcs)]
    b.close()
    g.close()
    _check_lanes_parallel(orc, reads, off, col, w)
