"""Duplicate-all + broadcast direction-optimizing BFS (fg_dup_*, Alg. 2 with
the duplicate-all vertex model and broadcast of Sec. III-C) emulated with
1-4 partitions on one GPU, through the C ABI, against the oracle:

* depths of every partition equal the FIFO BFS (O2) and the serial
  duplicate-all emulation (O11), bit-exact;
* the direction trace equals O11's and the single-graph prediction from the
  level sizes (O3); frontier sizes equal the level histogram;
* the CSR entries the partitions read per iteration add up to the oracle's
  early-exit count (O4);
* the shared parent array is a valid BFS tree (O7);
* the hand-worked fixture of tests/golden/dobfs_dupall.json.
"""
import json
import os

import numpy as np
import pytest
import torch

import synth
import workloads
from gpu_util import announce, gpu, need_gpu, to_np

pytestmark = gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
THRESH = [((1, 100), (1, 10)), ((1, 100000), (1, 1)), ((0, 1), (1, 1)), ((1 << 30, 1), (1, 1)),
          ((1, 2), (1, 1000))]


@pytest.fixture(scope="module")
def fg():
    need_gpu()
    import paper_1504_04804_amd as fg
    fg.lib()
    return fg


def check_run(fg, orc, off, col, owner, nparts, src, da, db, dup=None, rounds=False):
    n = len(off) - 1
    announce(f"dupall n={n} m={len(col)} nparts={nparts} src={src} do_a={da} do_b={db} "
             f"rounds={rounds}")
    own = dup is None
    if own:
        dup = fg.DupBfs(off, col, owner, nparts, do_a=da, do_b=db)
    if rounds:
        dup.seed(src)
        done = False
        for _ in range(n + 2):
            dup.round()
            done, it = dup.poll()
            if done:
                break
        assert done
    else:
        dup.run(src)
    want, _, cnt, _ = orc.bfs(off, col, src)
    odepth, odirs, oit = orc.dobfs_dupall(off, col, owner, nparts, src, da, db)
    assert np.array_equal(odepth, want)
    for p in range(nparts):
        got = to_np(dup.depth[p])
        assert np.array_equal(got, want), (p, np.flatnonzero(got != want)[:8])
    assert orc.check_bfs(off, col, src, want, to_np(dup.parent)) is None
    L = len(cnt)
    k = min(L, 64)
    sts = [dup.read_stats(p) for p in range(nparts)]
    for st in sts:
        assert st.status == 0 and st.iterations == L == oit
        assert st.reached == int((want >= 0).sum())
        dirs, front, _ = st.trace()
        assert dirs[:k] == odirs[:k].tolist()
        assert front[:k] == cnt[:k].tolist()
    sched = orc.do_schedule(cnt, n, len(col), da, db)
    assert odirs.tolist() == sched.tolist()
    insp = np.sum([np.array(st.trace()[2][:k], np.int64) for st in sts], axis=0)
    assert insp.tolist() == orc.edges_inspected(off, col, want, sched)[:k].tolist()
    if own:
        dup.close()


def test_golden_fixture(fg, orc):
    with open(os.path.join(GOLDEN, "dobfs_dupall.json")) as f:
        g = json.load(f)
    a = np.asarray(g["edges"], np.int32)
    off, col = orc.csr_from_edges(g["n"], a[:, 0], a[:, 1])
    dup = fg.DupBfs(off, col, g["owner"], g["nparts"], do_a=tuple(g["do_a"]),
                    do_b=tuple(g["do_b"]))
    dup.run(g["src"])
    for p in range(g["nparts"]):
        assert to_np(dup.depth[p]).tolist() == g["depth"]
        dirs, _, _ = dup.read_stats(p).trace()
        assert dirs == g["dirs"]
        assert dup.read_stats(p).iterations == g["iterations"]
    dup.close()


@pytest.mark.parametrize("nparts", [1, 2, 3, 4])
def test_small_graphs_all_thresholds(fg, orc, nparts):
    cases = [synth.rmat_csr(10), synth.rmat_csr(12), synth.grid_csr(9, 13)]
    for ci, (off, col) in enumerate(cases):
        owner = synth.owners(len(off) - 1, nparts, seed=ci + 7)
        for da, db in THRESH:
            dup = fg.DupBfs(off, col, owner, nparts, do_a=da, do_b=db)
            for src in [0] + [int(s) for s in synth.sources(off, 3, seed=ci)]:
                check_run(fg, orc, off, col, owner, nparts, src, da, db, dup=dup)
            dup.close()


def test_closed_forms_and_degenerate(fg, orc):
    # path with alternating owners: depth |i - s|
    n = 70
    a = np.array([(i, i + 1) for i in range(n - 1)], np.int32)
    off, col = orc.csr_from_edges(n, a[:, 0], a[:, 1])
    owner = np.arange(n) % 3
    for s in (0, 33, 69):
        for da, db in THRESH[:3]:
            check_run(fg, orc, off, col, owner, 3, s, da, db)
    # disconnected vertices stay -1; an isolated source reaches only itself;
    # a source hosted by a partition where it has no edges
    a = np.array([(0, 1), (1, 2), (5, 6)], np.int32)
    off, col = orc.csr_from_edges(9, a[:, 0], a[:, 1])
    owner = np.array([1, 0, 1, 0, 1, 0, 1, 0, 1])
    for s in (2, 3, 5, 8):
        check_run(fg, orc, off, col, owner, 2, s, (0, 1), (1, 1))
        check_run(fg, orc, off, col, owner, 2, s, (1, 100), (1, 10))
    # every vertex on one partition, the others host nothing
    off, col = synth.rmat_csr(9)
    check_run(fg, orc, off, col, np.zeros(len(off) - 1, np.uint8), 4, 0, (1, 100), (1, 10))


def test_round_by_round_calls_equal_run(fg, orc):
    """The per-iteration calls (seed, step, send, combine, poll) driven from
    Python give what fg_dup_run gives."""
    off, col = synth.rmat_csr(13)
    owner = synth.owners(len(off) - 1, 4, seed=5)
    for src in [int(s) for s in synth.sources(off, 2, seed=9)]:
        check_run(fg, orc, off, col, owner, 4, src, (1, 100), (1, 10), rounds=True)
        check_run(fg, orc, off, col, owner, 4, src, (1, 100000), (1, 1), rounds=True)


def test_long_rows_forward(fg, orc):
    """Forward steps over rows past the chunked-pass cut (R-MAT 18 hubs,
    thousands of entries) with push-only and paper thresholds."""
    off, col = synth.rmat_csr(18)
    assert int(np.diff(off).max()) >= 4096
    owner = synth.owners(len(off) - 1, 4)
    for da, db in (((1 << 30, 1), (1, 1)), ((1, 100), (1, 10))):
        dup = fg.DupBfs(off, col, owner, 4, do_a=da, do_b=db)
        for src in [0] + [int(s) for s in synth.sources(off, 2, seed=4)]:
            check_run(fg, orc, off, col, owner, 4, src, da, db, dup=dup)
        dup.close()


@pytest.mark.slow
def test_config_rmat22_four_partitions(fg, orc):
    """R-MAT 22 over four random owners, 16 of the 64 benchmark sources, with
    the benchmark's thresholds and the paper's example thresholds: depths of
    every partition bit-exact (oracle queries one per thread)."""
    off, col, _ = workloads.graph("rmat22")
    owner = synth.owners(len(off) - 1, 4)
    srcs = [int(s) for s in synth.sources(off, 64)[:16]]
    for da, db in (((1, 100000), (1, 1)), ((1, 100), (1, 10))):
        dup = fg.DupBfs(off, col, owner, 4, do_a=da, do_b=db)
        futs = []
        with workloads.pool() as ex:
            for s in srcs:
                announce(f"dupall rmat22 src={s} do_a={da} do_b={db}")
                dup.run(s)
                got = [to_np(d) for d in dup.depth]
                par = to_np(dup.parent)
                sts = [dup.read_stats(p) for p in range(4)]
                assert all(st.status == 0 for st in sts)

                def check(s_=s, got_=got, par_=par, sts_=sts):
                    want, _, cnt, _ = orc.bfs(off, col, s_)
                    for p, g_ in enumerate(got_):
                        if not np.array_equal(g_, want):
                            return f"src {s_} part {p}: depth mismatch"
                    err = orc.check_bfs(off, col, s_, want, par_)
                    if err:
                        return f"src {s_}: {err}"
                    sched = orc.do_schedule(cnt, len(off) - 1, len(col), da, db)
                    k = min(len(cnt), 64)
                    if sts_[0].trace()[0][:k] != sched[:k].tolist():
                        return f"src {s_}: direction trace"
                    return None

                futs.append(ex.submit(check))
            bad = [e for e in (f.result() for f in futs) if e]
        assert not bad, bad[:4]
        dup.close()
