"""Parity of the 64-lane batched SSSP: every lane's distances equal the
oracle's Dijkstra from that lane's source (bit-exact), alone or in the mix,
including lanes admitted mid-flight, lanes reused after release and a live
lane replaced by a new query."""
import numpy as np
import pytest

import synth
from gpu_util import announce, gpu, need_gpu, to_np

pytestmark = gpu

U32_MAX = 0xFFFFFFFF


@pytest.fixture(scope="module")
def fg():
    need_gpu()
    import paper_1504_04804_amd as fg
    fg.lib()
    return fg


def check_lanes(orc, b, off, col, w, srcs):
    for lane, s in srcs.items():
        got = to_np(b.read(lane)).astype(np.uint32)
        want = orc.dijkstra(off, col, w, int(s))[0]
        assert np.array_equal(got, want), \
            f"lane {lane} src {s}: {np.flatnonzero(got != want)[:8]}"


def run_batch(fg, g, srcs, opts=None, lanes=64, k_iters=16):
    b = fg.MsspBatch(g, lanes, opts)
    for lane, s in srcs.items():
        b.admit(lane, s)
    b.run(k_iters=k_iters)
    return b


@pytest.mark.parametrize("opts", [dict(), dict(delta=1), dict(delta=40), dict(delta=0xFFFFFFFF),
                                  dict(big_degree=2), dict(delta=3, big_degree=8),
                                  dict(dense_lanes=1), dict(dense_lanes=65),
                                  dict(dense_lanes=65, big_degree=2), dict(dense_lanes=4, big_degree=30),
                                  dict(split_wait=1), dict(split_lanes=64, split_wait=1000),
                                  dict(delta=2, split_lanes=3, split_wait=2)])
def test_rmat12_64_lanes(fg, orc, opts):
    off, col = synth.rmat_csr(12)
    w = synth.weights(off, col)
    g = fg.Graph(off, col, weights=w)
    srcs = {i: int(s) for i, s in enumerate(synth.sources(off, 64, seed=21))}
    announce(f"mssp rmat12 64 lanes {opts}")
    b = run_batch(fg, g, srcs, fg.mssp_opts(**opts))
    check_lanes(orc, b, off, col, w, srcs)
    e, el = b.counts()
    assert 0 < e <= el


@pytest.mark.parametrize("delta,dense,split", [(0, 0, 0), (1, 0, 0), (500, 0, 0), (0, 1, 0), (0, 0, 1),
                                               (7, 0, 100)])
def test_grid_lanes(fg, orc, delta, dense, split):
    off, col = synth.grid_csr(120, 130)
    w = synth.weights(off, col)
    g = fg.Graph(off, col, weights=w)
    rng = np.random.default_rng(4)
    srcs = {int(l): int(s) for l, s in zip(rng.choice(64, 9, replace=False),
                                           rng.choice(len(off) - 1, 9, replace=False))}
    announce(f"mssp grid 120x130 lanes {sorted(srcs)} delta={delta} dense={dense} split={split}")
    b = run_batch(fg, g, srcs, fg.mssp_opts(delta=delta, dense_lanes=dense, split_wait=split,
                                            split_lanes=split), k_iters=100)
    check_lanes(orc, b, off, col, w, srcs)


@pytest.mark.parametrize("team,team_e,lanes", [(32, 0, 1), (32, 0, 3), (64, 0, 8), (2, 0, 5),
                                               (7, 0, 64), (32, 500, 4), (-1, 0, 4)])
def test_team_iterations(fg, orc, team, team_e, lanes):
    # grid near iterations run as a team; k_iters=5 ends episodes in
    # mid-flight and lanes are admitted between steps
    R, C = 140, 160
    off, col = synth.grid_csr(R, C)
    w = synth.weights(off, col)
    g = fg.Graph(off, col, weights=w)
    rng = np.random.default_rng(abs(team) * 10 + lanes)
    srcs = {int(l): int(s) for l, s in zip(rng.choice(64, lanes, replace=False),
                                           rng.choice(R * C, lanes, replace=False))}
    announce(f"mssp team={team} team_e={team_e} lanes={lanes}")
    b = fg.MsspBatch(g, 64, fg.mssp_opts(team_blocks=team, team_edges=team_e))
    items = list(srcs.items())
    half = len(items) // 2
    for lane, s_ in items[:half]:
        b.admit(lane, s_)
    if half:
        b.step(5)
    for lane, s_ in items[half:]:
        b.admit(lane, s_)
    b.run(k_iters=5)
    check_lanes(orc, b, off, col, w, srcs)
    # R-MAT: hubs on the first levels hand the frontier back to the full grid
    off, col = synth.rmat_csr(12)
    w = synth.weights(off, col)
    g = fg.Graph(off, col, weights=w)
    srcs = {i: int(s_) for i, s_ in enumerate(synth.sources(off, lanes, seed=abs(team) + 9))}
    b = run_batch(fg, g, srcs, fg.mssp_opts(team_blocks=team, team_edges=team_e, delta=5), k_iters=7)
    check_lanes(orc, b, off, col, w, srcs)


def test_closed_form_grid(fg):
    R, C = 30, 40
    off, col = synth.grid_csr(R, C)
    w = np.full(len(col), 5, np.uint32)
    g = fg.Graph(off, col, weights=w)
    srcs = {0: 0, 1: R * C - 1, 2: 17 * C + 3}
    b = run_batch(fg, g, srcs, lanes=3)
    for lane, s in srcs.items():
        r0, c0 = divmod(s, C)
        want = [5 * (abs(r - r0) + abs(c - c0)) for r in range(R) for c in range(C)]
        assert to_np(b.read(lane)).astype(np.int64).tolist() == want


def test_duplicates_isolated_zero_weights(fg, orc):
    off, col = synth.from_edge_pairs(300, [(i, i + 1) for i in range(250)] + [(0, 260)])
    w = synth.weights(off, col) % 3  # many zero weights (symmetric)
    g = fg.Graph(off, col, weights=w)
    srcs = {0: 5, 1: 5, 2: 299, 3: 120, 7: 0}
    b = run_batch(fg, g, srcs, lanes=8, k_iters=64)
    check_lanes(orc, b, off, col, w, srcs)


def test_directed(fg, orc):
    rng = np.random.default_rng(3)
    n = 2000
    eu = rng.integers(0, n, 15000)
    ev = rng.integers(0, n, 15000)
    keep = eu != ev
    pairs = np.unique(np.stack([eu[keep], ev[keep]], 1), axis=0)
    pairs = pairs[np.lexsort((pairs[:, 1], pairs[:, 0]))]
    off = np.zeros(n + 1, np.int32)
    np.add.at(off, pairs[:, 0] + 1, 1)
    off = np.cumsum(off).astype(np.int32)
    col = pairs[:, 1].astype(np.int32)
    w = rng.integers(1, 65, len(col)).astype(np.uint32)
    g = fg.Graph(off, col, weights=w, symmetric=False)
    srcs = {i: i * 7 for i in range(20)}
    b = run_batch(fg, g, srcs)
    check_lanes(orc, b, off, col, w, srcs)


def test_continuous_admission_and_reuse(fg, orc):
    off, col = synth.rmat_csr(13)
    w = synth.weights(off, col)
    g = fg.Graph(off, col, weights=w)
    src = [int(s) for s in synth.sources(off, 100, seed=9)]
    b = fg.MsspBatch(g, 64, fg.mssp_opts(delta=20))
    first = {i: src[i] for i in range(30)}
    for lane, s in first.items():
        b.admit(lane, s)
    b.step(2)
    # more lanes join a running batch
    second = {30 + i: src[30 + i] for i in range(20)}
    for lane, s in second.items():
        b.admit(lane, s)
    b.step(1)
    # a live lane is replaced by a new query before it finishes
    b.admit(3, src[90])
    first[3] = src[90]
    b.run(k_iters=8)
    check_lanes(orc, b, off, col, w, {**first, **second})
    # finished lanes are released and reused
    third = {}
    for lane in range(10):
        b.release(lane)
        b.admit(lane, src[50 + lane])
        third[lane] = src[50 + lane]
    b.run(k_iters=8)
    check_lanes(orc, b, off, col, w, third)
    check_lanes(orc, b, off, col, w, second)


def test_same_alone_and_in_mix(fg, orc):
    off, col = synth.rmat_csr(11)
    w = synth.weights(off, col)
    g = fg.Graph(off, col, weights=w)
    srcs = [int(s) for s in synth.sources(off, 40, seed=2)]
    mix = run_batch(fg, g, {i: s for i, s in enumerate(srcs)})
    for i in (0, 17, 39):
        alone = run_batch(fg, g, {5: srcs[i]}, lanes=8)
        assert np.array_equal(to_np(alone.read(5)), to_np(mix.read(i)))
        d, _, st = fg.sssp(g, srcs[i])
        assert np.array_equal(to_np(d).astype(np.uint32), to_np(mix.read(i)).astype(np.uint32))


def test_overflow_and_errors(fg):
    off, col = synth.from_edge_pairs(3, [(0, 1), (1, 2)])
    w = np.full(len(col), 0x90000000, np.uint32)
    g = fg.Graph(off, col, weights=w)
    b = fg.MsspBatch(g, 4)
    b.admit(0, 0)
    b.step(100)
    with pytest.raises(fg.FGError) as e:
        b.poll()
    assert e.value.status == fg.FG_EOVERFLOW
    g2 = fg.Graph(off, col)
    with pytest.raises(fg.FGError) as e:
        fg.MsspBatch(g2, 4)
    assert e.value.status == fg.FG_EINVAL
    b2 = fg.MsspBatch(fg.Graph(off, col, weights=np.ones(len(col), np.uint32)), 4)
    for bad in ((4, 0), (-1, 0), (0, 3)):
        with pytest.raises(fg.FGError):
            b2.admit(*bad)
    b2.admit(1, 2)
    with pytest.raises(fg.FGError):
        b2.admit(1, 0)  # already pending
