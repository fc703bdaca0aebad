"""Parity of the 64-lane batched BFS: every lane's depths equal the oracle's
BFS from that lane's source (and fg_bfs's), alone or in the mix, including
lanes admitted mid-flight and lanes reused after release."""
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


def check_lanes(fg, orc, b, off, col, srcs):
    for lane, s in srcs.items():
        got = to_np(b.read(lane))
        want = orc.bfs(off, col, int(s))[0]
        assert np.array_equal(got, want), f"lane {lane} src {s}: {np.flatnonzero(got != want)[:8]}"


@pytest.mark.parametrize("opts", [dict(), dict(pull_div=1), dict(pull_div=1 << 30, push_div=1 << 30),
                                  dict(big_degree=4)])
def test_rmat12_64_lanes(fg, orc, opts):
    off, col = synth.rmat_csr(12)
    g = fg.Graph(off, col)
    srcs = {i: int(s) for i, s in enumerate(synth.sources(off, 64, seed=11))}
    announce(f"msbfs rmat12 64 lanes {opts}")
    b = fg.MsBatch(g, 64, fg.msbfs_opts(**opts))
    for lane, s in srcs.items():
        b.admit(lane, s)
    b.run(k_iters=4)
    check_lanes(fg, orc, b, off, col, srcs)


def test_few_lanes_duplicates_isolated(fg, orc):
    off, col = synth.from_edge_pairs(300, [(i, i + 1) for i in range(250)] + [(0, 260)])
    g = fg.Graph(off, col)
    srcs = {0: 5, 1: 5, 2: 299, 3: 120, 7: 0}
    b = fg.MsBatch(g, 8)
    for lane, s in srcs.items():
        b.admit(lane, s)
    b.run(k_iters=64)
    check_lanes(fg, orc, b, off, col, srcs)


def test_continuous_admission_and_reuse(fg, orc):
    off, col = synth.rmat_csr(13)
    g = fg.Graph(off, col)
    src = synth.sources(off, 96, seed=5)
    b = fg.MsBatch(g, 64)
    first = {i: int(src[i]) for i in range(32)}
    for lane, s in first.items():
        b.admit(lane, s)
    b.step(2)                       # mid-flight
    second = {32 + i: int(src[32 + i]) for i in range(32)}
    for lane, s in second.items():
        b.admit(lane, s)
    b.run(k_iters=3)
    check_lanes(fg, orc, b, off, col, {**first, **second})
    # reuse lanes 3, 40, 63 for new queries while the others stay done
    again = {3: int(src[64]), 40: int(src[65]), 63: int(src[66])}
    for lane in again:
        b.release(lane)
    for lane, s in again.items():
        b.admit(lane, s)
    b.run(k_iters=5)
    check_lanes(fg, orc, b, off, col, again)
    check_lanes(fg, orc, b, off, col, {5: first[5], 50: second[50]})  # untouched lanes


def test_alone_equals_in_the_mix(fg, orc):
    off, col = synth.rmat_csr(12)
    g = fg.Graph(off, col)
    srcs = [int(s) for s in synth.sources(off, 64, seed=2)]
    b = fg.MsBatch(g, 64)
    for lane, s in enumerate(srcs):
        b.admit(lane, s)
    b.run()
    alone = fg.MsBatch(g, 1)
    for lane in (0, 17, 63):
        single, _, _ = fg.bfs(g, srcs[lane], mode=fg.FG_MODE_DO)
        mix = to_np(b.read(lane))
        alone.admit(0, srcs[lane])
        alone.run()
        assert np.array_equal(mix, to_np(single))
        assert np.array_equal(mix, to_np(alone.read(0)))


def test_grid_64_sources_closed_form(fg):
    R = C = 96
    off, col = synth.grid_csr(R, C)
    g = fg.Graph(off, col)
    rng = np.random.default_rng(4)
    srcs = rng.choice(R * C, 64, replace=False)
    b = fg.MsBatch(g, 64)
    for lane, s in enumerate(srcs):
        b.admit(lane, int(s))
    b.run(k_iters=32)
    rr, cc = np.divmod(np.arange(R * C), C)
    for lane, s in enumerate(srcs):
        r0, c0 = divmod(int(s), C)
        assert np.array_equal(to_np(b.read(lane)), np.abs(rr - r0) + np.abs(cc - c0))


@pytest.mark.parametrize("team,team_e,lanes", [(32, 0, 1), (32, 0, 8), (2, 0, 5), (7, 0, 64),
                                               (64, 0, 3), (32, 300, 8), (-1, 0, 8), (0, 0, 4),
                                               (1, 0, 2)])
def test_team_levels(fg, orc, team, team_e, lanes):
    # grid levels run as a team; k_iters=3 ends episodes in mid-flight and
    # the next step resumes them; lanes are admitted between steps
    R, C = 150, 170
    off, col = synth.grid_csr(R, C)
    g = fg.Graph(off, col)
    rng = np.random.default_rng(abs(team) * 100 + lanes)
    srcs = {int(l): int(s) for l, s in zip(rng.choice(64, lanes, replace=False),
                                           rng.choice(R * C, lanes, replace=False))}
    announce(f"msbfs team={team} team_e={team_e} lanes={lanes}")
    b = fg.MsBatch(g, 64, fg.msbfs_opts(team_blocks=team, team_edges=team_e))
    items = list(srcs.items())
    half = len(items) // 2
    for lane, s in items[:half]:
        b.admit(lane, s)
    if half:
        b.step(3)
    for lane, s in items[half:]:
        b.admit(lane, s)
    b.run(k_iters=3)
    check_lanes(fg, orc, b, off, col, srcs)
    # R-MAT with pull off: push levels of every shape, hubs included
    off, col = synth.rmat_csr(13)
    g = fg.Graph(off, col)
    srcs = {i: int(s) for i, s in enumerate(synth.sources(off, lanes, seed=abs(team) + 50))}
    b = fg.MsBatch(g, 64, fg.msbfs_opts(team_blocks=team, team_edges=team_e, pull_div=1))
    for lane, s in srcs.items():
        b.admit(lane, s)
    b.run(k_iters=5)
    check_lanes(fg, orc, b, off, col, srcs)


def test_team_back_to_back_handoffs(fg, orc):
    # One-lane batches on R-MAT with the team requested: a team episode that
    # leaves because the frontier's degree grew is re-entered and handed back
    # at once, so two hand-offs follow each other within microseconds.  Every
    # step must finish (no wait reaching its limit) with the oracle's depths.
    off, col = synth.rmat_csr(16)
    g = fg.Graph(off, col)
    srcs = [int(s) for s in synth.sources(off, 64, seed=99)]
    want = {s: orc.bfs(off, col, s)[0] for s in srcs[:8]}
    announce("msbfs team hand-offs: 150 one-lane batches on rmat16")
    b = fg.MsBatch(g, 64, fg.msbfs_opts(team_blocks=1))
    for r in range(150):
        if r:
            b.release(0)
        s = srcs[r % 8]
        b.admit(0, s)
        b.step(1 << 30)
        done, _ = b.poll()  # raises FGError (FG_EDEVICE) if a wait hit its limit
        assert done & 1
        if r < 8 or r % 16 == 0:
            assert np.array_equal(to_np(b.read(0)), want[s]), f"batch {r} src {s}"


def test_msbfs_argument_errors(fg):
    off, col = synth.from_edge_pairs(4, [(0, 1)])
    g = fg.Graph(off, col)
    b = fg.MsBatch(g, 4)
    for bad in ((4, 0), (-1, 0), (0, 4), (0, -1)):
        with pytest.raises(fg.FGError):
            b.admit(*bad)
    b.admit(1, 0)
    with pytest.raises(fg.FGError):
        b.admit(1, 2)  # already pending


@pytest.mark.slow
def test_config_rmat23_64_sources(fg, orc):
    off, col = synth.rmat_csr(23)
    g = fg.Graph(off, col)
    srcs = [int(s) for s in synth.sources(off, 64, seed=23)]
    b = fg.MsBatch(g, 64)
    for lane, s in enumerate(srcs):
        b.admit(lane, s)
    b.run(k_iters=8)
    check_lanes(fg, orc, b, off, col, {lane: srcs[lane] for lane in (0, 31, 63)})


@pytest.mark.slow
def test_config_grid2048_64_sources(fg):
    R = 2048
    off, col = synth.grid_csr(R, R)
    g = fg.Graph(off, col)
    rng = np.random.default_rng(7)
    srcs = rng.choice(R * R, 64, replace=False)
    b = fg.MsBatch(g, 64)
    for lane, s in enumerate(srcs):
        b.admit(lane, int(s))
    b.run(k_iters=512)
    rr, cc = np.divmod(np.arange(R * R, dtype=np.int64), R)
    for lane in range(0, 64, 9):
        r0, c0 = divmod(int(srcs[lane]), R)
        assert np.array_equal(to_np(b.read(lane)), np.abs(rr - r0) + np.abs(cc - c0))
