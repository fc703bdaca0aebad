"""Parity of the standalone operators (advance, filter, pull step, queue /
bitmap conversions) with serial expectations computed from the oracle."""
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


def serial_advance(off, col, frontier):
    dst = [col[off[u]:off[u + 1]] for u in frontier]
    src = [np.full(off[u + 1] - off[u], u, np.int32) for u in frontier]
    if not dst:
        return np.zeros(0, np.int32), np.zeros(0, np.int32)
    return np.concatenate(dst), np.concatenate(src)


@pytest.mark.parametrize("scale", [10, 14])
def test_advance_exact_layout(fg, scale):
    off, col = synth.rmat_csr(scale)
    g = fg.Graph(off, col)
    rng = np.random.default_rng(scale)
    n = len(off) - 1
    for size in (0, 1, 63, 64, 65, 1000, n):
        fr = rng.choice(n, size=size, replace=False).astype(np.int32)
        if size and size < n:
            fr[0] = 0  # include the hub
        announce(f"advance scale={scale} size={size}")
        q = torch.from_numpy(fr).cuda() if size else torch.zeros(1, dtype=torch.int32, device="cuda")
        dst, src, tot = fg.advance(g, q[:size] if size else q[:0])
        wd, ws = serial_advance(off, col, fr)
        T = int(to_np(tot)[0])
        assert T == len(wd)
        assert np.array_equal(to_np(dst)[:T], wd)
        assert np.array_equal(to_np(src)[:T], ws)


def test_advance_capacity_overflow(fg):
    off, col = synth.rmat_csr(10)
    g = fg.Graph(off, col)
    q = torch.tensor([0, 1, 2], dtype=torch.int32, device="cuda")
    dst, src, tot = fg.advance(g, q, capacity=10)
    wd, _ = serial_advance(off, col, [0, 1, 2])
    assert int(to_np(tot)[0]) == len(wd)  # the size that would be needed
    assert np.array_equal(to_np(dst)[:10], wd[:10])


def test_filter_heavy_duplicates(fg):
    n = 5000
    off, col = synth.rmat_csr(12)
    g = fg.Graph(off, col)
    rng = np.random.default_rng(1)
    dst = rng.integers(0, 50, size=100000).astype(np.int32)  # heavy duplication
    src = rng.integers(0, n, size=100000).astype(np.int32)
    visited = torch.zeros((4096 + 31) // 32, dtype=torch.int32, device="cuda")
    pre = [3, 7, 49]
    vis_np = np.zeros(len(visited), np.uint32)
    for v in pre:
        vis_np[v >> 5] |= np.uint32(1 << (v & 31))
    visited.copy_(torch.from_numpy(vis_np.view(np.int32)))
    depth = torch.full((4096,), -1, dtype=torch.int32, device="cuda")
    parent = torch.full((4096,), -1, dtype=torch.int32, device="cuda")
    out_q = torch.empty(4096, dtype=torch.int32, device="cuda")
    out_len = torch.zeros(1, dtype=torch.int32, device="cuda")
    announce("filter duplicates")
    fg.filter_(g, torch.from_numpy(dst).cuda(), torch.from_numpy(src).cuda(), len(dst), visited,
               4, depth, parent, out_q, out_len)
    k = int(to_np(out_len)[0])
    got = to_np(out_q)[:k]
    want = sorted(set(dst.tolist()) - set(pre))
    assert sorted(got.tolist()) == want  # each vertex once
    d = to_np(depth)
    p = to_np(parent)
    assert (d[want] == 5).all() and (d[pre] == -1).all()
    for v in want:  # parent is one of the edges that reached v
        assert p[v] in set(src[dst == v].tolist())
    vis = to_np(visited).view(np.uint32)
    for v in want + pre:
        assert vis[v >> 5] >> (v & 31) & 1


def test_pull_step_matches_level(fg, orc):
    off, col = synth.rmat_csr(13)
    n = len(off) - 1
    g = fg.Graph(off, col)
    depth_ref, _, cnt, _ = orc.bfs(off, col, 0)
    nw = (n + 63) // 64
    for k in range(len(cnt)):
        # state at the start of iteration k: visited = depth <= k, frontier = depth == k
        vis = np.zeros(nw, np.uint64)
        fb = np.zeros(nw, np.uint64)
        for v in np.flatnonzero((depth_ref >= 0) & (depth_ref <= k)):
            vis[v >> 6] |= np.uint64(1) << np.uint64(v & 63)
        for v in np.flatnonzero(depth_ref == k):
            fb[v >> 6] |= np.uint64(1) << np.uint64(v & 63)
        T = lambda a: torch.from_numpy(a.view(np.int64)).cuda()
        visited, fbits = T(vis.copy()), T(fb)
        nxt = torch.full((nw,), -1, dtype=torch.int64, device="cuda")
        depth = torch.full((n,), -1, dtype=torch.int32, device="cuda")
        parent = torch.full((n,), -1, dtype=torch.int32, device="cuda")
        out_q = torch.empty(n, dtype=torch.int32, device="cuda")
        out_len = torch.zeros(1, dtype=torch.int32, device="cuda")
        insp = torch.zeros(1, dtype=torch.int64, device="cuda")
        announce(f"pull step k={k}")
        fg.pull_step(g, fbits, visited, nxt, k, depth, parent, out_q, out_len, insp)
        want_new = np.flatnonzero(depth_ref == k + 1)
        got = to_np(out_q)[:int(to_np(out_len)[0])]
        assert sorted(got.tolist()) == want_new.tolist()
        d = to_np(depth)
        p = to_np(parent)
        assert np.array_equal(np.flatnonzero(d == k + 1), want_new)
        for v in want_new:  # early exit: first neighbour in CSR order at depth k
            row = col[off[v]:off[v + 1]]
            assert p[v] == row[np.argmax(depth_ref[row] == k)]
        dirs = np.ones(k + 1, np.int8)
        assert int(to_np(insp)[0]) == orc.edges_inspected(off, col, depth_ref, dirs)[k]
        nb = to_np(nxt).view(np.uint64)
        want_nb = np.zeros(nw, np.uint64)
        for v in want_new:
            want_nb[v >> 6] |= np.uint64(1) << np.uint64(v & 63)
        assert np.array_equal(nb, want_nb)
        assert np.array_equal(to_np(visited).view(np.uint64), vis | want_nb)


def test_queue_bitmap_roundtrip(fg):
    off, col = synth.rmat_csr(12)
    n = len(off) - 1
    g = fg.Graph(off, col)
    rng = np.random.default_rng(5)
    for size in (0, 1, 64, 777, n):
        q = np.sort(rng.choice(n, size=size, replace=False)).astype(np.int32)
        bits = torch.zeros((n + 63) // 64, dtype=torch.int64, device="cuda")
        qt = torch.from_numpy(q).cuda() if size else torch.zeros(0, dtype=torch.int32, device="cuda")
        fg.queue_to_bitmap(g, qt, size, bits)
        out = torch.empty(n, dtype=torch.int32, device="cuda")
        out_len = torch.zeros(1, dtype=torch.int32, device="cuda")
        fg.bitmap_to_queue(g, bits, out, out_len)
        k = int(to_np(out_len)[0])
        assert k == size
        assert np.array_equal(to_np(out)[:k], q)  # ascending order


def test_graph_validation_errors(fg):
    off, col = synth.from_edge_pairs(4, [(0, 1), (1, 2)])
    bad_col = col.copy()
    bad_col[0] = 7
    with pytest.raises(fg.FGError) as e:
        fg.Graph(off, bad_col)
    assert e.value.status == fg.FG_EINVAL
    bad_off = off.copy()
    bad_off[2] = 0
    with pytest.raises(fg.FGError):
        fg.Graph(bad_off, col)
    # directed graph claimed symmetric
    doff = np.array([0, 1, 1, 1, 1], np.int32)
    dcol = np.array([1], np.int32)
    with pytest.raises(fg.FGError):
        fg.Graph(doff, dcol, symmetric=True)
    g = fg.Graph(doff, dcol, symmetric=False)
    with pytest.raises(fg.FGError) as e:
        fg.bfs(g, 0, mode=fg.FG_MODE_DO)
    assert e.value.status == fg.FG_EUNSUPPORTED
    d, p, st = fg.bfs(g, 0, mode=fg.FG_MODE_PUSH)  # push works on directed graphs
    assert to_np(d).tolist() == [0, 1, -1, -1]
    with pytest.raises(fg.FGError) as e:
        fg.bfs(g, 4, mode=fg.FG_MODE_PUSH)
    assert e.value.status == fg.FG_EINVAL
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    depth = torch.empty(4, dtype=torch.int32, device="cuda")
    with pytest.raises(fg.FGError) as e:
        fg.bfs_into(g, 0, depth, None, fg.bfs_opts(mode=1), ws=ws)
    assert e.value.status == fg.FG_ENOMEM
