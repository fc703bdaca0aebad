"""Parity of the share builder and the package step (split + gather) with
the oracle's share builder and serial package loop (exact, stable order)."""
import json
import os

import numpy as np
import pytest
import torch

import synth
from gpu_util import announce, gpu, need_gpu, to_np

pytestmark = gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def fg():
    need_gpu()
    import paper_1504_04804_amd as fg
    fg.lib()
    return fg


def check_share(fg, orc, off, col, owner, nparts, part):
    announce(f"share n={len(off)-1} nparts={nparts} part={part}")
    sh = fg.Share(off, col, owner, nparts, part)
    want = orc.share_build(off, col, owner, part)
    assert sh.n_local == want["n_local"] and sh.n_total == want["n_total"]
    lown, conv, l2g = sh.tables()
    assert np.array_equal(lown, want["owner"])
    assert np.array_equal(conv, want["conv"])
    assert np.array_equal(l2g, want["l2g"])
    loff, lcol = sh.csr()
    assert np.array_equal(loff, want["off"]) and np.array_equal(lcol, want["col"])
    return sh, want


def check_package(fg, orc, sh, want, frontier, depth, parent, nparts):
    announce(f"package len={len(frontier)}")
    dev = torch.from_numpy(np.ascontiguousarray(frontier, np.int32)).cuda()
    d_dev = torch.from_numpy(depth).cuda()
    p_dev = torch.from_numpy(parent).cuda()
    ids, dep, par, counts, local, lc = fg.package(sh, dev, len(frontier), d_dev, p_dev)
    bufs, wlocal = orc.package(frontier, want["n_local"], want["owner"], want["conv"], depth,
                               parent, want["l2g"], nparts=nparts)
    cap = max(len(frontier), 1)
    ids, dep, par, counts = to_np(ids), to_np(dep), to_np(par), to_np(counts)
    for p in range(nparts):
        c = len(bufs[p]["ids"])
        assert counts[p] == c
        s = slice(p * cap, p * cap + c)
        assert np.array_equal(ids[s], bufs[p]["ids"])
        assert np.array_equal(dep[s], bufs[p]["depth"])
        assert np.array_equal(par[s], bufs[p]["parent"])
    k = int(to_np(lc)[0])
    assert np.array_equal(to_np(local)[:k], wlocal)


def test_golden_share(fg, orc):
    g = json.load(open(os.path.join(GOLDEN, "small_graphs.json")))["share_build"]
    off, col = synth.from_edge_pairs(g["n"], g["edges"])
    sh, want = check_share(fg, orc, off, col, np.array(g["owner"], np.uint8), 2, g["part"])
    loff, lcol = sh.csr()
    assert loff.tolist() == g["row_offsets"] and lcol.tolist() == g["cols"]


@pytest.mark.parametrize("nparts", [2, 4, 7])
def test_share_and_package_rmat(fg, orc, nparts):
    off, col = synth.rmat_csr(13)
    owner = synth.owners(len(off) - 1, nparts)
    rng = np.random.default_rng(nparts)
    for part in range(nparts):
        sh, want = check_share(fg, orc, off, col, owner, nparts, part)
        # per-level output frontiers of a BFS on the share (from the oracle)
        src = 0
        depth, parent, cnt, _ = orc.bfs(want["off"], want["col"], src)
        for k in range(len(cnt) - 1):
            fr = np.flatnonzero(depth == k + 1).astype(np.int32)
            check_package(fg, orc, sh, want, fr, depth, parent, nparts)
            check_package(fg, orc, sh, want, rng.permutation(fr), depth, parent, nparts)


def test_package_edge_cases(fg, orc):
    off, col = synth.rmat_csr(12)
    owner = synth.owners(len(off) - 1, 4)
    sh, want = check_share(fg, orc, off, col, owner, 4, 1)
    depth, parent, cnt, _ = orc.bfs(want["off"], want["col"], 3)
    nt = want["n_total"]
    depth = np.where(depth < 0, 5, depth).astype(np.int32)
    parent = np.where(parent < 0, 0, parent).astype(np.int32)
    rng = np.random.default_rng(9)
    for L in (0, 1, 4095, 4096, 4097, 3 * 4096 + 17, nt):
        fr = rng.choice(nt, size=min(L, nt), replace=False).astype(np.int32)
        check_package(fg, orc, sh, want, fr, depth, parent, 4)
    loc = np.arange(min(5000, want["n_local"]), dtype=np.int32)  # all local
    check_package(fg, orc, sh, want, loc, depth, parent, 4)
    rem = np.arange(want["n_local"], nt, dtype=np.int32)  # all remote
    check_package(fg, orc, sh, want, rem, depth, parent, 4)
    with pytest.raises(fg.FGError) as e:
        fg.package(sh, torch.zeros(10, dtype=torch.int32, device="cuda"), 10,
                   torch.zeros(nt, dtype=torch.int32, device="cuda"), capacity=5)
    assert e.value.status == fg.FG_EINVAL


@pytest.mark.slow
def test_config_rmat24_quarter_share(fg, orc):
    """One GPU's quarter share of R-MAT scale 24 at its real shape."""
    off, col = synth.rmat_csr(24)
    owner = synth.owners(len(off) - 1, 4)
    sh, want = check_share(fg, orc, off, col, owner, 4, 0)
    depth, parent, cnt, _ = orc.bfs(want["off"], want["col"], 0)
    for k in range(len(cnt) - 1):
        fr = np.flatnonzero(depth == k + 1).astype(np.int32)
        check_package(fg, orc, sh, want, fr, depth, parent, 4)
