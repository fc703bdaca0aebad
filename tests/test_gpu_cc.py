"""Connected components (fg_cc, hooking + pointer jumping) against the
oracle's component-minimum labels (O12), bit-exact, through the C ABI:
sparse random graphs with many components, R-MAT (many isolated
vertices), grids, degenerate graphs, and the workload graphs R-MAT 22 and
the 4096 x 4096 grid."""
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


def er_graph(n, p, seed):
    rng = np.random.default_rng(seed)
    k = int(rng.binomial(n * (n - 1) // 2, p))
    eu = rng.integers(0, n, k).astype(np.int32)
    ev = rng.integers(0, n, k).astype(np.int32)
    return eu, ev


def check(fg, orc, off, col, what):
    announce(f"cc {what} n={len(off) - 1} m={len(col)}")
    g = fg.Graph(off, col, symmetric=True, validate=True)
    for rep in range(2):  # twice on the same graph: no state kept between calls
        label, comps = fg.cc(g)
        want, wc = orc.cc(off, col)
        got = to_np(label)
        assert np.array_equal(got, want), (what, rep, np.flatnonzero(got != want)[:8])
        assert comps == wc
    g.close()


@pytest.mark.parametrize("seed", range(6))
def test_sparse_random_many_components(fg, orc, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1000, 200000))
    for avg in (0.3, 0.9, 1.1, 3.0):
        eu, ev = er_graph(n, avg / n, seed * 10 + int(avg * 10))
        off, col = orc.csr_from_edges(n, eu, ev)
        check(fg, orc, off, col, f"er seed={seed} avg={avg}")


def test_rmat_and_grids(fg, orc):
    for s in (8, 12, 16, 18):
        off, col = synth.rmat_csr(s)
        check(fg, orc, off, col, f"rmat{s}")
    for r, c in ((1, 1), (1, 700), (33, 65), (512, 512)):
        off, col = synth.grid_csr(r, c)
        check(fg, orc, off, col, f"grid{r}x{c}")


def test_degenerate(fg, orc):
    # no edges; one vertex; a path written in descending order; a star whose
    # centre has the largest id; two components interleaved by parity
    off, col = orc.csr_from_edges(9, np.zeros(0, np.int32), np.zeros(0, np.int32))
    check(fg, orc, off, col, "empty")
    off, col = orc.csr_from_edges(1, np.zeros(0, np.int32), np.zeros(0, np.int32))
    check(fg, orc, off, col, "single")
    n = 5000
    eu = np.arange(n - 1, 0, -1, dtype=np.int32)
    off, col = orc.csr_from_edges(n, eu, eu - 1)
    check(fg, orc, off, col, "path")
    leaves = np.arange(0, 9999, dtype=np.int32)
    off, col = orc.csr_from_edges(10000, leaves, np.full_like(leaves, 9999))
    check(fg, orc, off, col, "star")
    a = np.arange(0, 20000 - 2, dtype=np.int32)
    off, col = orc.csr_from_edges(20000, a, a + 2)
    check(fg, orc, off, col, "parity")


def test_directed_graph_rejected(fg):
    off = np.array([0, 1, 1], np.int32)
    col = np.array([1], np.int32)
    g = fg.Graph(off, col, symmetric=False, validate=True)
    label = torch.empty(2, dtype=torch.int32, device="cuda")
    with pytest.raises(fg.FGError) as e:
        fg.cc_into(g, label)
    assert e.value.status == fg.FG_EUNSUPPORTED
    g.close()


@pytest.mark.slow
@pytest.mark.parametrize("name", ["rmat22", "grid4096"])
def test_workload_graphs(fg, orc, name):
    off, col, _ = workloads.graph(name)
    announce(f"cc {name}")
    g = fg.Graph(off, col, symmetric=True, validate=False)
    label, comps = fg.cc(g)
    got = to_np(label)
    g.close()
    want, wc = orc.cc(off, col)
    assert np.array_equal(got, want)
    assert comps == wc
