"""PageRank (fg_pagerank) against the oracle's double-precision power
iteration (O13), through the C ABI.

Tolerance.  Both sides evaluate the same formula in IEEE double; they
differ only in the order of the additions of a row's sum (the kernel sums
short rows in segments of a wave step, longer rows in strided partial sums
combined as a tree; the oracle in CSR order).  Summing k positive terms in any order is within
gamma_{k-1} = (k-1)u / (1 - (k-1)u) of the exact sum (u = 2^-53), and the
contributions, the update and the division add a few roundings more, so
after K iterations every rank agrees to the relative error
    K * (2 gamma_{D-1} + 8u),   D the largest degree,
which these tests assert elementwise (about 1e-9 for R-MAT 22 after 20
iterations; far tighter on grids).  Iteration counts under the
threshold-ratio stop must be equal.
"""
import numpy as np
import pytest
import torch

import synth
import workloads
from gpu_util import announce, gpu, need_gpu, to_np

pytestmark = gpu

U = 2.0 ** -53


def bound(off, iters):
    D = int(np.diff(off).max()) if len(off) > 1 else 0
    k = max(D - 1, 0)
    gamma = k * U / (1 - k * U)
    return max(iters, 1) * (2 * gamma + 8 * U)


@pytest.fixture(scope="module")
def fg():
    need_gpu()
    import paper_1504_04804_amd as fg
    fg.lib()
    return fg


def check(fg, orc, off, col, what, damping=0.85, tol=0.0, max_iter=20):
    announce(f"pagerank {what} n={len(off) - 1} d={damping} tol={tol} max_iter={max_iter}")
    g = fg.Graph(off, col, symmetric=True, validate=False)
    rank, st = fg.pagerank(g, damping, tol, max_iter)
    got = to_np(rank)
    g.close()
    want, it = orc.pagerank(off, col, damping, tol, max_iter)
    assert st.status == 0
    assert st.iterations == it, (what, st.iterations, it)
    rel = np.abs(got - want) / np.maximum(np.abs(want), 1e-300)
    b = bound(off, it)
    assert rel.max() <= b, (what, float(rel.max()), b)
    return got, st


def test_small_graphs(fg, orc):
    for s in (6, 10, 12, 16):
        off, col = synth.rmat_csr(s)
        check(fg, orc, off, col, f"rmat{s}")
    for r, c in ((1, 2), (9, 13), (100, 70)):
        off, col = synth.grid_csr(r, c)
        check(fg, orc, off, col, f"grid{r}x{c}")


def test_long_rows_and_iterations(fg, orc):
    """R-MAT 18 has rows past the workgroup cut (4096 entries) as well as
    wave-summed and lane-summed rows."""
    off, col = synth.rmat_csr(18)
    assert int(np.diff(off).max()) >= 4096
    for d, it in ((0.85, 1), (0.85, 30), (0.5, 10), (0.0, 3), (1.0, 5)):
        check(fg, orc, off, col, f"rmat18 d={d}", damping=d, max_iter=it)
    check(fg, orc, off, col, "rmat18 no iterations", max_iter=0)


def test_threshold_stop(fg, orc):
    off, col = synth.rmat_csr(14)
    for tol in (1e-2, 1e-4, 1e-6):
        _, st = check(fg, orc, off, col, f"rmat14 tol={tol}", tol=tol, max_iter=200)
        assert 1 <= st.iterations < 200
    off, col = synth.grid_csr(40, 40)
    check(fg, orc, off, col, "grid tol", tol=1e-5, max_iter=500)


def test_regular_graph_uniform_and_trace(fg):
    # every vertex of a cycle keeps 1/n; the trace records the vertices above
    # the threshold (none after the first iteration) and m entries read
    n = 1000
    a = np.arange(n, dtype=np.int32)
    import oracle
    off, col = oracle.oracle().csr_from_edges(n, a, (a + 1) % n)
    g = fg.Graph(off, col)
    rank, st = fg.pagerank(g, 0.85, 1e-12, 50)
    r = to_np(rank)
    assert np.allclose(r, 1.0 / n, rtol=1e-14, atol=0)
    assert st.iterations == 1
    assert st.trace()[1][0] == 0 and st.trace()[2][0] == len(col)
    g.close()


def test_argument_errors(fg):
    off, col = synth.grid_csr(3, 3)
    g = fg.Graph(off, col)
    rank = torch.empty(g.n, dtype=torch.float64, device="cuda")
    for kw, code in ((dict(damping=1.5), fg.FG_EINVAL), (dict(tol=-1.0), fg.FG_EINVAL),
                     (dict(max_iter=-1), fg.FG_EINVAL)):
        with pytest.raises(fg.FGError) as e:
            fg.pagerank_into(g, rank, **kw)
        assert e.value.status == code
    with pytest.raises(fg.FGError) as e:
        fg.pagerank_into(g, rank, ws=torch.zeros(16, dtype=torch.uint8, device="cuda"))
    assert e.value.status == fg.FG_ENOMEM
    g.close()
    gd = fg.Graph(np.array([0, 1, 1], np.int32), np.array([1], np.int32), symmetric=False)
    with pytest.raises(fg.FGError) as e:
        fg.pagerank_into(gd, torch.empty(2, dtype=torch.float64, device="cuda"))
    assert e.value.status == fg.FG_EUNSUPPORTED
    gd.close()


@pytest.mark.slow
def test_workload_rmat22(fg, orc):
    off, col, _ = workloads.graph("rmat22")
    check(fg, orc, off, col, "rmat22", max_iter=20)
