"""Serving: continuous batching over resident graphs.  Every result of the
mixed stream must equal the oracle's answer for that query alone, and the
one-at-a-time path must give the same answers."""
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
    from paper_1504_04804_amd import serve
    specs, graphs, csr = {}, {}, {}
    for name, (off, col) in {
        "rmat10": synth.rmat_csr(10), "rmat12": synth.rmat_csr(12),
        "grid40": synth.grid_csr(40, 40), "grid24x70": synth.grid_csr(24, 70),
    }.items():
        w = synth.weights(off, col)
        graphs[name] = fg.Graph(off, col, weights=w)
        specs[name] = (off, True)
        csr[name] = (off, col, w)
    return fg, serve, specs, graphs, csr


def check_results(orc, csr, done, serve):
    for r in done:
        off, col, w = csr[r.graph]
        got = to_np(r.result)
        if r.kind == serve.BFS:
            want = orc.bfs(off, col, r.src)[0]
            assert np.array_equal(got, want), (r.rid, r.graph, r.src)
        else:
            want = orc.dijkstra(off, col, w, r.src)[0]
            assert np.array_equal(got.astype(np.uint32), want), (r.rid, r.graph, r.src)


@pytest.mark.parametrize("budget,policy,step_ms", [(32 << 30, "batch", 4.0), (1 << 22, "batch", 0.05),
                                                    (32 << 30, "auto", 1.0), (64 << 20, "auto", 0.2),
                                                    (32 << 30, "single", 1.0)])
def test_served_mix_equals_alone(env, orc, budget, policy, step_ms):
    fg, serve, specs, graphs, csr = env
    reqs = serve.make_requests(specs, 160, qps=20000.0, seed=budget & 0xFFFF)
    announce(f"serve 160 requests budget={budget} policy={policy} step_ms={step_ms}")
    costs = None
    if policy == "auto":
        srcs = {n: synth.sources(csr[n][0], 8, seed=4) for n in graphs}
        costs = serve.calibrate(graphs, srcs)
    srv = serve.Server(graphs, hbm_budget=budget, policy=policy, costs=costs, step_ms=step_ms)
    done = serve.serve_stream(srv, reqs, time_limit=120)
    assert len(done) == len(reqs)
    assert sorted(r.rid for r in done) == list(range(len(reqs)))
    assert all(r.done >= r.arrival for r in done)
    check_results(orc, csr, done, serve)
    if policy == "batch":
        assert srv.counts["steps"] > 0
        if budget < (1 << 24):
            # idle batches were closed to make room for others; a request
            # whose batch does not fit while the others are busy runs alone
            assert srv.counts["evictions"] > 0
        else:
            assert all(r.path == "batch" for r in done)
    if policy == "single":
        # single runs, some of them lists run beside a grid query
        assert srv.counts["steps"] == 0
        assert srv.counts["singles"] + srv.counts["corun_list"] == len(reqs)
    st = serve.latency_stats(done)
    assert st["n"] == len(reqs)
    # workspaces stayed within the budget; the graphs' own bytes are counted apart
    assert 0 < srv.peak_used <= budget
    assert srv.resident_bytes == sum(int(g.info().resident_bytes) for g in graphs.values()) > 0


def test_budget_too_small_is_reported(env):
    fg, serve, specs, graphs, csr = env
    reqs = serve.make_requests(specs, 4, qps=20000.0, seed=1)
    srv = serve.Server(graphs, hbm_budget=1024, policy="batch")
    with pytest.raises(RuntimeError):
        serve.serve_stream(srv, reqs, time_limit=60)


def test_fifo_path_same_answers(env, orc):
    fg, serve, specs, graphs, csr = env
    reqs = serve.make_requests(specs, 40, qps=5000.0, seed=3)
    ws = {n: g.workspace(fg.FG_PRIM_SSSP) for n, g in graphs.items()}
    done = serve.serve_fifo(graphs, reqs, ws, time_limit=120)
    check_results(orc, csr, done, serve)


@pytest.mark.slow
def test_served_config_graphs_equal_alone(orc):
    """The serving workload's graph set at full size (R-MAT 16/18/20/22/24,
    grids 1024^2/2048^2/4096^2, weights in [1, 64]) under the benchmark's
    policy and HBM budget: a Poisson stream offered faster than it can be
    served, so queries share batches; every result kept and compared with
    the oracle's answer for that query alone."""
    need_gpu()
    import paper_1504_04804_amd as fg
    from paper_1504_04804_amd import serve
    import workloads
    names = ["rmat16", "rmat18", "rmat20", "rmat22", "rmat24", "grid1024", "grid2048", "grid4096"]
    graphs, specs, csr, srcs = {}, {}, {}, {}
    for name in names:
        off, col, w = workloads.graph(name)
        graphs[name] = fg.Graph(off, col, weights=w, symmetric=True, validate=False)
        specs[name] = (off, True)
        csr[name] = (off, col, w)
        srcs[name] = synth.sources(off, 8, seed=77)
    announce("serve config graphs: calibrate")
    costs = serve.calibrate(graphs, srcs)
    reqs = serve.make_requests(specs, 120, qps=400.0, bfs_frac=0.8, seed=11)
    announce("serve config graphs: 120 requests at 400 q/s, 16 GiB budget")
    srv = serve.Server(graphs, hbm_budget=16 << 30, policy="auto", costs=costs, keep_results=True)
    done = serve.serve_stream(srv, reqs, time_limit=300)
    assert sorted(r.rid for r in done) == list(range(len(reqs)))
    assert sum(1 for r in done if r.path == "batch") > 0
    reads = [(r.rid, r.graph, r.kind, r.src, to_np(r.result)) for r in done]
    for r in done:
        r.result = None

    def check(rid, name, kind, src, got):
        off, col, w = csr[name]
        if kind == serve.BFS:
            want = orc.bfs(off, col, src)[0]
        else:
            want = orc.dijkstra(off, col, w, src)[0]
            got = got.view(np.uint32)
        if not np.array_equal(got, want):
            return f"request {rid} ({name}, kind {kind}, src {src}) differs"
        return None

    with workloads.pool() as ex:
        bad = [e for e in ex.map(lambda t: check(*t), reads) if e is not None]
    assert not bad, bad[:4]
    for g in graphs.values():
        g.close()


def test_grid_singles_co_run_lists(env, orc):
    """Single runs only, a burst of BFS queries on grids (asynchronous
    singles) and on R-MAT graphs: the server runs lists of R-MAT queries
    beside grid queries in one launch, and every result equals the oracle's
    answer for that query alone."""
    fg, serve, specs, graphs, csr = env
    reqs = [r for r in serve.make_requests(specs, 240, qps=50000.0, bfs_frac=1.0, seed=77)]
    announce("serve 240 BFS requests, single runs, co-run lists beside grid queries")
    srv = serve.Server(graphs, hbm_budget=32 << 30, policy="single")
    done = serve.serve_stream(srv, reqs, time_limit=120)
    assert len(done) == len(reqs)
    assert sorted(r.rid for r in done) == list(range(len(reqs)))
    assert srv.counts["coruns"] > 0 and srv.counts["corun_list"] >= srv.counts["coruns"]
    assert sum(1 for r in done if r.path == "corun") == srv.counts["corun_list"]
    check_results(orc, csr, done, serve)
    srv.close()
