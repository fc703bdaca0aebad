"""Benchmark: BFS GTEPS and HBM-roofline fraction on one MI355X.

Workload (one "step"): direction-optimizing BFS on an undirected R-MAT
scale-22 graph (edge factor 16, a/b/c/d = 0.57/0.19/0.19/0.05, seeded,
symmetrized, self-loops and duplicates removed, int32 CSR) from 64 seeded
random sources of nonzero degree, run one at a time, followed by a push-only
BFS from vertex 0 of a 4096 x 4096 4-neighbour grid.  Inputs are synthetic
and resident in HBM before timing starts; every traversal writes int32
depths and parents.

Prints one JSON line.  `value` = traversed edges of the whole step (directed
CSR entries of each reached component, summed over the 65 traversals)
divided by the step time.  `roofline` covers the dominant kernel, measured
with HIP events on the stream the kernels run on; its algorithmic bytes
come from the per-iteration device statistics.  `cpu_baseline` times the
serial CPU oracle on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
SCALE = 22
EDGE_FACTOR = 16
NSRC = 64
GRID = 4096
# HBM bytes per call of the step (the co-run launch with the grid query's
# per-vertex kernels) and per launch of each part alone, from the two
# rocprofv3 counter passes (read = 2 x FETCH_SIZE KiB, written = 1 x
# WRITE_SIZE KiB, factors from a plain 512 MiB device copy;
# profiles/bfs_corun_hbm_counters_rmat22x64_grid4096.md).  They hold only for
# the kernel sources they were taken with: `traffic` is null when these files
# hash differently.
TRAFFIC_SOURCES = ('csrc/bfs.hip', 'csrc/fg_common.h', 'csrc/frontier.h', 'csrc/graph.hip')
TRAFFIC_SHA256 = "6ef736068ac5f3bec40429181f5da897c5f9528905629ce593264114577c3d23"
TRAFFIC_BYTES = {"bfs_corun<DO>": 17391240357, "bfs_persistent<DO,many> (alone)": 15681685012,
                 "bfs_async (alone)": 2284606114}
# The same for the side workloads' kernels (per launch; PageRank per
# iteration), from the same two passes
# (profiles/side_kernels_hbm_counters.md), each guarded by a hash of the
# sources its kernel is built from.
_COMMON = ('csrc/fg_common.h', 'csrc/frontier.h', 'csrc/graph.hip')
SIDE_TRAFFIC = {
    "sssp": (('csrc/sssp.hip',) + _COMMON, 12585977507),
    "c4_rmat23": (('csrc/msbfs.hip',) + _COMMON, 21726244032),
    "c4_grid2048": (('csrc/msbfs.hip',) + _COMMON, 519228470197),
    "mssp_rmat22": (('csrc/mssp.hip',) + _COMMON, 146081522000),
    "mssp_grid2048": (('csrc/mssp.hip',) + _COMMON, 515918020064),
    "pagerank_iter": (('csrc/pagerank.hip',) + _COMMON, 4345314838),
}
SIDE_TRAFFIC_SHA256 = {
    "sssp": "0c737dc3597a498653df2bc2c3f9d03779fecc203dcf69743c2fda4c247c17f9",
    "c4_rmat23": "d65b3c254cb6f58ea6a820a3443705ebc8ef5830fea8f8d67622caafa447cc04",
    "c4_grid2048": "d65b3c254cb6f58ea6a820a3443705ebc8ef5830fea8f8d67622caafa447cc04",
    "mssp_rmat22": "4e66b1cdc302c4f10bbded066dbb52a4cee6aa8a09bb20686e01b0b33720ea13",
    "mssp_grid2048": "4e66b1cdc302c4f10bbded066dbb52a4cee6aa8a09bb20686e01b0b33720ea13",
    "pagerank_iter": "cf991295ce6159f97056e3398989083834760a04a0e2907e1baa7230344e77ce",
}


def _sources_sha(names):
    import hashlib
    h = hashlib.sha256()
    for f in names:
        with open(os.path.join(ROOT, "paper_1504_04804_amd", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def side_traffic(name, seconds):
    """Counter bytes of a side workload's kernel and the rate they give, or
    Nones when its sources differ from those the counters were taken on."""
    if name not in SIDE_TRAFFIC or _sources_sha(SIDE_TRAFFIC[name][0]) != SIDE_TRAFFIC_SHA256.get(name):
        return {"traffic": None, "traffic_gbs": None}
    b = SIDE_TRAFFIC[name][1]
    return {"traffic": b, "traffic_gbs": round(b / seconds / 1e9, 2)}

# Launch options of every timed workload (DO thresholds do_a / do_b of
# Sec. VI-A, push load-balance cut, team width, batched push/pull switch
# points) come from paper_1504_04804_amd/tuned.json, which the autotuner
# (python -m paper_1504_04804_amd.autotune) writes for these workloads; the
# paper's own example thresholds for social graphs are 1/100 and 1/10.


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-sources", type=int, default=8)
    ap.add_argument("--headline-only", action="store_true",
                    help="skip the per-config side measurements (SSSP, package, batched, serving)")
    ap.add_argument("--only", default=None,
                    help="comma-separated side measurements to run (sssp, package, batched, "
                         "batched_sssp, overhead, dupall, cc, pagerank, serving); the others "
                         "are skipped")
    ap.add_argument("--no-widened", action="store_true",
                    help="skip the duplicate-all DOBFS, CC and PageRank measurements")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving sweep (the other side measurements still run)")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="first run a plain 512 MiB device copy three times (for the "
                         "rocprof FETCH_SIZE / WRITE_SIZE scale factor)")
    return ap.parse_args()


# ------------------------------------------------------------ algorithmic bytes

def bfs_alg_bytes(st, n, nwords, nnz, parents=True):
    """Compulsory HBM bytes of one traversal from its device statistics.

    outputs   : depth (+ parent) written once per vertex: by the level that
                reaches it (counted below) or, -1, after the last level
                (unreached vertices, with one read of the visited bitmap)
    init      : visited bitmap cleared
    push k    : queue + 2 offsets per frontier vertex (12|Q|), one column
                index per inspected edge (4 insp), the target's visited word
                (min(n/8, 4 insp): the bitmap is read at most once per
                iteration), depth + parent + queue entry per new vertex
    pull k    : visited-in, nonzero-degree mask and visited-out bitmaps
                (3 n/8), 2 offsets per candidate (8|U|), one column index
                per inspected edge, the frontier bitmap once (n/8),
                depth + parent per new vertex
    pull->push: two bitmaps read, the new queue written
    """
    pb = 8 if parents else 4
    total = 8 * nwords + 8 * nwords + pb * max(n - st.reached, 0)
    k_tr = min(st.iterations, 64)
    fr = list(st.frontier[:k_tr])
    ins = list(st.inspected[:k_tr])
    dirs = list(st.dir[:k_tr])
    reached_before = 0
    for k in range(k_tr):
        q = fr[k]
        new = fr[k + 1] if k + 1 < k_tr else (st.reached - reached_before - q if k + 1 == st.iterations else 0)
        new = max(new, 0)
        if dirs[k] == 0:
            total += 12 * q + 4 * ins[k] + min(n / 8, 4 * ins[k]) + (pb + 4) * new
            if k > 0 and dirs[k - 1] == 1:
                total += 2 * n / 8 + 4 * q
        else:
            u = max(nnz - (reached_before + q), 0)
            total += 4 * n / 8 + 8 * u + 4 * ins[k] + pb * new
        reached_before += q
    if st.iterations > 64:
        # untraced iterations are push iterations (push-only kernel); use totals
        q_rest = st.reached - sum(fr)
        ins_rest = st.edges_inspected - sum(ins)
        total += 12 * q_rest + 8 * ins_rest + (pb + 4) * q_rest
    return float(total)


# ------------------------------------------------------------------ CPU oracle

def cpu_info():
    """Host CPU model and the cores this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return model, os.cpu_count() or 1, avail


def cpu_threads():
    # the GPU machines give one GPU a 16-core share of the host, whatever
    # os.cpu_count() reports
    return max(1, min(16, cpu_info()[2]))


def cpu_serial(fn, queries, warmup=1):
    """Mode (a): one core, one query at a time.  fn(q) -> traversed edges.
    Returns (per-query seconds, edges)."""
    for q in queries[:warmup]:
        fn(q)
    secs, edges = [], []
    for q in queries:
        t0 = time.perf_counter()
        e = fn(q)
        secs.append(time.perf_counter() - t0)
        edges.append(e)
    return secs, edges


def cpu_parallel(fn, queries, threads, warmup=True):
    """Mode (b): every host core runs independent serial queries (one
    query per thread at a time; the oracle is C called through ctypes,
    which releases the GIL).  Returns (wall seconds, edges)."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=threads) as ex:
        if warmup:
            list(ex.map(fn, queries[:threads]))  # one query per thread
        t0 = time.perf_counter()
        edges = list(ex.map(fn, queries))
        wall = time.perf_counter() - t0
    return wall, edges


def cpu_record(kind, fn, queries_serial, queries_parallel, what, extra=None, par_warmup=True):
    """The oracle timed on the host in both modes of the CPU-baseline plan.
    extra: optional (seconds, edges) of further serial queries counted in
    the one-core value."""
    model, nproc, avail = cpu_info()
    thr = cpu_threads()
    secs, edges = cpu_serial(fn, queries_serial)
    if extra is not None:
        secs = secs + [extra[0]]
        edges = edges + [extra[1]]
    wall, pedges = cpu_parallel(fn, queries_parallel, thr, par_warmup)
    gteps1 = sum(edges) / sum(secs) / 1e9
    return {
        "value": round(gteps1, 4), "unit": "GTEPS", "cores": 1, "kind": "oracle",
        "sample": f"{kind} (oracle), one core: {len(queries_serial)} {what} one at a time after "
                  f"one warm-up query, {sum(secs):.1f}s",
        "ms_per_query_p50": round(float(np.percentile(secs, 50)) * 1e3, 2),
        "all_cores": {"queries_per_s": round(len(queries_parallel) / wall, 2),
                      "gteps": round(sum(pedges) / wall / 1e9, 4), "threads": thr,
                      "queries": len(queries_parallel), "wall_s": round(wall, 2),
                      "sample": f"{len(queries_parallel)} independent {kind} queries, one per "
                                f"thread at a time on {thr} threads"},
        "cpu_model": model, "nproc": nproc, "cores_available": avail,
    }


# ------------------------------------------------------- side measurements

def _ev():
    import torch
    return torch.cuda.Event(enable_timing=True)


def sssp_alg_bytes(st, n, nwords):
    """SSSP bytes from the device statistics: init 8n + n/8; per iteration
    16|F| (frontier id, 2 offsets, dist of u) + 12 per inspected edge (col,
    weight, dist of v) + 4|F'|."""
    total = 8 * n + nwords * 8
    k_tr = min(st.iterations, 64)
    fr = list(st.frontier[:k_tr])
    ins = list(st.inspected[:k_tr])
    for k in range(k_tr):
        nxt = fr[k + 1] if k + 1 < k_tr else 0
        total += 16 * fr[k] + 12 * ins[k] + 4 * nxt
    if st.iterations > 64:
        total += 12 * (st.edges_inspected - sum(ins))
    return float(total)


def side_sssp(fg, torch, off, col, srcs, stream, cpu):
    """C3a: SSSP on R-MAT 22 with uint32 weights in [1, 64] from the first 16
    of the DOBFS sources, one at a time."""
    import synth
    w = synth.weights(off, col)
    g = fg.Graph(off, col, weights=w, symmetric=True, validate=False)
    n = g.n
    dist = torch.empty(n, dtype=torch.int32, device="cuda")
    par = torch.empty(n, dtype=torch.int32, device="cuda")
    ws = g.workspace(fg.FG_PRIM_SSSP)
    st = fg.new_stats()
    deg = torch.diff(g.off)
    srcs = [int(x) for x in srcs[:16]]
    m_comp = []
    for s in srcs:
        fg.sssp_into(g, s, dist, par, ws=ws, stats=st, stream=stream)
        torch.cuda.synchronize()
        m_comp.append(int(deg[dist != -1].sum().item()))
    lat, byts = [], []
    for s in srcs:
        a, b = _ev(), _ev()
        a.record(stream)
        fg.sssp_into(g, s, dist, par, ws=ws, stats=st, stream=stream)
        b.record(stream)
        torch.cuda.synchronize()
        lat.append(a.elapsed_time(b))
        byts.append(sssp_alg_bytes(fg.read_stats(st), n, (n + 63) // 64))
    ms = float(np.mean(lat))
    gbs = float(np.mean(byts)) / (ms * 1e-3) / 1e9
    out = {
        "workload": "SSSP rmat22 ef16, uint32 weights in [1,64], first 16 of the 64 sources, one at a time",
        "ms_per_source": round(ms, 4), "ms_p50": round(float(np.percentile(lat, 50)), 4),
        "ms_p99": round(float(np.percentile(lat, 99)), 4),
        "gteps": round(sum(m_comp) / (sum(lat) * 1e-3) / 1e9, 3),
        "roofline": {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 5),
                     "alg_bytes_per_launch": round(float(np.mean(byts))),
                     **side_traffic("sssp", ms * 1e-3)},
    }
    if cpu:
        import oracle
        orc = oracle.oracle()
        deg_np = np.diff(off)

        def dij(s_):
            d = orc.dijkstra(off, col, w, int(s_))[0]
            return int(deg_np[d != 0xFFFFFFFF].sum())

        out["cpu_baseline"] = cpu_record("binary-heap Dijkstra", dij, srcs[:2], srcs,
                                         "of the 16 sources", par_warmup=False)
    g.close()
    return out


class _ShareGraph:
    """The share's local graph as an fg.bfs_into target."""

    def __init__(self, fg, torch, share):
        self.handle = share.graph_handle
        self.n = share.n_total
        nb = int(fg.lib().fg_workspace_bytes(self.handle, fg.FG_PRIM_BFS, 0))
        self.ws = torch.zeros(max(nb, 256), dtype=torch.uint8, device="cuda")

    def workspace(self, prim):
        return self.ws


def side_package(fg, torch, stream, cpu, off, col):
    """C3b: the package step (split + gather per peer) on one GPU's quarter
    share of R-MAT 24 (random 4-way owners, duplicate-1-hop), timed on the
    output frontiers of a push BFS over the local graph from local vertex 0."""
    import ctypes
    import synth
    t0 = time.time()
    owner = synth.owners(len(off) - 1, 4)
    sh = fg.Share(off, col, owner, 4, 0)
    print(f"[bench] rmat24 quarter share built in {time.time() - t0:.1f}s: "
          f"n_local={sh.n_local} n_total={sh.n_total} m_local={sh.m_local}",
          file=sys.stderr, flush=True)
    lg = _ShareGraph(fg, torch, sh)
    nt = sh.n_total
    depth = torch.empty(nt, dtype=torch.int32, device="cuda")
    parent = torch.empty(nt, dtype=torch.int32, device="cuda")
    fg.bfs_into(lg, 0, depth, parent, fg.bfs_opts(mode=fg.FG_MODE_PUSH), ws=lg.ws, stream=stream)
    torch.cuda.synchronize()
    levels = int(depth.max().item())
    fronts = [torch.nonzero(depth == k + 1).flatten().to(torch.int32) for k in range(levels)]
    cap = max(int(f.numel()) for f in fronts)
    P = 4
    ids = torch.empty(P * cap, dtype=torch.int32, device="cuda")
    dep = torch.empty(P * cap, dtype=torch.int32, device="cuda")
    par = torch.empty(P * cap, dtype=torch.int32, device="cuda")
    counts = torch.zeros(P, dtype=torch.int32, device="cuda")
    local = torch.empty(cap, dtype=torch.int32, device="cuda")
    lc = torch.zeros(1, dtype=torch.int32, device="cuda")
    pws = sh.workspace(cap)
    bufs = fg.PeerBufs(ids.data_ptr(), dep.data_ptr(), par.data_ptr(), counts.data_ptr(),
                       local.data_ptr(), lc.data_ptr(), cap)
    L = fg.lib()
    sp = fg._stream(stream)

    def run_all(evs):
        for k, f in enumerate(fronts):
            if evs:
                evs[k][0].record(stream)
            fg._check(L.fg_package(sh.handle, fg._ptr(f), int(f.numel()), None, fg._ptr(depth),
                                   fg._ptr(parent), ctypes.byref(bufs), fg._ptr(pws),
                                   pws.numel(), sp))
            if evs:
                evs[k][1].record(stream)

    run_all(None)
    evs = [(_ev(), _ev()) for _ in fronts]
    run_all(evs)
    torch.cuda.synchronize()
    us = [a.elapsed_time(b) * 1e3 for a, b in evs]
    nv = [int(f.numel()) for f in fronts]
    big = int(np.argmax(nv))
    bpv = 4 + 1 + 4 + 4 + 4 + 4 + 4 + 4  # id, owner, conv, depth, parent in; id, depth, parent out
    gbs_big = nv[big] * bpv / (us[big] * 1e-6) / 1e9
    out = {
        "workload": "package step on share 0 of 4 (rmat24 ef16, random owners, duplicate-1-hop), "
                    "output frontiers of a push BFS on the local graph from local vertex 0, with parents",
        "n_local": sh.n_local, "n_total": nt, "m_local": sh.m_local, "iterations": levels,
        "frontier_sizes": nv, "us_per_iteration": [round(x, 2) for x in us],
        "us_total": round(sum(us), 2),
        "vertices_per_s": round(sum(nv) / (sum(us) * 1e-6), 1),
        "roofline": {"bound": "hbm", "achieved": round(gbs_big, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(gbs_big / HBM_PEAK_GBS, 5),
                     "note": f"largest iteration ({nv[big]} vertices), {bpv} B per vertex"},
    }
    if cpu:
        import oracle
        orc = oracle.oracle()
        own, conv, l2g = sh.tables()
        fr = fronts[big].cpu().numpy()
        dh = depth.cpu().numpy()
        ph = parent.cpu().numpy()
        t0 = time.perf_counter()
        orc.package(fr, sh.n_local, own, conv, dh, ph, l2g, 4)
        t = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(len(fr) / t, 1), "unit": "vertices/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"oracle package of the largest iteration ({len(fr)} vertices)"}
    sh.close()
    return out


def side_batched(fg, torch, stream, do_kw, cpu):
    """C4: 64 sources per launch on R-MAT 23 and on a 2048 x 2048 grid,
    against the one-source-at-a-time path on the same GPU."""
    import synth
    from paper_1504_04804_amd import autotune
    res = {}
    for name in ("rmat23", "grid2048"):
        if name == "rmat23":
            off, col = synth.rmat_csr(23, EDGE_FACTOR)
            srcs = [int(x) for x in synth.sources(off, 64)]
            n_single = 64
        else:
            off, col = synth.grid_csr(2048, 2048)
            srcs = [int(x) for x in synth.sources(off, 64)]
            n_single = 8
        g = fg.Graph(off, col, symmetric=True, validate=False)
        mo, mkw = autotune.workload_opts(f"{name}_msbfs", g)
        # the one-at-a-time path with its own tuned options: DOBFS on R-MAT,
        # push BFS (the asynchronous team where it wins) on the grid
        o1, o1kw = autotune.workload_opts("rmat23_dobfs" if name == "rmat23" else
                                          "grid2048_push", g)
        b = fg.MsBatch(g, 64, mo)
        bt, work = [], []
        for rep in range(3):
            for lane, s in enumerate(srcs):
                if rep:
                    b.release(lane)
                b.admit(lane, s)
            c0 = b.counts(stream=stream)
            e0, e1 = _ev(), _ev()
            e0.record(stream)
            b.step(1 << 30, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            bt.append(e0.elapsed_time(e1))
            c1 = b.counts(stream=stream)
            work.append((c1[0] - c0[0], c1[1] - c0[1]))
        done, _ = b.poll()
        # the 64 depth rows; a vertex is in some lane's frontier once per
        # distinct depth it has over the lanes (its active (vertex, level)
        # pairs in a push-only run of the batch)
        rows = torch.stack([b.read(lane, stream=stream) for lane in range(64)])
        reached = int((rows >= 0).sum().item())
        srt = torch.sort(rows, dim=0).values
        distinct = (srt[:1] >= 0).to(torch.int64).squeeze(0) + \
            ((srt[1:] != srt[:-1]) & (srt[1:] >= 0)).to(torch.int64).sum(dim=0)
        deg64 = torch.diff(g.off).to(torch.int64)
        act_v = int(distinct.sum().item())
        act_e = int((distinct * deg64).sum().item())
        del rows, srt, distinct, deg64
        b.close()
        d = torch.empty(g.n, dtype=torch.int32, device="cuda")
        ws = g.workspace(fg.FG_PRIM_BFS)
        fg.bfs_into(g, srcs[0], d, None, o1, ws=ws, stream=stream)
        st = []
        for s in srcs[:n_single]:
            best = None
            for _ in range(2):
                e0, e1 = _ev(), _ev()
                e0.record(stream)
                fg.bfs_into(g, s, d, None, o1, ws=ws, stream=stream)
                e1.record(stream)
                torch.cuda.synchronize()
                t = e0.elapsed_time(e1)
                best = t if best is None else min(best, t)
            st.append(best)
        # the same statistic for both paths: the fastest of the repeats of
        # each query (the whole batch / each single source), averaged over
        # the single sources
        ms_b = float(min(bt))
        t1 = float(np.mean(st))
        ed, vv = work[int(np.argmin(bt))]
        # per adjacency entry read: column + the neighbour's lane word; per
        # vertex visit: visit + two frontier words; per lane: the depth row
        # filled at admission, plus one depth store per reached vertex.
        # Counted twice: over the work the batch did (its pull levels read
        # every unfinished vertex's lane words, much of it from cache) and
        # over a push-only run of the same batch (each active vertex and its
        # row once per level); the algorithmic bytes are the smaller.
        fixed = 4.0 * 64 * g.n + 4.0 * reached
        alg_done = 12.0 * ed + 24.0 * vv + fixed
        alg_push = 12.0 * act_e + 24.0 * act_v + fixed
        alg = min(alg_done, alg_push)
        gbs = alg / (ms_b * 1e-3) / 1e9
        # 64 queries arriving together: batched, all finish at the batch end;
        # one at a time, query i finishes after i + 1 traversals (modelled
        # from the median single-run time, not measured)
        fifo_lat = [t1 * (i + 1) for i in range(64)]
        res[name] = {
            "n": g.n, "m": int(g.m), "queries": 64, "all_done": done == (1 << 64) - 1,
            "batched_ms": round(ms_b, 3), "batched_queries_per_s": round(64 / (ms_b * 1e-3), 1),
            "batched_latency_ms_p50": round(ms_b, 3), "batched_latency_ms_p99": round(ms_b, 3),
            "single_ms": round(t1, 4), "single_queries_per_s": round(1000.0 / t1, 1),
            "single_fifo_latency_ms_p50": round(float(np.percentile(fifo_lat, 50)), 3),
            "single_fifo_latency_ms_p99": round(float(np.percentile(fifo_lat, 99)), 3),
            "single_fifo_latency_note": "modelled: query i of 64 arriving together finishes "
                                        "after i + 1 median single runs",
            "statistic": f"fastest of {len(bt)} batched runs; single: fastest of 2 runs per "
                         f"source, mean over {len(st)} sources",
            "batch_options": mkw,
            "qps_ratio": round((64 / (ms_b * 1e-3)) / (1000.0 / t1), 2),
            "single_path": ("DOBFS" if name == "rmat23" else "push BFS") + " with tuned options",
            "single_options": o1kw,
            "roofline": {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 5),
                         "alg_bytes_per_launch": round(alg),
                         "alg_bytes_as_run": round(alg_done),
                         "alg_bytes_push_only": round(alg_push),
                         **side_traffic(f"c4_{name}", ms_b * 1e-3),
                         "note": "12 B per adjacency entry read + 24 B per vertex visit + "
                                 "4 B per (lane, vertex) depth fill + 4 B per depth found, "
                                 "the smaller of the count over the work done and over a "
                                 "push-only run (active vertex-levels from the lanes' depths)"},
        }
        g.close()
        if cpu:
            import oracle
            orc = oracle.oracle()
            wall, _ = cpu_parallel(lambda s_: orc.bfs(off, col, s_)[3], srcs, cpu_threads())
            res[name]["cpu_all_cores"] = {
                "queries_per_s": round(len(srcs) / wall, 2), "threads": cpu_threads(),
                "kind": "oracle", "sample": f"the same {len(srcs)} queries, FIFO-queue BFS, "
                                            "one per thread at a time"}
    return res


def side_batched_sssp(fg, torch, stream, rmat22, cpu):
    """64 SSSP queries per launch (fg_mssp_*) on R-MAT 22 and a 2048 x 2048
    grid (weights in [1, 64]) against fg_sssp one source at a time."""
    import synth
    res = {}
    for name in ("rmat22", "grid2048"):
        off, col = rmat22 if name == "rmat22" else synth.grid_csr(2048, 2048)
        w = synth.weights(off, col)
        g = fg.Graph(off, col, weights=w, symmetric=True, validate=False)
        srcs = [int(x) for x in synth.sources(off, 64, seed=31)]
        b = fg.MsspBatch(g, 64, stream=stream)
        bt, byts = [], []
        for rep in range(2):
            for lane, s_ in enumerate(srcs):
                if rep:
                    b.release(lane)
                b.admit(lane, s_)
            e_0, el_0 = b.counts(stream=stream)
            e0, e1 = _ev(), _ev()
            e0.record(stream)
            b.step(1 << 30, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            bt.append(e0.elapsed_time(e1))
            e_1, el_1 = b.counts(stream=stream)
            # per edge visit: column + weight; per (edge, lane): distance read
            # + atomic; per (vertex, lane) relaxed: its own distance (in el)
            byts.append(8.0 * (e_1 - e_0) + 8.0 * (el_1 - el_0))
        done, _ = b.poll(stream=stream)
        b.close()
        d = torch.empty(g.n, dtype=torch.int32, device="cuda")
        ws = g.workspace(fg.FG_PRIM_SSSP)
        fg.sssp_into(g, srcs[0], d, None, ws=ws, stream=stream)
        st = []
        for s_ in srcs[:8]:
            best = None
            for _ in range(2):
                e0, e1 = _ev(), _ev()
                e0.record(stream)
                fg.sssp_into(g, s_, d, None, ws=ws, stream=stream)
                e1.record(stream)
                torch.cuda.synchronize()
                t = e0.elapsed_time(e1)
                best = t if best is None else min(best, t)
            st.append(best)
        # the same statistic for both paths: the fastest of the repeats of
        # each query (the whole batch / each single source), averaged over
        # the single sources
        ms_b = float(min(bt))
        t1 = float(np.mean(st))
        gbs = byts[int(np.argmin(bt))] / (ms_b * 1e-3) / 1e9
        res[name] = {
            "n": g.n, "m": int(g.m), "queries": 64, "all_done": done == (1 << 64) - 1,
            "batched_ms": round(ms_b, 3), "batched_queries_per_s": round(64 / (ms_b * 1e-3), 1),
            "single_ms": round(t1, 3), "single_queries_per_s": round(1000.0 / t1, 1),
            "qps_ratio": round((64 / (ms_b * 1e-3)) / (1000.0 / t1), 2),
            "statistic": f"fastest of {len(bt)} batched runs; single: fastest of 2 runs per "
                         f"source, mean over {len(st)} sources",
            "roofline": {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 5),
                         "alg_bytes_per_launch": round(float(byts[int(np.argmin(bt))])),
                         **side_traffic(f"mssp_{name}", ms_b * 1e-3),
                         "note": "8 B per edge visit + 8 B per (edge, lane) relaxation"},
        }
        g.close()
        if cpu:
            import oracle
            orc = oracle.oracle()
            thr = cpu_threads()
            wall, _ = cpu_parallel(lambda s_: int(orc.dijkstra(off, col, w, s_)[0][0]),
                                   srcs[:thr], thr, warmup=False)
            res[name]["cpu_all_cores"] = {
                "queries_per_s": round(thr / wall, 3), "threads": thr, "kind": "oracle",
                "sample": f"the first {thr} of the queries, binary-heap Dijkstra, one per thread"}
    return res


# ------------------------------------------- widened rows: dup-all, CC, PR

def dup_alg_bytes(sts, n, nparts, hosted_nz):
    """Algorithmic bytes of one duplicate-all DOBFS traversal over all
    partitions, from their traces (identical dir / frontier, per-partition
    inspected).  Per iteration and partition:
      forward : 12 B per hosted frontier vertex (id, 2 offsets), 4 B per
                row entry read, the visited word of each target (at most
                n/8), 12 B per vertex it discovers (depth, parent, message
                entry); the message (4 B per id) is read once and written
                to each of the nparts - 1 peers; the combine reads each
                received id and labels the new ones (4 B);
      backward: nonzero mask + visited (2 n/8), 8 B per hosted candidate,
                4 B per row entry read, the visited bitmap as frontier (n/8),
                8 B per discovered vertex, the n/8 message written and copied
                to every peer; the combine reads the nparts messages and
                writes visited + frontier bitmaps (n/8 each) and 4 B per
                vertex labelled from a message."""
    st0 = sts[0]
    k = min(st0.iterations, 64)
    dirs = list(st0.dir[:k])
    fr = list(st0.frontier[:k])
    total = float(nparts * (4 * n + 4 * n + n / 8))  # seeds: depth, parent, visited
    labelled = 0
    for i in range(k):
        new = fr[i + 1] if i + 1 < k else 0
        insp = [st.inspected[i] for st in sts]
        if dirs[i] == 0:
            for p in range(nparts):
                total += 12 * fr[i] / nparts + 4 * insp[p] + min(n / 8, 4 * insp[p])
            total += 12 * new + 4 * new * (nparts - 1) * 2 + 4 * new * (nparts - 1)
        else:
            u = max(sum(hosted_nz) - labelled - fr[i], 0)
            for p in range(nparts):
                total += 3 * n / 8 + 4 * insp[p]
            total += 8 * u + 8 * new
            total += nparts * (n / 8) * (nparts - 1) * 2          # sends
            total += nparts * ((nparts + 2) * n / 8) + 4 * new * (nparts - 1)
        labelled += fr[i]
    return total


def side_dupall(fg, torch, stream, off, col, srcs, cpu):
    """Duplicate-all + broadcast DOBFS (Alg. 2) on R-MAT 22 over 4 random
    owners, the 4 partitions emulated on this GPU, 16 of the 64 sources with
    the DOBFS workload's thresholds."""
    import synth
    from paper_1504_04804_amd import autotune
    P = 4
    owner = synth.owners(len(off) - 1, P)
    g0 = fg.Graph(off, col, symmetric=True, validate=False)
    _, kw = autotune.workload_opts("rmat22_dobfs", g0)
    g0.close()
    t0 = time.time()
    dup = fg.DupBfs(off, col, owner, P, do_a=kw["do_a"], do_b=kw["do_b"], stream=stream)
    build_s = time.time() - t0
    n = len(off) - 1
    deg = np.diff(off)
    hosted_nz = [int(((owner == p) & (deg > 0)).sum()) for p in range(P)]
    srcs = [int(x) for x in srcs[:16]]
    lat, byts, m_comp, iters = [], [], [], []
    degd = torch.from_numpy(deg).to("cuda")
    dup.run(srcs[0], stream=stream)
    for s_ in srcs:
        a, b = _ev(), _ev()
        a.record(stream)
        dup.run(s_, stream=stream)
        b.record(stream)
        torch.cuda.synchronize()
        lat.append(a.elapsed_time(b))
        sts = [dup.read_stats(p) for p in range(P)]
        assert all(st.status == 0 for st in sts)
        byts.append(dup_alg_bytes(sts, n, P, hosted_nz))
        d0 = dup.depth[0]
        m_comp.append(int(degd[d0 >= 0].sum().item()))
        iters.append(sts[0].iterations)
    ms = float(np.mean(lat))
    gbs = float(np.mean(byts)) / (ms * 1e-3) / 1e9
    info = [dup.info(p) for p in range(P)]
    out = {
        "workload": "duplicate-all + broadcast DOBFS, rmat22 ef16, 4 random owners emulated on one "
                    "GPU (each partition's step, broadcast copies and combine run back to back), "
                    f"16 of the 64 sources, do_a={kw['do_a'][0]}/{kw['do_a'][1]} "
                    f"do_b={kw['do_b'][0]}/{kw['do_b'][1]}",
        "partitions": P, "m_local": [int(i.m_local) for i in info],
        "build_s": round(build_s, 2),
        "ms_per_traversal": round(ms, 4), "ms_p50": round(float(np.percentile(lat, 50)), 4),
        "iterations_mean": round(float(np.mean(iters)), 2),
        "us_per_iteration_all_partitions": round(ms * 1e3 / float(np.mean(iters)), 2),
        "gteps_emulated": round(sum(m_comp) / (sum(lat) * 1e-3) / 1e9, 3),
        "roofline": {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 5),
                     "alg_bytes_per_traversal": round(float(np.mean(byts))),
                     "note": "all partitions' step, send and combine kernels and the host's "
                             "stop-flag reads in the timed region"},
    }
    dup.close()
    if cpu:
        import oracle
        orc = oracle.oracle()
        t0 = time.perf_counter()
        orc.dobfs_dupall(off, col, owner, P, srcs[0], kw["do_a"], kw["do_b"])
        t = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(m_comp[0] / t / 1e9, 4), "unit": "GTEPS", "cores": 1,
                               "kind": "oracle", "sample": f"oracle duplicate-all emulation "
                                                           f"from the first source, {t:.1f}s"}
    return out


def side_cc(fg, torch, stream, graphs, cpu):
    """Connected components (min-id labels) on R-MAT 22 and the 4096 x 4096
    grid."""
    res = {}
    for name, (off, col) in graphs.items():
        g = fg.Graph(off, col, symmetric=True, validate=False)
        n, m = g.n, int(g.m)
        label = torch.empty(n, dtype=torch.int32, device="cuda")
        comps = torch.zeros(1, dtype=torch.int64, device="cuda")
        fg.cc_into(g, label, comps, stream=stream)
        lat = []
        for _ in range(5):
            a, b = _ev(), _ev()
            a.record(stream)
            fg.cc_into(g, label, comps, stream=stream)
            b.record(stream)
            torch.cuda.synchronize()
            lat.append(a.elapsed_time(b))
        ms = float(np.median(lat))
        # column indices once, offsets once, first neighbour, label written
        # at init, read and written at compress
        alg = 4.0 * m + 20.0 * n
        gbs = alg / (ms * 1e-3) / 1e9
        res[name] = {"n": n, "m": m, "components": int(comps.item()),
                     "ms": round(ms, 4), "statistic": "median of 5",
                     "gteps": round(m / (ms * 1e-3) / 1e9, 3),
                     "roofline": {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS,
                                  "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 5),
                                  "alg_bytes_per_call": round(alg),
                                  "note": "4 B per CSR entry + 20 B per vertex"}}
        g.close()
        if cpu:
            import oracle
            orc = oracle.oracle()
            t0 = time.perf_counter()
            orc.cc(off, col)
            t = time.perf_counter() - t0
            res[name]["cpu_baseline"] = {"value": round(m / t / 1e9, 4), "unit": "GTEPS",
                                         "cores": 1, "kind": "oracle",
                                         "sample": f"oracle BFS labelling, one call, {t:.1f}s"}
    return res


def side_pagerank(fg, torch, stream, off, col, cpu):
    """PageRank, 20 fp64 power iterations (damping 0.85) on R-MAT 22."""
    g = fg.Graph(off, col, symmetric=True, validate=False)
    n, m = g.n, int(g.m)
    rank = torch.empty(n, dtype=torch.float64, device="cuda")
    ws = g.workspace(fg.FG_PRIM_PR)
    st = fg.new_stats()
    iters = 20
    fg.pagerank_into(g, rank, 0.85, 0.0, iters, ws=ws, stats=st, stream=stream)
    lat = []
    for _ in range(3):
        a, b = _ev(), _ev()
        a.record(stream)
        fg.pagerank_into(g, rank, 0.85, 0.0, iters, ws=ws, stats=st, stream=stream)
        b.record(stream)
        torch.cuda.synchronize()
        lat.append(a.elapsed_time(b))
    ms = float(np.median(lat))
    per_it = ms / iters
    # per iteration: column index (4) and neighbour contribution (8) per CSR
    # entry; 2 offsets, rank read + written, contribution written per vertex
    alg = 12.0 * m + 32.0 * n
    gbs = alg / (per_it * 1e-3) / 1e9
    out = {"workload": "PageRank rmat22 ef16, damping 0.85, 20 iterations (no early stop), fp64",
           "n": n, "m": m, "ms_total": round(ms, 4), "ms_per_iteration": round(per_it, 4),
           "statistic": "median of 3",
           "gteps_per_iteration": round(m / (per_it * 1e-3) / 1e9, 3),
           "roofline": {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 5),
                        "alg_bytes_per_iteration": round(alg),
                        **side_traffic("pagerank_iter", per_it * 1e-3),
                        "note": "12 B per CSR entry + 32 B per vertex per iteration"}}
    g.close()
    if cpu:
        import oracle
        orc = oracle.oracle()
        t0 = time.perf_counter()
        orc.pagerank(off, col, 0.85, 0.0, 2)
        t = (time.perf_counter() - t0) / 2
        out["cpu_baseline"] = {"value": round(m / t / 1e9, 4), "unit": "GTEPS per iteration",
                               "cores": 1, "kind": "oracle",
                               "sample": f"oracle power iteration, 2 iterations, {2 * t:.1f}s"}
    return out


SERVE_QPS = (25, 50, 100, 150, 200, 250, 300)
SERVE_SECONDS = 8.0          # arrivals span about this long per load ...
SERVE_NREQ = (300, 1600)     # ... with at least / at most this many requests
SERVE_BUDGET = 16 << 30
SERVE_P99_TARGETS_MS = (250, 500, 1000)
SERVE_SUSTAIN = 0.95         # a load counts as sustained when achieved >= this x arrived


def serving_graphs(fg, cpu_graphs):
    """The 8 resident graphs of the serving workload, with weights."""
    import synth
    graphs, specs, srcs = {}, {}, {}
    for name, maker in (("rmat16", lambda: synth.rmat_csr(16, EDGE_FACTOR)),
                        ("rmat18", lambda: synth.rmat_csr(18, EDGE_FACTOR)),
                        ("rmat20", lambda: synth.rmat_csr(20, EDGE_FACTOR)),
                        ("rmat22", lambda: cpu_graphs["rmat22"]),
                        ("rmat24", lambda: cpu_graphs["rmat24"]),
                        ("grid1024", lambda: synth.grid_csr(1024, 1024)),
                        ("grid2048", lambda: synth.grid_csr(2048, 2048)),
                        ("grid4096", lambda: cpu_graphs["grid4096"])):
        off, col = maker()
        w = synth.weights(off, col)
        graphs[name] = fg.Graph(off, col, weights=w, symmetric=True, validate=False)
        specs[name] = (off, True)
        srcs[name] = synth.sources(off, 8, seed=77)
    return graphs, specs, srcs


def max_sustained_at(sweep, path, target):
    """The highest swept load that `path` sustained (achieved q/s at least
    SERVE_SUSTAIN x the rate at which that replay's requests arrived: a
    Poisson sample's own rate, not the nominal one) with p99 latency within
    `target` ms; returns (offered, achieved) or (None, None)."""
    ok = [(row["qps_offered"], row[path]["qps"]) for row in sweep
          if row[path]["p99_ms"] <= target and row[path]["qps"] >= SERVE_SUSTAIN * row["qps_arrived"]]
    return max(ok) if ok else (None, None)


def level_table(recs):
    """Per-level device time of the multi-source DOBFS launch, by level
    index over the sources that reach it (from each record's clock stamps):
    mean / max microseconds, share of pull levels, mean frontier and entries
    read; `init_us` is the gap from one traversal's last level to the next
    one's first stamp (outputs and bitmap cleared, source seeded)."""
    khz = recs[0].clock_khz
    rows, init = {}, []
    for j, st in enumerate(recs):
        us = st.iteration_us()
        dirs, fr, ins = st.trace()
        if j:
            prev = recs[j - 1]
            init.append((st.t_start - prev.t_end[min(prev.iterations, 64) - 1]) * 1000.0 / khz)
        for k, row in enumerate(zip(us, dirs, fr, ins)):
            rows.setdefault(k, []).append(row)
    table = []
    for k in sorted(rows):
        a = np.array(rows[k], dtype=np.float64)
        table.append({"level": k, "sources": len(a), "us_mean": round(float(a[:, 0].mean()), 2),
                      "us_max": round(float(a[:, 0].max()), 2),
                      "pull_share": round(float(a[:, 1].mean()), 3),
                      "frontier_mean": round(float(a[:, 2].mean()), 1),
                      "inspected_mean": round(float(a[:, 3].mean()), 1)})
    per_src = sum(r["us_mean"] * r["sources"] for r in table) / len(recs)
    return {"init_us_mean": round(float(np.mean(init)), 2) if init else None,
            "levels_us_per_source": round(per_src, 2), "table": table}


def side_overhead(fg, torch, stream):
    """Per-iteration overhead (the paper's l, Sec. V): BFS on a path, one
    vertex and one edge per level, so a level's time is all overhead.  The
    persistent kernel (one workgroup runs such levels from LDS), the
    asynchronous team (one member) and the unfused host loop of advance +
    filter launches (the paper's baseline structure)."""
    import synth
    res = {}
    for what, n, opts in (("persistent push", 1 << 16, fg.bfs_opts(mode=fg.FG_MODE_PUSH)),
                          ("asynchronous push, 1 member, K = 128", 1 << 16,
                           fg.bfs_opts(mode=fg.FG_MODE_PUSH, async_levels=128, team_blocks=1)),
                          ("unfused host loop", 1 << 12,
                           fg.bfs_opts(mode=fg.FG_MODE_PUSH_UNFUSED))):
        off, col = synth.grid_csr(1, n)
        g = fg.Graph(off, col, symmetric=True, validate=False)
        depth = torch.empty(n, dtype=torch.int32, device="cuda")
        parent = torch.empty(n, dtype=torch.int32, device="cuda")
        ws = g.workspace(fg.FG_PRIM_BFS_UNFUSED if opts.mode == fg.FG_MODE_PUSH_UNFUSED
                         else fg.FG_PRIM_BFS)
        st = fg.new_stats("cuda")
        ts = []
        for rep in range(3):
            a, b = _ev(), _ev()
            a.record(stream)
            fg.bfs_into(g, 0, depth, parent, opts, ws=ws, stats=st, stream=stream)
            b.record(stream)
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        r = fg.read_stats(st)
        ok = r.status == 0 and r.iterations == n and int(depth[-1].item()) == n - 1
        ms = float(min(ts))
        res[what] = {"vertices": n, "levels": int(r.iterations), "ms": round(ms, 3),
                     "us_per_level": round(ms * 1e3 / max(r.iterations, 1), 3), "ok": bool(ok)}
        del ws, depth, parent
        g.close()
    res["note"] = ("path graph 0-1-...-(n-1) from vertex 0: every level has one vertex and "
                   "one new edge; fastest of 3 runs, launch included")
    return res


def side_serving(fg, torch, cpu_graphs):
    """C5: Poisson streams of BFS / SSSP queries over 8 resident graphs of
    mixed size at a sweep of offered loads, served with HBM-budget admission
    and continuous batching, against the one-at-a-time path at the same
    offered load; the highest swept load each sustains under a p99 target."""
    from paper_1504_04804_amd import serve
    graphs, specs, srcs = serving_graphs(fg, cpu_graphs)
    t0 = time.time()
    costs = serve.calibrate(graphs, srcs)
    cal_s = time.time() - t0
    print(f"[bench] serving cost model calibrated in {cal_s:.1f}s", file=sys.stderr, flush=True)
    bfs_ws = {n: g.workspace(fg.FG_PRIM_BFS) for n, g in graphs.items()}
    sssp_ws = {n: g.workspace(fg.FG_PRIM_SSSP) for n, g in graphs.items()}
    sweep = []
    for qps in SERVE_QPS:
        nreq = int(min(max(qps * SERVE_SECONDS, SERVE_NREQ[0]), SERVE_NREQ[1]))
        reqs = serve.make_requests(specs, nreq, qps=float(qps), bfs_frac=0.8, seed=11)
        srv = serve.Server(graphs, hbm_budget=SERVE_BUDGET, policy="auto", costs=costs,
                           keep_results=False)
        done = serve.serve_stream(srv, reqs, time_limit=300)
        served = serve.latency_stats(done)
        nb = sum(1 for r in done if r.path == "batch")
        reqs2 = serve.make_requests(specs, nreq, qps=float(qps), bfs_frac=0.8, seed=11)
        done2 = serve.serve_fifo(graphs, reqs2, sssp_ws, bfs_ws=bfs_ws, time_limit=300,
                                 keep_results=False)
        fifo = serve.latency_stats(done2)
        arrived = (nreq - 1) / (reqs[-1].arrival - reqs[0].arrival)
        row = {"qps_offered": qps, "qps_arrived": round(arrived, 3), "requests": nreq,
               "served": {k: round(v, 3) for k, v in served.items()},
               "fifo": {k: round(v, 3) for k, v in fifo.items()},
               "served_batched_frac": round(nb / len(done), 3),
               "served_steps": srv.counts["steps"], "served_singles": srv.counts["singles"],
               "served_coruns": srv.counts["coruns"],
               "served_corun_list_queries": srv.counts["corun_list"],
               "served_evictions": srv.counts["evictions"],
               "hbm_resident_graphs_bytes": srv.resident_bytes,
               "hbm_workspace_peak_bytes": srv.peak_used,
               "hbm_total_peak_bytes": srv.resident_bytes + srv.peak_used}
        sweep.append(row)
        print(f"[bench] serving qps={qps} ({nreq} requests): served p50={served['p50_ms']:.1f} "
              f"p99={served['p99_ms']:.1f} qps={served['qps']:.1f} | fifo p50={fifo['p50_ms']:.1f} "
              f"p99={fifo['p99_ms']:.1f} qps={fifo['qps']:.1f}", file=sys.stderr, flush=True)
        srv.close()
        del srv
    at = {}
    for tgt in SERVE_P99_TARGETS_MS:
        (s_o, s_a), (f_o, f_a) = (max_sustained_at(sweep, "served", tgt),
                                  max_sustained_at(sweep, "fifo", tgt))
        at[f"p99<={tgt}ms"] = {"served_offered_qps": s_o, "served_achieved_qps": s_a,
                               "fifo_offered_qps": f_o, "fifo_achieved_qps": f_a,
                               "achieved_ratio": round(s_a / f_a, 2) if s_a and f_a else None}
    for g in graphs.values():
        g.close()
    return {
        "workload": f"Poisson arrivals for about {SERVE_SECONDS:.0f}s per load "
                    f"({SERVE_NREQ[0]}-{SERVE_NREQ[1]} requests), 80% BFS / 20% SSSP, uniform "
                    "over 8 resident graphs (rmat16/18/20/22/24 ef16, grids 1024^2/2048^2/4096^2, "
                    f"weights in [1,64]), HBM budget {SERVE_BUDGET >> 30} GiB for workspaces",
        "policy": "64-lane BFS and SSSP batches per graph with continuous admission; a cost "
                  "model (single run vs 1- and 8-lane batches, measured per graph and kind) "
                  "picks batch or single run when a batch is idle; oldest request first",
        "calibration_s": round(cal_s, 1),
        "cost_model_ms": {f"{n}/{'bfs' if k == serve.BFS else 'sssp'}": c.as_dict()
                          for (n, k), c in costs.items()},
        "sweep": sweep,
        "max_sustained_qps_at_p99": at,
        "sustained_rule": f"achieved q/s >= {SERVE_SUSTAIN} x the replay's arrival rate "
                          "(qps_arrived) and p99 within the target",
        "single_query_options": "the same for both paths: direction-optimizing BFS on the R-MAT "
                                "graphs, the asynchronous push team (64 levels, 64 workgroups) "
                                "on the grids, SSSP with defaults",
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU (the traversal of one GPU's share); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1504_04804_amd as fg
    from paper_1504_04804_amd import autotune
    import synth

    torch.cuda.set_device(0)
    dev = "cuda"
    if args.calibration_copy:
        a = torch.ones(128 << 20, dtype=torch.int32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    t0 = time.time()
    off, col = synth.rmat_csr(SCALE, EDGE_FACTOR)
    srcs = synth.sources(off, NSRC)
    goff, gcol = synth.grid_csr(GRID, GRID)
    print(f"[bench] inputs generated in {time.time() - t0:.1f}s: rmat{SCALE} m={len(col)}, "
          f"grid{GRID} m={len(gcol)}", file=sys.stderr, flush=True)
    g = fg.Graph(off, col, symmetric=True, validate=True)
    gg = fg.Graph(goff, gcol, symmetric=True, validate=True)
    n, ng = g.n, gg.n
    nnz = g.info().nonzero_degree
    depth = torch.empty(n, dtype=torch.int32, device=dev)
    parent = torch.empty(n, dtype=torch.int32, device=dev)
    gdepth = torch.empty(ng, dtype=torch.int32, device=dev)
    gparent = torch.empty(ng, dtype=torch.int32, device=dev)
    ws = g.workspace(fg.FG_PRIM_BFS)
    gws = gg.workspace(fg.FG_PRIM_BFS)
    stats = [fg.new_stats(dev) for _ in range(NSRC + 1)]
    srcs_dev = torch.tensor([int(s) for s in srcs], dtype=torch.int32, device=dev)
    mstats = fg.new_stats_many(NSRC, dev)
    o_do, do_kw = autotune.workload_opts("rmat22_dobfs", g)
    o_push, push_kw = autotune.workload_opts("grid4096_push", gg)
    # the list's options in the step: the same, with the tuned share of the
    # workgroups beside the grid query's team
    o_step, step_kw = autotune.workload_opts("rmat22_dobfs_corun", g)
    stream = torch.cuda.current_stream()

    # traversed edges per query (graph + source only), outside the timed region
    deg = torch.diff(g.off)
    gdeg = torch.diff(gg.off)
    m_comp = []
    for s in srcs:
        fg.bfs_into(g, int(s), depth, parent, o_do, ws=ws, stats=stats[0])
        m_comp.append(int(deg[depth >= 0].sum().item()))
    fg.bfs_into(gg, 0, gdepth, gparent, o_push, ws=gws, stats=stats[NSRC])
    m_grid = int(gdeg[gdepth >= 0].sum().item())
    edges_step = sum(m_comp) + m_grid

    def pair():
        return (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))

    def run_many(ev=None):
        if ev:
            ev[0].record(stream)
        fg.bfs_many_into(g, srcs_dev, depth, parent, o_do, ws=ws, stats=mstats, stream=stream)
        if ev:
            ev[1].record(stream)

    def run_grid(ev=None):
        if ev:
            ev[0].record(stream)
        fg.bfs_into(gg, 0, gdepth, gparent, o_push, ws=gws, stats=stats[NSRC], stream=stream)
        if ev:
            ev[1].record(stream)

    def step(ev=None):
        # the 64 sources one after another and, beside them in the same
        # launch, the grid query on its own team of workgroups (fg_bfs_corun)
        if ev:
            ev[0].record(stream)
        fg.bfs_corun_into(g, srcs_dev, depth, parent, o_step, ws, mstats, gg, 0, gdepth, gparent,
                          o_push, ws2=gws, stats2=stats[NSRC], stream=stream)
        if ev:
            ev[1].record(stream)

    # each part alone, and the two in sequence on one stream, outside the
    # timed region (the per-workload figures and the sequential step)
    alone = {"many": [], "grid": [], "seq": []}
    for rep in range(4):
        e_m, e_g, e_s = pair(), pair(), pair()
        run_many(e_m)
        run_grid(e_g)
        e_s[0].record(stream)
        run_many()
        run_grid()
        e_s[1].record(stream)
        torch.cuda.synchronize()
        if rep:
            for k, e in (("many", e_m), ("grid", e_g), ("seq", e_s)):
                alone[k].append(e[0].elapsed_time(e[1]))
    recs_alone = fg.read_stats_many(mstats, NSRC)
    stg_alone = fg.read_stats(stats[NSRC])

    for _ in range(args.warmup):
        step()
    step_events = [pair() for _ in range(args.steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record(stream)
    for it in range(args.steps):
        step(step_events[it])
    t_end.record(stream)
    torch.cuda.synchronize()
    total_ms = t_start.elapsed_time(t_end)
    ms_per_step = total_ms / args.steps
    lat_step = [e[0].elapsed_time(e[1]) for e in step_events]
    status_bad = 0

    # records of the last timed step (same sources every step)
    recs = fg.read_stats_many(mstats, NSRC)
    stg = fg.read_stats(stats[NSRC])
    status_bad += sum(st.status != 0 for st in recs) + (stg.status != 0)
    bytes_do = [bfs_alg_bytes(st, n, (n + 63) // 64, nnz) for st in recs]
    grid_bytes = float(bfs_alg_bytes(stg, ng, (ng + 63) // 64, gg.info().nonzero_degree))
    khz = recs[0].clock_khz

    def last_end(st):
        return st.t_end[min(st.iterations, 64) - 1]

    # per-source spans on the device clock, from one traversal's last level
    # to the next one's (the next source's init included), DOBFS alone
    ends = [last_end(st) for st in recs_alone]
    lat_do = [(ends[j] - ends[j - 1]) / khz for j in range(1, NSRC)]
    # spans of the two parts inside the timed step
    co_list_ms = (last_end(recs[-1]) - recs[0].t_start) / khz
    co_grid_ms = ((last_end(stg) - stg.t_start) / khz) if stg.iterations else None

    # the same 64 sources with one launch each (fg_bfs), outside the step,
    # for comparison
    sep = []
    for rep in range(2):
        evs = [(_ev(), _ev()) for _ in srcs]
        for (a, b), s in zip(evs, srcs):
            a.record(stream)
            fg.bfs_into(g, int(s), depth, parent, o_do, ws=ws, stats=stats[0], stream=stream)
            b.record(stream)
        torch.cuda.synchronize()
        if rep:
            sep = [a.elapsed_time(b) for a, b in evs]
    # leave the step's outputs in place for the oracle check below
    step()
    torch.cuda.synchronize()

    lat_many = alone["many"]
    lat_grid = alone["grid"]
    do_ms = float(np.mean(lat_many)) / NSRC
    grid_ms = float(np.mean(lat_grid))
    seq_ms = float(np.mean(alone["seq"]))
    do_bytes = float(np.mean(bytes_do))
    grid_name = "bfs_async" if push_kw.get("async_levels", 0) > 1 else "bfs_persistent<PUSH>"
    # the step is one launch (plus the grid query's per-vertex kernels around
    # it): the dominant kernel; the two parts alone for comparison
    kernels = {
        "bfs_corun<DO>": dict(ms=float(np.mean(lat_step)), bytes=do_bytes * NSRC + grid_bytes,
                              launches=1, traversals=NSRC + 1),
        "bfs_persistent<DO,many> (alone)": dict(ms=float(np.mean(lat_many)),
                                                bytes=do_bytes * NSRC, launches=1,
                                                traversals=NSRC),
        grid_name + " (alone)": dict(ms=grid_ms, bytes=grid_bytes, launches=1),
    }
    traffic_ok = _sources_sha(TRAFFIC_SOURCES) == TRAFFIC_SHA256
    for name, k in kernels.items():
        k["share_ms"] = k["ms"] * k["launches"]
        k["gbs"] = k["bytes"] / (k["ms"] * 1e-3) / 1e9
        k["frac"] = k["gbs"] / HBM_PEAK_GBS
        k["traffic"] = TRAFFIC_BYTES.get(name) if traffic_ok else None
    dom = "bfs_corun<DO>"
    dk = kernels[dom]
    traffic = kernels[dom]["traffic"]
    step_ms = ms_per_step
    value = edges_step / (step_ms * 1e-3) / 1e9

    out = {
        "metric": "BFS GTEPS (traversed edges / s) + % HBM roofline, 1 GPU",
        "value": round(value, 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic (seeded R-MAT and grid, generated on the host, resident in HBM)",
        "config": {
            "workload": f"DOBFS rmat{SCALE} ef{EDGE_FACTOR} x{NSRC} sources one at a time + "
                        f"push BFS grid {GRID}x{GRID} from vertex 0",
            "launch": "fg_bfs_corun: the sources one after another on all but the grid "
                      "query's team of workgroups, the grid query on that team, in one launch",
            "rmat_n": n, "rmat_m": int(g.m), "grid_n": ng, "grid_m": int(gg.m),
            "do_a": "%d/%d" % do_kw["do_a"], "do_b": "%d/%d" % do_kw["do_b"],
            "dobfs_options": {k: v for k, v in do_kw.items() if k not in ("do_a", "do_b")},
            "step_list_workgroups": step_kw.get("grid_blocks", 0) or None,
            "grid_options": {k: v for k, v in push_kw.items() if k not in ("do_a", "do_b")},
            "options_from": "paper_1504_04804_amd/tuned.json (autotuner)", "parents": True,
        },
        "roofline": {
            "kernel": dom,
            "bound": "hbm",
            "achieved": round(dk["gbs"], 2),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(dk["frac"], 5),
            "traffic": traffic,
            "avg_launch_ms": round(dk["ms"], 4),
            "alg_bytes_per_launch": round(dk["bytes"]),
            "note": "one step = one fg_bfs_corun call (events around it: the co-run launch "
                    "plus the grid query's per-vertex kernels before and after it); bytes = "
                    "the 64 traversals' + the grid traversal's algorithmic bytes",
        },
        "step": {
            "ms_corun": round(float(np.mean(lat_step)), 4),
            "ms_sequential": round(seq_ms, 4),
            "speedup_vs_sequential": round(seq_ms / float(np.mean(lat_step)), 3),
            "list_span_ms": round(co_list_ms, 4),
            "grid_span_ms": round(co_grid_ms, 4) if co_grid_ms is not None else None,
            "list_workgroups": recs[0].grid_blocks,
            "note": "sequential = fg_bfs_many then fg_bfs on one stream (measured outside the "
                    "timed region); spans on the device clock inside the last timed step: the "
                    "list's from its first start to its last level, the grid query's from its "
                    "start to its record (written after the launch ends)",
        },
        "kernels": {k: {kk: (round(vv, 5) if isinstance(vv, float) else vv)
                        for kk, vv in v.items()} for k, v in kernels.items()},
        "dobfs": {
            "launch": "the 64 sources one after another in one launch (fg_bfs_many), alone "
                      "on the GPU, outside the timed step",
            "ms_per_source": round(do_ms, 4),
            "ms_per_launch": round(float(np.mean(lat_many)), 4),
            "gteps_harmonic": round((NSRC - 1) / sum((l * 1e-3) / (mc / 1e9)
                                                     for l, mc in zip(lat_do, m_comp[1:])), 2),
            "ms_p50": round(float(np.percentile(lat_do, 50)), 4),
            "ms_p99": round(float(np.percentile(lat_do, 99)), 4),
            "latency_note": "per source on the device clock, from one traversal's last level "
                            "to the next one's (sources 2-64 of the launch)",
            "queries_per_s": round(1000.0 / do_ms, 1),
            "bytes_per_traversed_edge": round(do_bytes / (sum(m_comp) / len(m_comp)), 3),
            "levels": level_table(recs_alone),
            "separate_launches": {
                "ms_mean": round(float(np.mean(sep)), 4),
                "ms_p50": round(float(np.percentile(sep, 50)), 4),
                "ms_p99": round(float(np.percentile(sep, 99)), 4),
                "note": "one fg_bfs launch per source, events around each launch"},
        },
        "grid": {
            "ms": round(grid_ms, 3),
            "gteps": round(m_grid / (grid_ms * 1e-3) / 1e9, 3),
            "levels": stg_alone.iterations,
            "us_per_level": round(grid_ms * 1e3 / max(stg_alone.iterations, 1), 3),
            "note": "fg_bfs alone on the GPU (events around the call), outside the timed step",
        },
        "device_status_errors": status_bad,
        "timed_region_ms": round(total_ms, 3),
    }
    # batched queries (the same 64 sources on the same graph, one 64-lane
    # batched traversal), outside the step: queries/s and per-query latency
    b = fg.MsBatch(g, NSRC)
    bt = []
    for rep in range(3):
        for lane, s in enumerate(srcs):
            if rep:
                b.release(lane)
            b.admit(lane, int(s))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        b.step(1 << 20, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        bt.append(e0.elapsed_time(e1))
    done, _ = b.poll()
    ms_b = float(np.median(bt))
    out["batched"] = {
        "queries": NSRC, "ms_per_batch": round(ms_b, 3),
        "queries_per_s": round(NSRC / (ms_b * 1e-3), 1),
        "latency_ms_p50": round(ms_b, 3), "latency_ms_p99": round(float(np.max(bt)), 3),
        "all_done": done == (1 << NSRC) - 1,
        "vs_one_at_a_time_qps": round((NSRC / (ms_b * 1e-3)) / (1000.0 / do_ms), 2),
        "note": "64-lane batched BFS (depths only) over the same sources; every query of a batch "
                "completes at the batch end, so p50 = the batch time",
    }
    b.close()
    verified = None
    if not args.no_cpu:
        # CPU baseline: the oracle timed on the host on a sample of the same
        # queries.  Its answers for the last timed R-MAT source (whose
        # depths the step leaves in `depth`) and for the grid are compared
        # with the GPU's depths: a mismatch fails the run.
        import oracle
        orc = oracle.oracle()
        nsamp = max(1, min(args.cpu_sources, NSRC))
        t0 = time.perf_counter()
        g_want, _, _, mg = orc.bfs(goff, gcol, 0)
        tg = time.perf_counter() - t0
        last = int(srcs[-1])
        kept = {}

        def bfs_q(s_):
            d_, _, _, mc_ = orc.bfs(off, col, int(s_))
            if int(s_) == last:
                kept[last] = d_
            return mc_

        serial = [last] + [int(x) for x in srcs[:nsamp - 1]]
        rec = cpu_record("FIFO-queue BFS", bfs_q, serial, [int(x) for x in srcs],
                         f"of the {NSRC} R-MAT sources (the last timed one first) + the grid "
                         "from vertex 0", extra=(tg, mg))
        rec["all_cores"]["note"] = "all 64 R-MAT 22 sources; compare dobfs.queries_per_s"
        out["cpu_baseline"] = rec
        verified = bool(np.array_equal(depth.cpu().numpy(), kept[last]) and
                        np.array_equal(gdepth.cpu().numpy(), g_want))
        out["verified_against_oracle"] = {
            "ok": verified, "what": f"depths of R-MAT source {last} (the last one timed) and of "
                                    "the grid from vertex 0, as left by the timed step"}
    if not args.headline_only:
        # per-config side measurements (outside the step)
        del depth, parent, gdepth, gparent, ws, gws
        only = set(args.only.split(",")) if args.only else None

        def want(name):
            return only is None or name in only

        if want("sssp"):
            out["sssp"] = side_sssp(fg, torch, off, col, srcs, stream, not args.no_cpu)
            print(f"[bench] sssp done", file=sys.stderr, flush=True)
        off24 = col24 = None
        if want("package") or (want("serving") and not args.no_serving):
            t0 = time.time()
            off24, col24 = synth.rmat_csr(24, EDGE_FACTOR)
            print(f"[bench] rmat24 generated in {time.time() - t0:.1f}s, m={len(col24)}",
                  file=sys.stderr, flush=True)
        if want("package"):
            out["package"] = side_package(fg, torch, stream, not args.no_cpu, off24, col24)
            print(f"[bench] package done", file=sys.stderr, flush=True)
        if want("batched"):
            out["batched_c4"] = side_batched(fg, torch, stream, do_kw, not args.no_cpu)
            print(f"[bench] batched done", file=sys.stderr, flush=True)
        if want("batched_sssp"):
            out["batched_sssp"] = side_batched_sssp(fg, torch, stream, (off, col), not args.no_cpu)
            print(f"[bench] batched sssp done", file=sys.stderr, flush=True)
        if want("overhead"):
            out["overhead_l"] = side_overhead(fg, torch, stream)
            print(f"[bench] overhead done", file=sys.stderr, flush=True)
        if not args.no_widened:
            if want("dupall"):
                out["dupall"] = side_dupall(fg, torch, stream, off, col, srcs, not args.no_cpu)
                print(f"[bench] dupall done", file=sys.stderr, flush=True)
            if want("cc"):
                out["cc"] = side_cc(fg, torch, stream,
                                    {"rmat22": (off, col), "grid4096": (goff, gcol)},
                                    not args.no_cpu)
                print(f"[bench] cc done", file=sys.stderr, flush=True)
            if want("pagerank"):
                out["pagerank"] = side_pagerank(fg, torch, stream, off, col, not args.no_cpu)
                print(f"[bench] pagerank done", file=sys.stderr, flush=True)
        if want("serving") and not args.no_serving:
            out["serving"] = side_serving(fg, torch, {"rmat22": (off, col),
                                                      "grid4096": (goff, gcol),
                                                      "rmat24": (off24, col24)})
            print(f"[bench] serving done", file=sys.stderr, flush=True)
    # release every library object before the interpreter tears down
    torch.cuda.synchronize()
    g.close()
    gg.close()
    torch.cuda.synchronize()
    print(json.dumps(out), flush=True)
    if verified is False:
        print("bench.py: GPU depths differ from the oracle's", file=sys.stderr, flush=True)
        sys.exit(1)


if __name__ == "__main__":
    main()
