"""Query server: continuous batching of BFS / SSSP queries over resident graphs.

Requests (graph, kind, source) arrive over time.  Per graph and kind the
server keeps a 64-lane batch (fg_msbfs_* for BFS, fg_mssp_* for SSSP):
requests are admitted into free lanes at step boundaries, so queries that
arrive while others run join the same device launches, and a lane retires
as soon as its query is done and its result is copied out.  A batch over a
few lanes costs more device time than one single-source run (fg_bfs /
fg_sssp) but far less than many, so when a batch is idle a cost model
measured per graph and kind decides whether the waiting requests start a
batch or the oldest one runs alone.  Batch and single-run workspaces are
admitted against an explicit HBM budget: idle batches are closed, least
recently used first, to make room, and requests wait while nothing fits.

The device runs one unit of work at a time (each is a cooperative
persistent launch).  The next unit -- a step of a running batch, the start
of a batch, or a single run -- is the one holding the oldest request, and
steps are sized from the measured time per iteration so the device changes
hands every few milliseconds.  A single BFS on a graph of mean degree <= 8
runs as an asynchronous push team on 64 workgroups; when BFS queries on a
direction-optimizing graph are waiting outside a batch, the oldest of those
kinds runs a list of them one after another on the other workgroups of the
same launch (fg_bfs_corun), as many as take about as long as the team.
"""
import collections
import time

import numpy as np
import torch

import paper_1504_04804_amd as fg

BFS, SSSP = 0, 1
LANES = 64


def single_bfs_opts(g):
    """Options of a single-source BFS on `g`, the same for the server and the
    one-at-a-time path: direction-optimizing on undirected graphs with
    hubs, push otherwise; on graphs of mean degree <= 8 (grids, road-like,
    high diameter) the asynchronous push team (64 levels between
    synchronisations, 64 workgroups), several times faster there than a
    level-synchronous traversal."""
    if g.m <= 8 * g.n:
        return fg.bfs_opts(mode=fg.FG_MODE_PUSH, async_levels=64, team_blocks=64)
    return fg.bfs_opts(mode=fg.FG_MODE_DO if g.symmetric else fg.FG_MODE_PUSH)


class Request:
    __slots__ = ("rid", "graph", "kind", "src", "arrival", "start", "done", "result", "path")

    def __init__(self, rid, graph, kind, src, arrival):
        self.rid, self.graph, self.kind, self.src, self.arrival = rid, graph, kind, src, arrival
        self.start = None
        self.done = None
        self.result = None
        self.path = None  # "batch" or "single" once served


class Cost:
    """Device time of one graph and kind, in ms: `single` per single-source
    run; a batch of L lanes run to the end takes batch(L), linear between
    the measured 1-lane and 8-lane batches; `it_ms` per batched iteration."""

    def __init__(self, single, batch1, batch8, it_ms):
        self.single, self.batch1, self.batch8, self.it_ms = single, batch1, batch8, it_ms

    def batch(self, lanes):
        return self.batch1 + (self.batch8 - self.batch1) * (lanes - 1) / 7.0

    def prefer_batch(self, lanes):
        return lanes > 1 and self.batch(lanes) < lanes * self.single

    def as_dict(self):
        return dict(single_ms=round(self.single, 3), batch1_ms=round(self.batch1, 3),
                    batch8_ms=round(self.batch8, 3), it_ms=round(self.it_ms, 4))


class _Kind:
    """State of one (graph, kind): waiting requests, the batch and its lanes."""

    def __init__(self, name, g, kind):
        self.name, self.g, self.kind = name, g, kind
        self.waiting = collections.deque()
        self.batch = None
        self.batch_bytes = 0
        self.lane_req = {}
        self.free = list(range(LANES - 1, -1, -1))
        self.single_ws = None
        self.single_bytes = 0
        self.single_out = None
        # a single BFS here runs as an asynchronous push team
        self.async_single = kind == BFS and single_bfs_opts(g).async_levels > 1
        self.cost = None
        self.it_ms = None  # running estimate of the batch's time per iteration
        self.it_seen = 0   # the batch's iteration count after its last step
        self.last_used = 0.0

    def oldest(self):
        t = self.waiting[0].arrival if self.waiting else float("inf")
        for r in self.lane_req.values():
            t = min(t, r.arrival)
        return t

    def prim(self):
        return fg.FG_PRIM_MSBFS if self.kind == BFS else fg.FG_PRIM_MSSSP

    def open_batch(self):
        return fg.MsBatch(self.g, LANES) if self.kind == BFS else fg.MsspBatch(self.g, LANES)


class Server:
    """Continuous-batching query server over resident graphs.

    graphs: dict name -> fg.Graph (SSSP needs weights).  hbm_budget: bytes
    the server may hold in workspaces (the resident graphs' own bytes come on
    top: `resident_bytes`; `peak_used` is the most the workspaces held).  policy: "auto" (the cost model picks
    batch or single when a batch is idle), "batch" (always batch) or
    "single" (always single runs, oldest first).  costs: dict (name, kind) ->
    Cost, e.g. from calibrate(); missing entries default to batching.
    step_ms: target device time of one batched step.
    """

    def __init__(self, graphs, hbm_budget=32 << 30, policy="auto", costs=None, step_ms=4.0,
                 keep_results=True, stream=None):
        self.kinds = {}
        for name, g in graphs.items():
            self.kinds[(name, BFS)] = _Kind(name, g, BFS)
            if g.w is not None:
                self.kinds[(name, SSSP)] = _Kind(name, g, SSSP)
        for key, c in (costs or {}).items():
            if key in self.kinds:
                self.kinds[key].cost = c
        self.budget = int(hbm_budget)
        self.used = 0
        self.peak_used = 0
        # HBM the resident graphs hold (CSR, weights, head table, masks),
        # outside the workspace budget; reported beside it
        self.resident_bytes = sum(int(g.info().resident_bytes) for g in graphs.values())
        self.policy = policy
        self.step_ms = float(step_ms)
        self.keep = keep_results
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.finished = []
        self.counts = collections.Counter()
        self.stats = None
        self.list_stats = None

    def close(self):
        """Close every batch and drop the workspaces (waits for the device)."""
        self.stream.synchronize()
        for k in self.kinds.values():
            if k.batch is not None:
                self._close_batch(k)
            k.single_ws = None
            k.single_out = None
            self.used -= k.single_bytes
            k.single_bytes = 0

    # ---------------------------------------------------------- memory
    def _reserve(self, nbytes, keep=None):
        """Reserve nbytes, closing idle batches (least recently used first)."""
        if self.used + nbytes <= self.budget:
            self.used += nbytes
            self.peak_used = max(self.peak_used, self.used)
            return True
        idle = sorted((k for k in self.kinds.values()
                       if k.batch is not None and not k.lane_req and k is not keep),
                      key=lambda k: k.last_used)
        for k in idle:
            self._close_batch(k)
            self.counts["evictions"] += 1
            if self.used + nbytes <= self.budget:
                self.used += nbytes
                self.peak_used = max(self.peak_used, self.used)
                return True
        return False

    def _close_batch(self, k):
        k.batch.close()
        k.batch = None
        self.used -= k.batch_bytes
        k.batch_bytes = 0
        k.free = list(range(LANES - 1, -1, -1))

    def _ensure_batch(self, k):
        if k.batch is None:
            nb = k.g.workspace_bytes(k.prim(), LANES)
            if not self._reserve(nb, keep=k):
                return False
            k.batch = k.open_batch()
            k.batch_bytes = nb
            k.it_seen = 0
        return True

    def _ensure_single(self, k):
        if k.single_ws is None:
            prim = fg.FG_PRIM_BFS if k.kind == BFS else fg.FG_PRIM_SSSP
            nb = k.g.workspace_bytes(prim)
            if not self._reserve(nb, keep=k):
                return False
            k.single_ws = k.g.workspace(prim)
            k.single_bytes = nb
        return True

    # ---------------------------------------------------------- scheduling
    def submit(self, req):
        self.kinds[(req.graph, req.kind)].waiting.append(req)

    def busy(self):
        return any(k.waiting or k.lane_req for k in self.kinds.values())

    def _want_batch(self, k):
        if self.policy == "batch":
            return True
        if self.policy == "single":
            return False
        c = k.cost
        return c is None or c.prefer_batch(min(len(k.waiting), LANES))

    def _admit(self, k, now):
        while k.waiting and k.free:
            r = k.waiting.popleft()
            lane = k.free.pop()
            k.batch.admit(lane, r.src)
            k.lane_req[lane] = r
            r.start = now
            r.path = "batch"

    def _step(self, k, now_fn):
        it_ms = k.it_ms or (k.cost.it_ms if k.cost else 0.05)
        iters = int(max(1, min(1 << 20, round(self.step_ms / max(it_ms, 1e-4)))))
        it0 = k.it_seen
        t0 = time.perf_counter()
        k.batch.step(iters, stream=self.stream)
        done, it1 = k.batch.poll(stream=self.stream)
        dt = (time.perf_counter() - t0) * 1e3
        ran = it1 - it0
        k.it_seen = it1
        if ran > 0:
            est = dt / ran
            k.it_ms = est if k.it_ms is None else 0.5 * k.it_ms + 0.5 * est
        self.counts["steps"] += 1
        t = now_fn()
        for lane in [l for l in k.lane_req if (done >> l) & 1]:
            r = k.lane_req.pop(lane)
            if self.keep:
                r.result = k.batch.read(lane, stream=self.stream).clone()
            k.batch.release(lane)
            k.free.append(lane)
            r.done = t
            self.finished.append(r)
        if self.keep:
            self.stream.synchronize()

    def _single(self, k, now_fn):
        r = k.waiting.popleft()
        r.start = now_fn()
        r.path = "single"
        g = k.g
        if self.keep or k.single_out is None:
            out = torch.empty(g.n, dtype=torch.int32, device=g.off.device)
            if not self.keep:
                k.single_out = out  # results are dropped: one buffer per kind
        else:
            out = k.single_out
        if self.stats is None:
            self.stats = fg.new_stats(g.off.device)
        if k.kind == BFS:
            o = single_bfs_opts(g)
            fg.bfs_into(g, r.src, out, None, o, ws=k.single_ws, stats=self.stats,
                        stream=self.stream)
        else:
            fg.sssp_into(g, r.src, out, None, ws=k.single_ws, stats=self.stats, stream=self.stream)
        st = fg.read_stats(self.stats, stream=self.stream)
        if st.status != 0:
            raise RuntimeError(f"single {'BFS' if k.kind == BFS else 'SSSP'} on {k.name} "
                               f"from {r.src} ended with status {st.status}")
        self.counts["singles"] += 1
        r.done = now_fn()
        if self.keep:
            r.result = out
        self.finished.append(r)

    def _corun_partner(self, k):
        """Among the BFS kinds on direction-optimizing graphs with waiting
        requests and no running batch, the one holding the oldest request."""
        best = None
        for k2 in self.kinds.values():
            if k2 is k or k2.kind != BFS or k2.async_single or not k2.g.symmetric:
                continue
            if not k2.waiting or k2.lane_req:
                continue
            if best is None or k2.waiting[0].arrival < best.waiting[0].arrival:
                best = k2
        return best

    def _corun(self, k, now_fn):
        """The oldest request of k (an asynchronous single BFS) with a list of
        a partner kind's waiting requests beside it in one launch; False if
        there is no partner."""
        k2 = self._corun_partner(k)
        if k2 is None or not self._ensure_single(k2):
            return False
        # as many list queries as take about as long as the team
        nl = int(k.cost.single / max(k2.cost.single, 1e-3)) if k.cost and k2.cost else 8
        nl = max(1, min(nl, len(k2.waiting), LANES))
        r = k.waiting.popleft()
        lst = [k2.waiting.popleft() for _ in range(nl)]
        t = now_fn()
        r.start, r.path = t, "single"
        for q in lst:
            q.start, q.path = t, "corun"
        g, g2 = k.g, k2.g
        dev = g.off.device
        if self.keep or k.single_out is None:
            out = torch.empty(g.n, dtype=torch.int32, device=dev)
            if not self.keep:
                k.single_out = out
        else:
            out = k.single_out
        if self.keep:
            lout = torch.empty(nl * g2.n, dtype=torch.int32, device=dev)
            stride = g2.n
        else:
            if k2.single_out is None:
                k2.single_out = torch.empty(g2.n, dtype=torch.int32, device=dev)
            lout, stride = k2.single_out, 0
        if self.stats is None:
            self.stats = fg.new_stats(dev)
        if self.list_stats is None:
            self.list_stats = fg.new_stats_many(LANES, dev)
        srcs = torch.tensor([q.src for q in lst], dtype=torch.int32, device=dev)
        fg.bfs_corun_into(g2, srcs, lout, None, single_bfs_opts(g2), k2.single_ws,
                          self.list_stats, g, r.src, out, None, single_bfs_opts(g),
                          ws2=k.single_ws, stats2=self.stats, stream=self.stream, out_stride=stride)
        sts = fg.read_stats_many(self.list_stats, nl, stream=self.stream)
        st = fg.read_stats(self.stats, stream=self.stream)
        bad = [(q.src, s_.status) for q, s_ in zip(lst, sts) if s_.status != 0]
        if st.status != 0 or bad:
            raise RuntimeError(f"co-run of BFS on {k.name} from {r.src} (status {st.status}) and "
                               f"{nl} BFS on {k2.name} (failed: {bad})")
        t = now_fn()
        r.done = t
        r.result = out if self.keep else None
        self.finished.append(r)
        for j, q in enumerate(lst):
            q.done = t
            q.result = lout[j * g2.n:(j + 1) * g2.n] if self.keep else None
            self.finished.append(q)
        k2.last_used = time.perf_counter()
        self.counts["singles"] += 1
        self.counts["coruns"] += 1
        self.counts["corun_list"] += nl
        return True

    def tick(self, now_fn):
        """Run the unit of work that holds the oldest request; False when
        there is nothing to run."""
        live = [k for k in self.kinds.values() if k.waiting or k.lane_req]
        if not live:
            return False
        live.sort(key=lambda k: k.oldest())
        for k in live:
            k.last_used = time.perf_counter()
            if k.lane_req:
                self._admit(k, now_fn())
                self._step(k, now_fn)
                return True
            if self._want_batch(k) and self._ensure_batch(k):
                k.it_ms = None
                self._admit(k, now_fn())
                self._step(k, now_fn)
                return True
            if self._ensure_single(k):
                if not (k.async_single and self._corun(k, now_fn)):
                    self._single(k, now_fn)
                return True
            # nothing of this kind fits the budget now; try the next one
        raise RuntimeError("no waiting request fits the HBM budget")


def calibrate(graphs, sources_per_graph, stream=None):
    """Measure the cost model of every graph and kind: single-source runs
    (one warm-up, two timed) and batches of 1 and 8 lanes run to the end
    (the faster of two runs each).
    sources_per_graph: dict name -> at least 8 source vertices."""
    stream = stream if stream is not None else torch.cuda.current_stream()
    costs = {}

    def timed(fn):
        stream.synchronize()
        t0 = time.perf_counter()
        fn()
        stream.synchronize()
        return (time.perf_counter() - t0) * 1e3

    for name, g in graphs.items():
        srcs = [int(s) for s in sources_per_graph[name][:8]]
        kinds = [BFS] + ([SSSP] if g.w is not None else [])
        for kind in kinds:
            out = torch.empty(g.n, dtype=torch.int32, device=g.off.device)
            if kind == BFS:
                ws = g.workspace(fg.FG_PRIM_BFS)
                o = single_bfs_opts(g)
                run1 = lambda s: fg.bfs_into(g, s, out, None, o, ws=ws, stream=stream)
                b = fg.MsBatch(g, LANES, stream=stream)
            else:
                ws = g.workspace(fg.FG_PRIM_SSSP)
                run1 = lambda s: fg.sssp_into(g, s, out, None, ws=ws, stream=stream)
                b = fg.MsspBatch(g, LANES, stream=stream)
            run1(srcs[0])
            single = (timed(lambda: run1(srcs[1])) + timed(lambda: run1(srcs[2]))) / 2

            def batch_run(lanes_srcs):
                for lane in range(LANES):
                    if (b.admitted >> lane) & 1:
                        b.release(lane)
                for lane, s in enumerate(lanes_srcs):
                    b.admit(lane, s)
                _, it0 = b.poll(stream=stream)
                t = timed(lambda: b.step(1 << 30, stream=stream))
                _, it1 = b.poll(stream=stream)
                return t, it1 - it0

            batch_run(srcs[:1])
            # the faster of two runs: one-off stalls (a first touch of fresh
            # workspace memory) must not set the model
            t1 = min(batch_run(srcs[1:2])[0], batch_run(srcs[2:3])[0])
            t8, it8 = batch_run(srcs[:8])
            t8b, it8b = batch_run(srcs[:8])
            if t8b < t8:
                t8, it8 = t8b, it8b
            b.close()
            del ws
            costs[(name, kind)] = Cost(single, t1, t8, t8 / max(it8, 1))
    return costs


def poisson_arrivals(n, qps, seed):
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / qps, size=n))


def make_requests(graph_specs, nreq, qps, bfs_frac=0.8, seed=1):
    """graph_specs: dict name -> (row_offsets numpy, has_weights).  Uniform
    graph, uniform source of nonzero degree, Poisson arrivals."""
    rng = np.random.default_rng(seed)
    names = sorted(graph_specs)
    arr = poisson_arrivals(nreq, qps, seed + 1)
    reqs = []
    for i in range(nreq):
        name = names[rng.integers(len(names))]
        off, weighted = graph_specs[name]
        deg = np.diff(off)
        while True:
            s = int(rng.integers(len(off) - 1))
            if deg[s] > 0:
                break
        kind = BFS if (rng.random() < bfs_frac or not weighted) else SSSP
        reqs.append(Request(i, name, kind, s, float(arr[i])))
    return reqs


def serve_stream(server, reqs, time_limit=600.0):
    """Replay `reqs` against `server` in real time; returns finished requests."""
    t0 = time.perf_counter()
    now = lambda: time.perf_counter() - t0
    i = 0
    while i < len(reqs) or server.busy():
        while i < len(reqs) and reqs[i].arrival <= now():
            server.submit(reqs[i])
            i += 1
        if not server.tick(now):
            # idle: wait for the next arrival
            if i < len(reqs):
                dt = reqs[i].arrival - now()
                if dt > 0:
                    time.sleep(min(dt, 0.002))
        if now() > time_limit:
            raise RuntimeError("serving replay exceeded its time limit")
    return server.finished


def serve_fifo(graphs, reqs, sssp_ws, time_limit=600.0, bfs_ws=None, keep_results=True):
    """The one-at-a-time plain path: each request runs alone (fg_bfs /
    fg_sssp) in arrival order, on the same stream and device.  Without
    keep_results the outputs go to one buffer per graph and are dropped."""
    t0 = time.perf_counter()
    now = lambda: time.perf_counter() - t0
    out = []
    bufs = {}
    for r in reqs:
        while True:
            dt = r.arrival - now()  # one clock read: the wait left, if any
            if dt <= 0:
                break
            time.sleep(min(dt, 0.002))
        r.start = now()
        g = graphs[r.graph]
        if keep_results:
            d = torch.empty(g.n, dtype=torch.int32, device="cuda")
        else:
            d = bufs.get(r.graph)
            if d is None:
                d = bufs[r.graph] = torch.empty(g.n, dtype=torch.int32, device="cuda")
        if r.kind == BFS:
            ws = bfs_ws[r.graph] if bfs_ws else None
            fg.bfs_into(g, r.src, d, None, single_bfs_opts(g), ws=ws)
        else:
            fg.sssp_into(g, r.src, d, None, ws=sssp_ws[r.graph])
        torch.cuda.current_stream().synchronize()
        r.done = now()
        r.result = d if keep_results else None
        r.path = "single"
        out.append(r)
        if now() > time_limit:
            raise RuntimeError("FIFO replay exceeded its time limit")
    return out


def latency_stats(done):
    lat = np.array([r.done - r.arrival for r in done]) * 1e3
    span = max(r.done for r in done) - min(r.arrival for r in done)
    return dict(n=len(done), p50_ms=float(np.percentile(lat, 50)),
                p99_ms=float(np.percentile(lat, 99)), qps=len(done) / span)
