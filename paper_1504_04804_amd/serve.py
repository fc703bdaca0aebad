"""Query server: continuous batching of BFS / SSSP queries over resident graphs.

Requests (graph, kind, source) arrive over time.  BFS requests are admitted
into free lanes of a 64-lane batched traversal of their graph (fg_msbfs_*)
at step boundaries, so queries that arrive while others run join the same
device launches; a lane retires as soon as its frontier empties and its
depths are copied out.  SSSP requests run as single-query launches between
batched steps.  Memory for batches and SSSP workspaces is admitted against an
explicit HBM budget: a request waits while its graph's batch or an SSSP
workspace does not fit.

All device work is issued on one stream: every traversal is a cooperative
persistent launch that expects the whole device, so two of them must not
run concurrently; the overlap between queries comes from sharing launches.
"""
import collections
import time

import numpy as np
import torch

import paper_1504_04804_amd as fg

BFS, SSSP = 0, 1


class Request:
    __slots__ = ("rid", "graph", "kind", "src", "arrival", "start", "done", "result")

    def __init__(self, rid, graph, kind, src, arrival):
        self.rid, self.graph, self.kind, self.src, self.arrival = rid, graph, kind, src, arrival
        self.start = None
        self.done = None
        self.result = None


class _GraphSlot:
    def __init__(self, name, g):
        self.name = name
        self.g = g
        self.batch = None          # fg.MsBatch, allocated on first BFS request
        self.lane_req = {}         # lane -> Request
        self.free = list(range(63, -1, -1))
        self.sssp_ws = None


class Server:
    """Continuous-batching query server over resident graphs.

    graphs: dict name -> fg.Graph (SSSP needs weights).  hbm_budget: bytes the
    server may allocate for batch workspaces, SSSP workspaces and results.
    k_iters: BFS levels per batched step (the admission granularity).
    """

    def __init__(self, graphs, hbm_budget=32 << 30, k_iters=4, keep_results=True):
        self.slots = {name: _GraphSlot(name, g) for name, g in graphs.items()}
        self.budget = int(hbm_budget)
        self.used = 0
        self.k_iters = k_iters
        self.keep = keep_results
        self.pending = collections.deque()
        self.finished = []
        self.stream = torch.cuda.current_stream()

    # ---------------------------------------------------------- memory
    def _reserve(self, nbytes):
        if self.used + nbytes > self.budget:
            return False
        self.used += nbytes
        return True

    def _batch(self, slot):
        if slot.batch is None:
            nb = slot.g.workspace_bytes(fg.FG_PRIM_MSBFS, 64)
            if not self._reserve(nb):
                return None
            slot.batch = fg.MsBatch(slot.g, 64)
        return slot.batch

    def _sssp_ws(self, slot):
        if slot.sssp_ws is None:
            nb = slot.g.workspace_bytes(fg.FG_PRIM_SSSP)
            if not self._reserve(nb):
                return None
            slot.sssp_ws = torch.zeros(max(nb, 256), dtype=torch.uint8, device="cuda")
        return slot.sssp_ws

    # ---------------------------------------------------------- scheduling
    def submit(self, req):
        self.pending.append(req)

    def _admit(self, now):
        """Admit pending requests whose resources are available (FIFO per kind)."""
        sssp_now = []
        keep = collections.deque()
        while self.pending:
            r = self.pending.popleft()
            slot = self.slots[r.graph]
            if r.kind == BFS:
                b = self._batch(slot)
                if b is None or not slot.free:
                    keep.append(r)
                    continue
                lane = slot.free.pop()
                b.admit(lane, r.src)
                slot.lane_req[lane] = r
                r.start = now
            else:
                if self._sssp_ws(slot) is None:
                    keep.append(r)
                    continue
                r.start = now
                sssp_now.append(r)
        self.pending = keep
        return sssp_now

    def _run_sssp(self, r):
        slot = self.slots[r.graph]
        g = slot.g
        dist = torch.empty(g.n, dtype=torch.int32, device="cuda")
        fg.sssp_into(g, r.src, dist, None, ws=slot.sssp_ws, stream=self.stream)
        return dist

    def tick(self, now_fn):
        """One scheduling round: admit, run SSSP queries, one batched step per
        graph with live lanes, then retire finished lanes."""
        sssp_now = self._admit(now_fn())
        outs = [(r, self._run_sssp(r)) for r in sssp_now]
        stepped = []
        for slot in self.slots.values():
            if slot.lane_req:
                slot.batch.step(self.k_iters, stream=self.stream)
                stepped.append(slot)
        if outs:
            self.stream.synchronize()
            t = now_fn()
            for r, dist in outs:
                r.done = t
                if self.keep:
                    r.result = dist
                self.finished.append(r)
        for slot in stepped:
            done, _ = slot.batch.poll(stream=self.stream)
            t = now_fn()
            for lane in [l for l in slot.lane_req if (done >> l) & 1]:
                r = slot.lane_req.pop(lane)
                if self.keep:
                    r.result = slot.batch.read(lane, stream=self.stream).clone()
                slot.batch.release(lane)
                slot.free.append(lane)
                r.done = t
                self.finished.append(r)
        return bool(sssp_now or stepped)

    def busy(self):
        return bool(self.pending) or any(s.lane_req for s in self.slots.values())


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


def serve_fifo(graphs, reqs, sssp_ws, time_limit=600.0):
    """The one-at-a-time plain path: each request runs alone (fg_bfs /
    fg_sssp) in arrival order, on the same stream and device."""
    t0 = time.perf_counter()
    now = lambda: time.perf_counter() - t0
    out = []
    o = fg.bfs_opts(mode=fg.FG_MODE_DO)
    for r in reqs:
        while now() < r.arrival:
            time.sleep(min(r.arrival - now(), 0.002))
        r.start = now()
        g = graphs[r.graph]
        if r.kind == BFS:
            d = torch.empty(g.n, dtype=torch.int32, device="cuda")
            fg.bfs_into(g, r.src, d, None, o if g.symmetric else fg.bfs_opts(mode=fg.FG_MODE_PUSH))
        else:
            d = torch.empty(g.n, dtype=torch.int32, device="cuda")
            fg.sssp_into(g, r.src, d, None, ws=sssp_ws[r.graph])
        torch.cuda.current_stream().synchronize()
        r.done = now()
        r.result = d
        out.append(r)
        if now() > time_limit:
            raise RuntimeError("FIFO replay exceeded its time limit")
    return out


def latency_stats(done):
    lat = np.array([r.done - r.arrival for r in done]) * 1e3
    span = max(r.done for r in done) - min(r.arrival for r in done)
    return dict(n=len(done), p50_ms=float(np.percentile(lat, 50)),
                p99_ms=float(np.percentile(lat, 99)), qps=len(done) / span)
