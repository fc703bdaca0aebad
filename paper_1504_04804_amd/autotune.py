"""Autotuner for the traversal parameters.

Sweeps the direction-optimizing thresholds do_a / do_b (Sec. VI-A: good
values are consistent within a graph type, e.g. 0.01 / 0.1 for social
graphs on the paper's GPUs), the high-degree cut of the push load balance,
the team-mode width, for push BFS the asynchronous team (levels between
synchronisations, team width), for batched BFS the push/pull switch
points, and for a list of sources run beside an asynchronous query in one
launch (fg_bfs_corun) the list's share of the workgroups.  Every
candidate runs on the device on a sample of sources; the fastest mean time
wins.  Results never change depths (the schedule only affects speed), which
the test suite checks separately.

Two caches:
  * a JSON file keyed by a graph signature (tuned_bfs_opts), tuned on a miss;
  * ``tuned.json`` beside this file, keyed by workload name, written by
    ``python -m paper_1504_04804_amd.autotune`` for the benchmark
    workloads and read (never re-tuned) by the benchmark and the
    config-scale tests through workload_opts().
"""
import itertools
import json
import os
import sys
import time

import torch

import paper_1504_04804_amd as fg

DO_A = [(1, 10), (1, 100), (1, 1000), (1, 10000), (1, 100000), (1, 10**6), (1, 10**7),
        (1, 10**8), (1, 10**9)]
DO_B = [(1, 10), (1, 1), (10, 1)]
BIG_DEG = [32, 64, 256]
TEAM = [-1, 8, 16, 24, 32]
ASYNC = [16, 32, 64, 128, 256]
ASYNC_TEAM = [32, 48, 64]
PULL_DIV = [4, 8, 16, 64, 256]
PUSH_DIV = [64, 512, 4096]
CORUN_WIDTH = [0, 184, 176, 168, 160, 152, 144, 128]

TUNED_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")


def signature(g):
    i = g.info()
    return f"n{i.n}_m{i.m}_dmax{i.max_degree}_nz{i.nonzero_degree}"


def _time_bfs(g, srcs, opts, reps=2):
    """Mean time per source, with parents, run as the benchmark runs them:
    the sources one after another in one launch (fg_bfs_many, shared
    outputs), or one launch each in the asynchronous push mode."""
    dev = g.off.device
    depth = torch.empty(g.n, dtype=torch.int32, device=dev)
    parent = torch.empty(g.n, dtype=torch.int32, device=dev)
    ws = g.workspace(fg.FG_PRIM_BFS)
    if opts.async_levels <= 1:
        sd = torch.tensor([int(s) for s in srcs], dtype=torch.int32, device=dev)

        def run():
            fg.bfs_many_into(g, sd, depth, parent, opts, ws=ws)
    else:
        def run():
            for s in srcs:
                fg.bfs_into(g, int(s), depth, parent, opts, ws=ws)
    run()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        run()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / (reps * len(srcs))


def tune_bfs(g, srcs, mode=fg.FG_MODE_DO, log=None, do_a=None, do_b=None, big_deg=None,
             team=None, async_levels=None, async_team=None):
    """Returns (best kwargs for fg.bfs_opts, ms per traversal).  The search
    spaces default to the module lists; tests pass smaller ones."""
    best = None
    da_l = DO_A if do_a is None else do_a
    db_l = DO_B if do_b is None else do_b
    do_space = itertools.product(da_l, db_l) if mode == fg.FG_MODE_DO else [((1, 100), (1, 10))]
    base = dict(mode=mode)
    # stage 1: direction thresholds with default balance parameters
    for da, db in do_space:
        kw = dict(base, do_a=da, do_b=db)
        ms = _time_bfs(g, srcs, fg.bfs_opts(**kw))
        if log:
            log(f"bfs {kw}: {ms:.4f} ms")
        if best is None or ms < best[1]:
            best = (kw, ms)
    # stage 2: load balance cut and team width around the best thresholds
    for bd, tm in itertools.product(BIG_DEG if big_deg is None else big_deg,
                                    TEAM if team is None else team):
        kw = dict(best[0], big_degree=bd, team_blocks=tm)
        ms = _time_bfs(g, srcs, fg.bfs_opts(**kw))
        if log:
            log(f"bfs {kw}: {ms:.4f} ms")
        if ms < best[1]:
            best = (kw, ms)
    # stage 3 (push, one source per call): the asynchronous team
    if mode == fg.FG_MODE_PUSH:
        for k, tm in itertools.product(ASYNC if async_levels is None else async_levels,
                                       ASYNC_TEAM if async_team is None else async_team):
            kw = dict(best[0], async_levels=k, team_blocks=tm)
            ms = _time_bfs(g, srcs, fg.bfs_opts(**kw))
            if log:
                log(f"bfs {kw}: {ms:.4f} ms")
            if ms < best[1]:
                best = (kw, ms)
    return best


def tune_msbfs(g, srcs, log=None, pull_div=None, push_div=None, reps=2):
    """Returns (best kwargs for fg.msbfs_opts, ms per batch of len(srcs) <= 64
    queries); each candidate's time is the faster of `reps` runs."""
    best = None
    for pd, sd in itertools.product(PULL_DIV if pull_div is None else pull_div,
                                    PUSH_DIV if push_div is None else push_div):
        b = fg.MsBatch(g, min(64, len(srcs)), fg.msbfs_opts(pull_div=pd, push_div=sd))
        ts = []
        for rep in range(reps):
            for lane, s in enumerate(srcs[:64]):
                if rep:
                    b.release(lane)
                b.admit(lane, int(s))
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            e = torch.cuda.Event(enable_timing=True)
            a.record()
            b.step(1 << 30)
            e.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(e))
        b.close()
        ms = min(ts)
        kw = dict(pull_div=pd, push_div=sd)
        if log:
            log(f"msbfs {kw}: {ms:.3f} ms")
        if best is None or ms < best[1]:
            best = (kw, ms)
    return best


def tune_corun(g, srcs, list_kw, g2, src2, opts2, log=None, widths=None, reps=2):
    """The list's workgroups in fg_bfs_corun (grid_blocks; 0 = every one the
    second query's team leaves): the list of `srcs` on g with the options
    `list_kw` beside the asynchronous push query from src2 on g2 (opts2).
    Returns (list_kw with the best grid_blocks, ms per call); each
    candidate's time is the mean of `reps` calls after one untimed one."""
    dev = g.off.device
    depth = torch.empty(g.n, dtype=torch.int32, device=dev)
    parent = torch.empty(g.n, dtype=torch.int32, device=dev)
    depth2 = torch.empty(g2.n, dtype=torch.int32, device=dev)
    parent2 = torch.empty(g2.n, dtype=torch.int32, device=dev)
    ws = g.workspace(fg.FG_PRIM_BFS)
    ws2 = g2.workspace(fg.FG_PRIM_BFS)
    sd = torch.tensor([int(s) for s in srcs], dtype=torch.int32, device=dev)
    best = None
    for w in CORUN_WIDTH if widths is None else widths:
        kw = dict(list_kw, grid_blocks=w)
        o = fg.bfs_opts(**kw)

        def run():
            fg.bfs_corun_into(g, sd, depth, parent, o, ws, None, g2, src2, depth2, parent2, opts2,
                              ws2=ws2)
        run()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            run()
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / reps
        if log:
            log(f"corun {kw}: {ms:.3f} ms")
        if best is None or ms < best[1]:
            best = (kw, ms)
    return best


def load(path):
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def save(path, cache):
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
        f.write("\n")
    os.replace(tmp, path)


def _to_json(kw):
    return {k: (list(v) if isinstance(v, tuple) else v) for k, v in kw.items()}


def _from_json(kw):
    return {k: (tuple(v) if isinstance(v, list) else v) for k, v in kw.items()}


def tuned_bfs_opts(g, srcs, path, mode=fg.FG_MODE_DO, log=None, **space):
    """fg.bfs_opts for `g` from the cache at `path`, tuning on a miss."""
    cache = load(path)
    key = f"bfs{mode}:{signature(g)}"
    if key not in cache:
        kw, ms = tune_bfs(g, srcs, mode, log, **space)
        cache[key] = dict(kwargs=_to_json(kw), ms=ms)
        save(path, cache)
    kw = _from_json(cache[key]["kwargs"])
    return fg.bfs_opts(**kw), kw


def workload_opts(name, g, path=TUNED_PATH):
    """(options object, kwargs) the autotuner stored for workload `name`;
    raises if the entry is missing or was tuned on another graph."""
    cache = load(path)
    if name not in cache:
        raise KeyError(f"{path} has no entry for {name}: run python -m paper_1504_04804_amd.autotune")
    ent = cache[name]
    if ent["signature"] != signature(g):
        raise ValueError(f"{name} was tuned on {ent['signature']}, not {signature(g)}")
    kw = _from_json(ent["kwargs"])
    make = fg.msbfs_opts if ent["kind"] == "msbfs" else fg.bfs_opts
    return make(**kw), kw


def main():
    """Tunes the benchmark workloads and writes tuned.json:
    rmat22_dobfs (direction-optimizing BFS, R-MAT 22, the 64 sources),
    grid4096_push (push BFS, 4096 x 4096 grid, vertex 0),
    rmat23_msbfs and grid2048_msbfs (64-lane batches, their 64 sources),
    rmat23_dobfs and grid2048_push (the one-at-a-time paths the batches are
    compared with: R-MAT 23's 64 sources, the grid's first 4),
    rmat22_dobfs_corun (rmat22_dobfs's options and the list's share of the
    workgroups when the 64 sources run beside the grid4096_push query in
    one launch; needs those two entries)."""
    ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import synth
    torch.cuda.set_device(0)
    log = lambda s: print(f"[autotune] {s}", flush=True)
    cache = load(TUNED_PATH)
    every = lambda off: [int(s) for s in synth.sources(off, 64)]
    jobs = [("rmat22_dobfs", lambda: synth.rmat_csr(22, 16), "bfs", fg.FG_MODE_DO, every),
            ("grid4096_push", lambda: synth.grid_csr(4096, 4096), "bfs", fg.FG_MODE_PUSH,
             lambda off: [0]),
            ("rmat23_msbfs", lambda: synth.rmat_csr(23, 16), "msbfs", None, every),
            ("grid2048_msbfs", lambda: synth.grid_csr(2048, 2048), "msbfs", None, every),
            ("rmat23_dobfs", lambda: synth.rmat_csr(23, 16), "bfs", fg.FG_MODE_DO, every),
            ("grid2048_push", lambda: synth.grid_csr(2048, 2048), "bfs", fg.FG_MODE_PUSH,
             lambda off: every(off)[:4])]
    jobs.append(("rmat22_dobfs_corun", lambda: synth.rmat_csr(22, 16), "corun", None, every))
    only = set(sys.argv[1:])
    for name, make, kind, mode, pick in jobs:
        if only and name not in only:
            continue
        t0 = time.time()
        off, col = make()
        g = fg.Graph(off, col, symmetric=True, validate=False)
        srcs = pick(off)
        if kind == "bfs":
            kw, ms = tune_bfs(g, srcs, mode, log)
        elif kind == "corun":
            goff, gcol = synth.grid_csr(4096, 4096)
            g2 = fg.Graph(goff, gcol, symmetric=True, validate=False)
            _, list_kw = workload_opts("rmat22_dobfs", g)
            opts2, _ = workload_opts("grid4096_push", g2)
            kw, ms = tune_corun(g, srcs, list_kw, g2, 0, opts2, log)
            g2.close()
            kind = "bfs"
        else:
            kw, ms = tune_msbfs(g, srcs, log)
        cache[name] = dict(kind=kind, signature=signature(g), kwargs=_to_json(kw),
                           ms=round(ms, 4), sources=len(srcs),
                           tuned_s=round(time.time() - t0, 1))
        log(f"{name}: {kw} {ms:.4f} ms")
        g.close()
        save(TUNED_PATH, cache)


if __name__ == "__main__":
    main()
