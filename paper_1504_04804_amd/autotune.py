"""Autotuner for the traversal parameters.

Sweeps the direction-optimizing thresholds do_a / do_b (Sec. VI-A: good
values are consistent within a graph type, e.g. 0.01 / 0.1 for social
graphs on the paper's GPUs), the high-degree cut of the push load balance,
the team-mode width, and for batched BFS the push/pull switch points.  Every
candidate runs on the device on a sample of sources; the fastest mean time
wins.  Results never change depths (the schedule only affects speed), which
the test suite checks separately.  The cache is a JSON file keyed by a graph
signature.
"""
import itertools
import json
import os

import torch

import paper_1504_04804_amd as fg

DO_A = [(1, 10), (1, 100), (1, 1000), (1, 10000), (1, 100000)]
DO_B = [(1, 10), (1, 1), (10, 1)]
BIG_DEG = [32, 64, 256]
TEAM = [-1, 8, 16, 32]


def signature(g):
    i = g.info()
    return f"n{i.n}_m{i.m}_dmax{i.max_degree}_nz{i.nonzero_degree}"


def _time_bfs(g, srcs, opts, reps=2):
    depth = torch.empty(g.n, dtype=torch.int32, device=g.off.device)
    ws = g.workspace(fg.FG_PRIM_BFS)
    for s in srcs[:1]:
        fg.bfs_into(g, int(s), depth, None, opts, ws=ws)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        for s in srcs:
            fg.bfs_into(g, int(s), depth, None, opts, ws=ws)
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / (reps * len(srcs))


def tune_bfs(g, srcs, mode=fg.FG_MODE_DO, log=None):
    """Returns (best kwargs for fg.bfs_opts, ms per traversal)."""
    best = None
    do_space = itertools.product(DO_A, DO_B) if mode == fg.FG_MODE_DO else [((1, 100), (1, 10))]
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
    for bd, team in itertools.product(BIG_DEG, TEAM):
        kw = dict(best[0], big_degree=bd, team_blocks=team)
        ms = _time_bfs(g, srcs, fg.bfs_opts(**kw))
        if log:
            log(f"bfs {kw}: {ms:.4f} ms")
        if ms < best[1]:
            best = (kw, ms)
    return best


def tune_msbfs(g, srcs, log=None):
    best = None
    for pull_div, push_div in itertools.product([4, 8, 16, 64, 256], [64, 512, 4096]):
        b = fg.MsBatch(g, min(64, len(srcs)), fg.msbfs_opts(pull_div=pull_div, push_div=push_div))
        for lane, s in enumerate(srcs[:64]):
            b.admit(lane, int(s))
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        a.record()
        b.step(1 << 30)
        e.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(e)
        b.close()
        kw = dict(pull_div=pull_div, push_div=push_div)
        if log:
            log(f"msbfs {kw}: {ms:.3f} ms")
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
    os.replace(tmp, path)


def tuned_bfs_opts(g, srcs, path, mode=fg.FG_MODE_DO, log=None):
    """fg.bfs_opts for `g` from the cache at `path`, tuning on a miss."""
    cache = load(path)
    key = f"bfs{mode}:{signature(g)}"
    if key not in cache:
        kw, ms = tune_bfs(g, srcs, mode, log)
        cache[key] = dict(kwargs={k: (list(v) if isinstance(v, tuple) else v) for k, v in kw.items()},
                          ms=ms)
        save(path, cache)
    kw = {k: (tuple(v) if isinstance(v, list) else v) for k, v in cache[key]["kwargs"].items()}
    return fg.bfs_opts(**kw), kw
