"""MI355X frontier graph traversal: Python binding of libfg.so.

Argument marshalling only: every step of the traversal runs in the HIP
kernels of ``libfg.so`` (see ``include/fg.h`` for the C ABI).  PyTorch
provides device memory and streams.  Importing this package never falls
back to a CPU implementation: if the library is missing, calls raise.
"""
import ctypes
import os

import torch  # loaded first so libfg.so binds to the HIP runtime torch uses

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfg.so")

FG_OK, FG_EINVAL, FG_ENOMEM, FG_EDEVICE, FG_EOVERFLOW, FG_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
FG_DEVICE_PTRS, FG_BORROW, FG_VALIDATE, FG_SYMMETRIC = 1, 2, 4, 8
FG_PRIM_BFS, FG_PRIM_BFS_UNFUSED, FG_PRIM_SSSP, FG_PRIM_MSBFS, FG_PRIM_MSSSP = 0, 1, 2, 3, 4
FG_PRIM_PR, FG_PRIM_CC = 5, 6
FG_MODE_DO, FG_MODE_PUSH, FG_MODE_PUSH_UNFUSED = 0, 1, 2
FG_TRACE_MAX = 64
PUSH, PULL = 0, 1


class FGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"fg status {status}: {msg}")
        self.status = status


class RunStats(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("iterations", ctypes.c_int32),
        ("reached", ctypes.c_int64),
        ("edges_inspected", ctypes.c_int64),
        ("direction_switches", ctypes.c_int32),
        ("grid_blocks", ctypes.c_int32),
        ("clock_khz", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("t_start", ctypes.c_int64),
        ("dir", ctypes.c_int8 * FG_TRACE_MAX),
        ("frontier", ctypes.c_int64 * FG_TRACE_MAX),
        ("inspected", ctypes.c_int64 * FG_TRACE_MAX),
        ("t_end", ctypes.c_int64 * FG_TRACE_MAX),
    ]

    def iteration_us(self):
        """Device time per iteration (first FG_TRACE_MAX), in microseconds."""
        if self.clock_khz <= 0:
            return []
        k = min(self.iterations, FG_TRACE_MAX)
        t = [self.t_start] + list(self.t_end[:k])
        return [(t[i + 1] - t[i]) * 1000.0 / self.clock_khz for i in range(k)]

    def trace(self):
        k = min(self.iterations, FG_TRACE_MAX)
        return (list(self.dir[:k]), list(self.frontier[:k]), list(self.inspected[:k]))


class BfsOpts(ctypes.Structure):
    _fields_ = [
        ("mode", ctypes.c_int32),
        ("do_a_num", ctypes.c_uint32),
        ("do_a_den", ctypes.c_uint32),
        ("do_b_num", ctypes.c_uint32),
        ("do_b_den", ctypes.c_uint32),
        ("small_frontier", ctypes.c_int32),
        ("small_edges", ctypes.c_int32),
        ("big_degree", ctypes.c_int32),
        ("blocks_per_cu", ctypes.c_int32),
        ("team_blocks", ctypes.c_int32),
        ("team_edges", ctypes.c_int32),
        ("async_levels", ctypes.c_int32),
        ("grid_blocks", ctypes.c_int32),
    ]


class SsspOpts(ctypes.Structure):
    _fields_ = [
        ("small_frontier", ctypes.c_int32),
        ("small_edges", ctypes.c_int32),
        ("big_degree", ctypes.c_int32),
        ("blocks_per_cu", ctypes.c_int32),
        ("grid_blocks", ctypes.c_int32),
        ("delta", ctypes.c_uint32),
        ("team_blocks", ctypes.c_int32),
        ("team_edges", ctypes.c_int32),
    ]


class MsOpts(ctypes.Structure):
    _fields_ = [
        ("big_degree", ctypes.c_int32),
        ("pull_div", ctypes.c_int32),
        ("push_div", ctypes.c_int32),
        ("blocks_per_cu", ctypes.c_int32),
        ("grid_blocks", ctypes.c_int32),
        ("team_blocks", ctypes.c_int32),
        ("team_edges", ctypes.c_int32),
    ]


class MpOpts(ctypes.Structure):
    _fields_ = [
        ("delta", ctypes.c_uint32),
        ("big_degree", ctypes.c_int32),
        ("blocks_per_cu", ctypes.c_int32),
        ("grid_blocks", ctypes.c_int32),
        ("dense_lanes", ctypes.c_int32),
        ("split_lanes", ctypes.c_int32),
        ("split_wait", ctypes.c_int32),
        ("team_blocks", ctypes.c_int32),
        ("team_edges", ctypes.c_int32),
    ]


class GraphInfo(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("has_weights", ctypes.c_int32),
        ("m", ctypes.c_int64),
        ("symmetric", ctypes.c_int32),
        ("max_degree", ctypes.c_int32),
        ("nonzero_degree", ctypes.c_int32),
        ("device", ctypes.c_int32),
        ("resident_bytes", ctypes.c_int64),
    ]


class ShareInfo(ctypes.Structure):
    _fields_ = [
        ("n_global", ctypes.c_int32),
        ("n_local", ctypes.c_int32),
        ("n_total", ctypes.c_int32),
        ("nparts", ctypes.c_int32),
        ("part", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("m_local", ctypes.c_int64),
    ]


class DupInfo(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("nparts", ctypes.c_int32),
        ("part", ctypes.c_int32),
        ("hosted", ctypes.c_int32),
        ("m_local", ctypes.c_int64),
        ("m_total", ctypes.c_int64),
        ("resident_bytes", ctypes.c_int64),
    ]


class PeerBufs(ctypes.Structure):
    _fields_ = [
        ("ids", ctypes.c_void_p),
        ("depth", ctypes.c_void_p),
        ("parent", ctypes.c_void_p),
        ("counts", ctypes.c_void_p),
        ("local", ctypes.c_void_p),
        ("local_count", ctypes.c_void_p),
        ("capacity", ctypes.c_int64),
    ]


_lib = None

# Every symbol declared in include/fg.h, with (restype, argtypes).
_P = ctypes.c_void_p
_I32, _I64, _U32, _SZ = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_size_t
SIGNATURES = {
    "fg_last_error": (ctypes.c_char_p, []),
    "fg_version": (ctypes.c_char_p, []),
    "fg_graph_create_csr": (_I32, [_I32, _I64, _P, _P, _P, _U32, _P, ctypes.POINTER(_P)]),
    "fg_graph_destroy": (_I32, [_P]),
    "fg_graph_info": (_I32, [_P, ctypes.POINTER(GraphInfo)]),
    "fg_workspace_bytes": (_SZ, [_P, _I32, _I32]),
    "fg_stats_read": (_I32, [_P, ctypes.POINTER(RunStats), _P]),
    "fg_bfs_opts_default": (None, [ctypes.POINTER(BfsOpts)]),
    "fg_bfs": (_I32, [_P, _I32, ctypes.POINTER(BfsOpts), _P, _SZ, _P, _P, _P, _P]),
    "fg_bfs_many": (_I32, [_P, _P, _I32, ctypes.POINTER(BfsOpts), _P, _SZ, _P, _P, _I64, _P, _P]),
    "fg_bfs_corun": (_I32, [_P, _P, _I32, ctypes.POINTER(BfsOpts), _P, _SZ, _P, _P, _I64, _P,
                             _P, _I32, ctypes.POINTER(BfsOpts), _P, _SZ, _P, _P, _P, _P]),
    "fg_bfs_noalloc": (_I32, [_P, _I32, ctypes.POINTER(BfsOpts), _P, _P, _P, _P]),
    "fg_sssp_opts_default": (None, [ctypes.POINTER(SsspOpts)]),
    "fg_sssp": (_I32, [_P, _I32, ctypes.POINTER(SsspOpts), _P, _SZ, _P, _P, _P, _P]),
    "fg_msbfs_opts_default": (None, [ctypes.POINTER(MsOpts)]),
    "fg_msbfs_open": (_I32, [_P, _I32, _P, _SZ, ctypes.POINTER(MsOpts), _P, ctypes.POINTER(_P)]),
    "fg_msbfs_close": (_I32, [_P]),
    "fg_msbfs_admit": (_I32, [_P, _I32, _I32]),
    "fg_msbfs_step": (_I32, [_P, _I32, _P]),
    "fg_msbfs_poll": (_I32, [_P, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(_I32), _P]),
    "fg_msbfs_read": (_I32, [_P, _I32, _P, _P]),
    "fg_msbfs_release": (_I32, [_P, _I32]),
    "fg_msbfs_counts": (_I32, [_P, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64), _P]),
    "fg_mssp_opts_default": (None, [ctypes.POINTER(MpOpts)]),
    "fg_mssp_open": (_I32, [_P, _I32, _P, _SZ, ctypes.POINTER(MpOpts), _P, ctypes.POINTER(_P)]),
    "fg_mssp_close": (_I32, [_P]),
    "fg_mssp_admit": (_I32, [_P, _I32, _I32]),
    "fg_mssp_step": (_I32, [_P, _I32, _P]),
    "fg_mssp_poll": (_I32, [_P, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(_I32), _P]),
    "fg_mssp_counts": (_I32, [_P, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64), _P]),
    "fg_mssp_read": (_I32, [_P, _I32, _P, _P]),
    "fg_mssp_release": (_I32, [_P, _I32]),
    "fg_graph_csr": (_I32, [_P, ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P)]),
    "fg_share_create": (_I32, [_I32, _I64, _P, _P, _P, _I32, _I32, _P, ctypes.POINTER(_P)]),
    "fg_share_destroy": (_I32, [_P]),
    "fg_share_info": (_I32, [_P, ctypes.POINTER(ShareInfo)]),
    "fg_share_graph": (_P, [_P]),
    "fg_share_tables": (_I32, [_P, ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P)]),
    "fg_package_workspace_bytes": (_SZ, [_P, _I32]),
    "fg_package": (_I32, [_P, _P, _I32, _P, _P, _P, ctypes.POINTER(PeerBufs), _P, _SZ, _P]),
    "fg_combine": (_I32, [_P, _P, _P, _P, _I32, _P, _P, _P, _P, _P, _P, _P]),
    "fg_share_seed": (_I32, [_P, _I32, _P, _P, _P, _P, _P, _P]),
    "fg_advance": (_I32, [_P, _P, _I32, _P, _P, _P, _I64, _P, _P, _SZ, _P]),
    "fg_filter": (_I32, [_P, _P, _P, _I64, _P, _P, _I32, _P, _P, _P, _P, _P]),
    "fg_pull_step": (_I32, [_P, _P, _P, _P, _I32, _P, _P, _P, _P, _P, _P]),
    "fg_queue_to_bitmap": (_I32, [_P, _P, _I32, _P, _P]),
    "fg_bitmap_to_queue": (_I32, [_P, _P, _P, _P, _P, _SZ, _P]),
    "fg_cc": (_I32, [_P, _P, _P, _P, _SZ, _P]),
    "fg_pagerank": (_I32, [_P, ctypes.c_double, ctypes.c_double, _I32, _P, _SZ, _P, _P, _P]),
    "fg_dup_create": (_I32, [_I32, _I64, _P, _P, _P, _I32, _I32, ctypes.POINTER(BfsOpts), _P,
                             ctypes.POINTER(_P)]),
    "fg_dup_destroy": (_I32, [_P]),
    "fg_dup_info": (_I32, [_P, ctypes.POINTER(DupInfo)]),
    "fg_dup_graph": (_P, [_P]),
    "fg_dup_seed": (_I32, [_P, _I32, _P, _P, _P, _P]),
    "fg_dup_step": (_I32, [_P, _P]),
    "fg_dup_send": (_I32, [_P, _P, _P]),
    "fg_dup_combine": (_I32, [_P, _P]),
    "fg_dup_poll": (_I32, [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32), _P]),
    "fg_dup_run": (_I32, [ctypes.POINTER(_P), _I32, _I32, ctypes.POINTER(_P), ctypes.POINTER(_P),
                          ctypes.POINTER(_P), _I32, _P]),
}


def lib():
    """The loaded libfg.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(status):
    if status != FG_OK:
        raise FGError(status, lib().fg_last_error().decode())
    return status


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def last_error():
    return lib().fg_last_error().decode()


def bfs_opts(mode=FG_MODE_DO, do_a=(1, 100), do_b=(1, 10), small_frontier=0, small_edges=0,
             big_degree=0, blocks_per_cu=0, team_blocks=0, team_edges=0, async_levels=0,
             grid_blocks=0):
    o = BfsOpts()
    lib().fg_bfs_opts_default(ctypes.byref(o))
    o.mode = mode
    o.do_a_num, o.do_a_den = do_a
    o.do_b_num, o.do_b_den = do_b
    o.small_frontier = small_frontier
    o.small_edges = small_edges
    o.big_degree = big_degree
    o.blocks_per_cu = blocks_per_cu
    o.team_blocks = team_blocks
    o.team_edges = team_edges
    o.async_levels = async_levels
    o.grid_blocks = grid_blocks
    return o


class Graph:
    """A CSR graph resident on the current GPU (fg_graph_create_csr)."""

    def __init__(self, row_offsets, col_idx, weights=None, symmetric=True, validate=True,
                 device="cuda"):
        L = lib()
        off = torch.as_tensor(row_offsets, dtype=torch.int32).to(device).contiguous()
        col = torch.as_tensor(col_idx, dtype=torch.int32).to(device).contiguous()
        w = None
        if weights is not None:
            w = torch.as_tensor(weights).view(torch.int32) if isinstance(weights, torch.Tensor) \
                else torch.from_numpy(weights.view("int32"))
            w = w.to(device).contiguous()
        self.n = off.numel() - 1
        self.m = col.numel()
        self.symmetric = bool(symmetric)
        # the library keeps its own copies (no FG_BORROW)
        flags = FG_DEVICE_PTRS | (FG_VALIDATE if validate else 0) | (FG_SYMMETRIC if symmetric else 0)
        h = ctypes.c_void_p()
        _check(L.fg_graph_create_csr(self.n, self.m, _ptr(off), _ptr(col) if self.m else _ptr(col),
                                     _ptr(w), flags, _stream(), ctypes.byref(h)))
        self.handle = h
        self.off = off
        self.col = col
        self.w = w
        self._ws = {}

    def info(self):
        i = GraphInfo()
        _check(lib().fg_graph_info(self.handle, ctypes.byref(i)))
        return i

    def workspace_bytes(self, prim=FG_PRIM_BFS, lanes=0):
        return int(lib().fg_workspace_bytes(self.handle, prim, lanes))

    def workspace(self, prim=FG_PRIM_BFS, lanes=0):
        """A cached device workspace for `prim` (one per primitive)."""
        key = (prim, lanes)
        if key not in self._ws:
            nb = self.workspace_bytes(prim, lanes)
            # zero-filled once; the library keeps it ready between calls
            self._ws[key] = torch.zeros(max(nb, 256), dtype=torch.uint8, device=self.off.device)
        return self._ws[key]

    def close(self):
        if getattr(self, "handle", None):
            lib().fg_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def new_stats(device="cuda"):
    return torch.zeros(ctypes.sizeof(RunStats), dtype=torch.uint8, device=device)


def read_stats(stats_dev, stream=None):
    s = RunStats()
    _check(lib().fg_stats_read(_ptr(stats_dev), ctypes.byref(s), _stream(stream)))
    return s


def bfs_into(g, src, depth, parent=None, opts=None, ws=None, stats=None, stream=None):
    """Enqueue fg_bfs on `stream`; outputs are caller-provided device tensors."""
    prim = FG_PRIM_BFS_UNFUSED if (opts is not None and opts.mode == FG_MODE_PUSH_UNFUSED) \
        else FG_PRIM_BFS
    ws = ws if ws is not None else g.workspace(prim)
    _check(lib().fg_bfs(g.handle, int(src), ctypes.byref(opts) if opts is not None else None,
                        _ptr(ws), ws.numel(), _ptr(depth), _ptr(parent), _ptr(stats),
                        _stream(stream)))


def bfs_many_into(g, srcs, depth, parent=None, opts=None, ws=None, stats=None, out_stride=0,
                  stream=None):
    """Enqueue fg_bfs_many: the sources of `srcs` (device int32 tensor) one
    after another in one launch; traversal j writes depth / parent +
    j * out_stride and stats + j (stats: device tensor of len(srcs) records,
    see new_stats_many)."""
    ws = ws if ws is not None else g.workspace(FG_PRIM_BFS)
    _check(lib().fg_bfs_many(g.handle, _ptr(srcs), int(srcs.numel()),
                             ctypes.byref(opts) if opts is not None else None, _ptr(ws),
                             ws.numel(), _ptr(depth), _ptr(parent), int(out_stride), _ptr(stats),
                             _stream(stream)))


def bfs_corun_into(g, srcs, depth, parent, opts, ws, stats, g2, src2, depth2, parent2, opts2,
                   ws2=None, stats2=None, out_stride=0, stream=None):
    """Enqueue fg_bfs_corun: the sources of `srcs` on g one after another (as
    bfs_many_into) and, beside them in the same launch, the asynchronous
    push query from src2 on g2 (opts2: push mode, async_levels > 1)."""
    ws = ws if ws is not None else g.workspace(FG_PRIM_BFS)
    ws2 = ws2 if ws2 is not None else g2.workspace(FG_PRIM_BFS)
    _check(lib().fg_bfs_corun(g.handle, _ptr(srcs), int(srcs.numel()),
                              ctypes.byref(opts) if opts is not None else None, _ptr(ws),
                              ws.numel(), _ptr(depth), _ptr(parent), int(out_stride), _ptr(stats),
                              g2.handle, int(src2), ctypes.byref(opts2), _ptr(ws2), ws2.numel(),
                              _ptr(depth2), _ptr(parent2), _ptr(stats2), _stream(stream)))


def new_stats_many(k, device="cuda"):
    """Device records for k traversals (fg_bfs_many)."""
    return torch.zeros(k * ctypes.sizeof(RunStats), dtype=torch.uint8, device=device)


def read_stats_many(stats_dev, k, stream=None):
    """Host copies of k device records."""
    sz = ctypes.sizeof(RunStats)
    return [read_stats(stats_dev[i * sz:(i + 1) * sz], stream) for i in range(k)]


FG_NOALLOC_SCRATCH_BYTES = 64 << 20


def bfs_noalloc_into(g, src, depth, parent=None, opts=None, stats=None, stream=None):
    """Enqueue fg_bfs_noalloc (workspace in the library's static device
    array, no allocation) on `stream`."""
    _check(lib().fg_bfs_noalloc(g.handle, int(src), ctypes.byref(opts) if opts is not None else None,
                                _ptr(depth), _ptr(parent), _ptr(stats), _stream(stream)))


def bfs(g, src, mode=FG_MODE_DO, parents=True, opts=None, **kw):
    """Run one BFS and return (depth, parent or None, RunStats) after a sync."""
    dev = g.off.device
    depth = torch.empty(g.n, dtype=torch.int32, device=dev)
    parent = torch.empty(g.n, dtype=torch.int32, device=dev) if parents else None
    stats = new_stats(dev)
    o = opts if opts is not None else bfs_opts(mode=mode, **kw)
    bfs_into(g, src, depth, parent, o, stats=stats)
    st = read_stats(stats)
    return depth, parent, st


SSSP_NO_THRESHOLD = 0xFFFFFFFF  # delta: plain frontier Bellman-Ford


def sssp_opts(small_frontier=0, small_edges=0, big_degree=0, blocks_per_cu=0, delta=0,
              grid_blocks=0, team_blocks=0, team_edges=0):
    o = SsspOpts()
    lib().fg_sssp_opts_default(ctypes.byref(o))
    o.small_frontier, o.small_edges = small_frontier, small_edges
    o.big_degree, o.blocks_per_cu = big_degree, blocks_per_cu
    o.delta, o.grid_blocks = delta, grid_blocks
    o.team_blocks, o.team_edges = team_blocks, team_edges
    return o


def sssp_into(g, src, dist, parent=None, opts=None, ws=None, stats=None, stream=None):
    """Enqueue fg_sssp on `stream` into caller-provided device tensors."""
    ws = ws if ws is not None else g.workspace(FG_PRIM_SSSP)
    _check(lib().fg_sssp(g.handle, int(src), ctypes.byref(opts) if opts is not None else None,
                         _ptr(ws), ws.numel(), _ptr(dist), _ptr(parent), _ptr(stats),
                         _stream(stream)))


def sssp(g, src, parents=True, opts=None, **kw):
    """Run one SSSP; returns (dist as int64 tensor, parent or None, RunStats)."""
    dev = g.off.device
    dist = torch.empty(g.n, dtype=torch.int32, device=dev)  # uint32 bits
    parent = torch.empty(g.n, dtype=torch.int32, device=dev) if parents else None
    stats = new_stats(dev)
    sssp_into(g, src, dist, parent, opts if opts is not None else sssp_opts(**kw), stats=stats)
    st = read_stats(stats)
    return dist.to(torch.int64) & 0xFFFFFFFF, parent, st


def advance(g, frontier, capacity=None, ws=None, len_dev=None, length=None):
    """Edge frontier (dst, src, total) of `frontier` (fg_advance).  With
    `len_dev` (device int32[1]) the length is read on the device and
    `length` (default frontier.numel()) is its upper bound."""
    dev = g.off.device
    cap = g.m if capacity is None else capacity
    dst = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    src = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    out_len = torch.zeros(1, dtype=torch.int64, device=dev)
    ws = ws if ws is not None else g.workspace(FG_PRIM_BFS_UNFUSED)
    n = frontier.numel() if length is None else int(length)
    _check(lib().fg_advance(g.handle, _ptr(frontier), n, _ptr(len_dev), _ptr(dst), _ptr(src),
                            cap, _ptr(out_len), _ptr(ws), ws.numel(), _stream()))
    return dst, src, out_len


def filter_(g, dst, src, length, visited, it, depth, parent, out_q, out_len, len_dev=None):
    _check(lib().fg_filter(g.handle, _ptr(dst), _ptr(src), int(length), _ptr(len_dev),
                           _ptr(visited), int(it), _ptr(depth), _ptr(parent), _ptr(out_q),
                           _ptr(out_len), _stream()))


def pull_step(g, frontier_bits, visited, next_bits, it, depth, parent, out_q, out_len,
              inspected=None):
    _check(lib().fg_pull_step(g.handle, _ptr(frontier_bits), _ptr(visited), _ptr(next_bits),
                              int(it), _ptr(depth), _ptr(parent), _ptr(out_q), _ptr(out_len),
                              _ptr(inspected), _stream()))


def queue_to_bitmap(g, queue, length, bits):
    _check(lib().fg_queue_to_bitmap(g.handle, _ptr(queue), int(length), _ptr(bits), _stream()))


def bitmap_to_queue(g, bits, out_q, out_len, ws=None):
    ws = ws if ws is not None else g.workspace(FG_PRIM_BFS_UNFUSED)
    _check(lib().fg_bitmap_to_queue(g.handle, _ptr(bits), _ptr(out_q), _ptr(out_len), _ptr(ws),
                                    ws.numel(), _stream()))


class Share:
    """One partition of a graph under an owner map (fg_share_create)."""

    def __init__(self, row_offsets, col_idx, owner, nparts, part):
        import numpy as np
        L = lib()
        off = np.ascontiguousarray(row_offsets, dtype=np.int32)
        col = np.ascontiguousarray(col_idx, dtype=np.int32)
        own = np.ascontiguousarray(owner, dtype=np.uint8)
        h = ctypes.c_void_p()
        _check(L.fg_share_create(len(off) - 1, len(col), off.ctypes.data, col.ctypes.data,
                                 own.ctypes.data, nparts, part, _stream(), ctypes.byref(h)))
        self.handle = h
        i = ShareInfo()
        _check(L.fg_share_info(h, ctypes.byref(i)))
        self.n_local, self.n_total, self.nparts, self.part = i.n_local, i.n_total, i.nparts, i.part
        self.m_local = i.m_local
        self.graph_handle = L.fg_share_graph(h)

    def tables(self):
        """(owner uint8, conv int32, l2g int32) copied to host numpy arrays."""
        import numpy as np
        po, pc, pl = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        _check(lib().fg_share_tables(self.handle, ctypes.byref(po), ctypes.byref(pc),
                                     ctypes.byref(pl)))
        torch.cuda.synchronize()
        out = []
        for p, dt, sz in ((po, np.uint8, 1), (pc, np.int32, 4), (pl, np.int32, 4)):
            a = np.empty(self.n_total, dt)
            _memcpy_d2h(a, p.value, self.n_total * sz)
            out.append(a)
        return tuple(out)

    def csr(self):
        """The share's local CSR (row_offsets, cols) copied to host numpy arrays."""
        return graph_csr(self.graph_handle, self.n_total, self.m_local)

    def workspace(self, max_len):
        nb = int(lib().fg_package_workspace_bytes(self.handle, int(max_len)))
        return torch.zeros(max(nb, 256), dtype=torch.uint8, device="cuda")

    def close(self):
        if getattr(self, "handle", None):
            lib().fg_share_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _memcpy_d2h(dst_np, src_dev_ptr, nbytes):
    """Copy device memory owned by the library into a host numpy array."""
    rt = ctypes.CDLL("libamdhip64.so.7")
    rt.hipMemcpy.restype = ctypes.c_int
    rt.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    err = rt.hipMemcpy(ctypes.c_void_p(dst_np.ctypes.data), ctypes.c_void_p(src_dev_ptr),
                       nbytes, 2)  # hipMemcpyDeviceToHost
    if err != 0:
        raise RuntimeError(f"hipMemcpy failed ({err})")


def package(share, frontier, length, depth, parent=None, capacity=None, ws=None, len_dev=None):
    """fg_package: returns device tensors (ids, depth, parent, counts, local, local_count).
    With `len_dev` (device int32[1]) the length is read on the device and
    `length` is its upper bound."""
    cap = int(capacity if capacity is not None else max(length, 1))
    P = share.nparts
    dev = "cuda"
    ids = torch.full((P * cap,), -7, dtype=torch.int32, device=dev)
    dep = torch.full((P * cap,), -7, dtype=torch.int32, device=dev)
    par = torch.full((P * cap,), -7, dtype=torch.int32, device=dev) if parent is not None else None
    counts = torch.zeros(P, dtype=torch.int32, device=dev)
    local = torch.full((cap,), -7, dtype=torch.int32, device=dev)
    lc = torch.zeros(1, dtype=torch.int32, device=dev)
    bufs = PeerBufs(ids.data_ptr(), dep.data_ptr(), par.data_ptr() if par is not None else None,
                    counts.data_ptr(), local.data_ptr(), lc.data_ptr(), cap)
    ws = ws if ws is not None else share.workspace(length)
    _check(lib().fg_package(share.handle, _ptr(frontier), int(length), _ptr(len_dev), _ptr(depth),
                            _ptr(parent), ctypes.byref(bufs), _ptr(ws), ws.numel(), _stream()))
    return ids, dep, par, counts, local, lc


def graph_csr(handle, n, m):
    """Host copies of a graph's device CSR arrays (fg_graph_csr)."""
    import numpy as np
    po, pc, pw = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
    _check(lib().fg_graph_csr(handle, ctypes.byref(po), ctypes.byref(pc), ctypes.byref(pw)))
    torch.cuda.synchronize()
    off = np.empty(n + 1, np.int32)
    col = np.empty(m, np.int32)
    _memcpy_d2h(off, po.value, 4 * (n + 1))
    if m:
        _memcpy_d2h(col, pc.value, 4 * m)
    return off, col


def msbfs_opts(big_degree=0, pull_div=0, push_div=0, blocks_per_cu=0, grid_blocks=0,
               team_blocks=0, team_edges=0):
    o = MsOpts()
    lib().fg_msbfs_opts_default(ctypes.byref(o))
    o.big_degree, o.pull_div, o.push_div, o.blocks_per_cu = big_degree, pull_div, push_div, blocks_per_cu
    o.grid_blocks, o.team_blocks, o.team_edges = grid_blocks, team_blocks, team_edges
    return o


class MsBatch:
    """Up to 64 BFS queries sharing one traversal (fg_msbfs_*)."""

    def __init__(self, g, lanes=64, opts=None, stream=None):
        self.g = g
        self.lanes = lanes
        nb = g.workspace_bytes(FG_PRIM_MSBFS, lanes)
        self.ws = torch.zeros(max(nb, 256), dtype=torch.uint8, device=g.off.device)
        h = ctypes.c_void_p()
        o = opts if opts is not None else msbfs_opts()
        _check(lib().fg_msbfs_open(g.handle, lanes, _ptr(self.ws), self.ws.numel(),
                                   ctypes.byref(o), _stream(stream), ctypes.byref(h)))
        self.handle = h
        self.admitted = 0

    def admit(self, lane, src):
        _check(lib().fg_msbfs_admit(self.handle, int(lane), int(src)))
        self.admitted |= 1 << int(lane)

    def step(self, k_iters, stream=None):
        _check(lib().fg_msbfs_step(self.handle, int(k_iters), _stream(stream)))

    def poll(self, stream=None):
        done = ctypes.c_uint64()
        it = ctypes.c_int32()
        _check(lib().fg_msbfs_poll(self.handle, ctypes.byref(done), ctypes.byref(it),
                                   _stream(stream)))
        return int(done.value), int(it.value)

    def read(self, lane, out=None, stream=None):
        out = out if out is not None else torch.empty(self.g.n, dtype=torch.int32,
                                                      device=self.g.off.device)
        _check(lib().fg_msbfs_read(self.handle, int(lane), _ptr(out), _stream(stream)))
        return out

    def release(self, lane):
        _check(lib().fg_msbfs_release(self.handle, int(lane)))
        self.admitted &= ~(1 << int(lane))

    def counts(self, stream=None):
        """(adjacency entries read, vertex visits) since open."""
        e = ctypes.c_uint64()
        v = ctypes.c_uint64()
        _check(lib().fg_msbfs_counts(self.handle, ctypes.byref(e), ctypes.byref(v),
                                     _stream(stream)))
        return int(e.value), int(v.value)

    def run(self, k_iters=16, max_steps=1 << 20):
        """Step until every admitted lane is done; returns the done mask."""
        for _ in range(max_steps):
            self.step(k_iters)
            done, _ = self.poll()
            if done & self.admitted == self.admitted:
                return done
        raise RuntimeError("msbfs did not finish")

    def close(self):
        if getattr(self, "handle", None):
            lib().fg_msbfs_close(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mssp_opts(delta=0, big_degree=0, blocks_per_cu=0, dense_lanes=0, grid_blocks=0,
              split_lanes=0, split_wait=0, team_blocks=0, team_edges=0):
    o = MpOpts()
    lib().fg_mssp_opts_default(ctypes.byref(o))
    o.delta, o.big_degree, o.blocks_per_cu = delta, big_degree, blocks_per_cu
    o.dense_lanes, o.grid_blocks = dense_lanes, grid_blocks
    o.split_lanes, o.split_wait = split_lanes, split_wait
    o.team_blocks, o.team_edges = team_blocks, team_edges
    return o


class MsspBatch:
    """Up to 64 SSSP queries sharing one traversal (fg_mssp_*)."""

    def __init__(self, g, lanes=64, opts=None, stream=None):
        self.g = g
        self.lanes = lanes
        nb = g.workspace_bytes(FG_PRIM_MSSSP, lanes)
        self.ws = torch.zeros(max(nb, 256), dtype=torch.uint8, device=g.off.device)
        h = ctypes.c_void_p()
        o = opts if opts is not None else mssp_opts()
        _check(lib().fg_mssp_open(g.handle, lanes, _ptr(self.ws), self.ws.numel(),
                                  ctypes.byref(o), _stream(stream), ctypes.byref(h)))
        self.handle = h
        self.admitted = 0

    def admit(self, lane, src):
        _check(lib().fg_mssp_admit(self.handle, int(lane), int(src)))
        self.admitted |= 1 << int(lane)

    def step(self, k_iters, stream=None):
        _check(lib().fg_mssp_step(self.handle, int(k_iters), _stream(stream)))

    def poll(self, stream=None):
        done = ctypes.c_uint64()
        it = ctypes.c_int32()
        _check(lib().fg_mssp_poll(self.handle, ctypes.byref(done), ctypes.byref(it),
                                  _stream(stream)))
        return int(done.value), int(it.value)

    def counts(self, stream=None):
        e = ctypes.c_uint64()
        el = ctypes.c_uint64()
        _check(lib().fg_mssp_counts(self.handle, ctypes.byref(e), ctypes.byref(el),
                                    _stream(stream)))
        return int(e.value), int(el.value)

    def read(self, lane, out=None, stream=None):
        """Lane's distances as an int32 tensor holding the uint32 bits."""
        out = out if out is not None else torch.empty(self.g.n, dtype=torch.int32,
                                                      device=self.g.off.device)
        _check(lib().fg_mssp_read(self.handle, int(lane), _ptr(out), _stream(stream)))
        return out

    def release(self, lane):
        _check(lib().fg_mssp_release(self.handle, int(lane)))
        self.admitted &= ~(1 << int(lane))

    def run(self, k_iters=64, max_steps=1 << 20):
        """Step until every admitted lane is done; returns the done mask."""
        for _ in range(max_steps):
            self.step(k_iters)
            done, _ = self.poll()
            if done & self.admitted == self.admitted:
                return done
        raise RuntimeError("batched SSSP did not finish")

    def close(self):
        if getattr(self, "handle", None):
            lib().fg_mssp_close(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def combine(graph_handle, ids, labels, parents, length, visited, depth, parent, out_q, out_len,
            len_dev=None):
    """fg_combine on the graph handle (e.g. Share.graph_handle)."""
    _check(lib().fg_combine(graph_handle, _ptr(ids), _ptr(labels), _ptr(parents), int(length),
                            _ptr(len_dev), _ptr(visited), _ptr(depth), _ptr(parent), _ptr(out_q),
                            _ptr(out_len), _stream()))


def _op_handle(g):
    return g.handle if isinstance(g, Graph) else g


def cc_into(g, label, components=None, ws=None, stream=None):
    """Enqueue fg_cc: label (device int32[n]) receives the smallest vertex id
    of each vertex's component; components (device int64[1] or None) the
    number of components."""
    ws = ws if ws is not None else g.workspace(FG_PRIM_CC)
    _check(lib().fg_cc(g.handle, _ptr(label), _ptr(components), _ptr(ws), ws.numel(),
                       _stream(stream)))


def cc(g):
    """Connected components after a sync: (labels, number of components)."""
    label = torch.empty(g.n, dtype=torch.int32, device=g.off.device)
    comps = torch.zeros(1, dtype=torch.int64, device=g.off.device)
    cc_into(g, label, comps)
    torch.cuda.synchronize()
    return label, int(comps.item())


def pagerank_into(g, rank, damping=0.85, tol=0.0, max_iter=20, ws=None, stats=None, stream=None):
    """Enqueue fg_pagerank: rank (device float64[n]) receives the ranks."""
    ws = ws if ws is not None else g.workspace(FG_PRIM_PR)
    _check(lib().fg_pagerank(g.handle, float(damping), float(tol), int(max_iter), _ptr(ws),
                             ws.numel(), _ptr(rank), _ptr(stats), _stream(stream)))


def pagerank(g, damping=0.85, tol=0.0, max_iter=20):
    """PageRank after a sync: (ranks as a float64 tensor, RunStats)."""
    rank = torch.empty(g.n, dtype=torch.float64, device=g.off.device)
    stats = new_stats(g.off.device)
    pagerank_into(g, rank, damping, tol, max_iter, stats=stats)
    return rank, read_stats(stats)


class DupBfs:
    """Direction-optimizing BFS over `nparts` duplicate-all partitions with
    broadcast communication (fg_dup_*), all on the current GPU: one fg_dup
    per partition, each with its own depth array and trace; the partitions
    share one parent array."""

    def __init__(self, row_offsets, col_idx, owner, nparts, do_a=(1, 100), do_b=(1, 10),
                 stream=None):
        import numpy as np
        L = lib()
        off = np.ascontiguousarray(row_offsets, dtype=np.int32)
        col = np.ascontiguousarray(col_idx, dtype=np.int32)
        own = np.ascontiguousarray(owner, dtype=np.uint8)
        o = bfs_opts(mode=FG_MODE_DO, do_a=do_a, do_b=do_b)
        self.n = len(off) - 1
        self.nparts = nparts
        self.handles = []
        for p in range(nparts):
            h = ctypes.c_void_p()
            _check(L.fg_dup_create(self.n, len(col), off.ctypes.data,
                                   col.ctypes.data if len(col) else None, own.ctypes.data,
                                   nparts, p, ctypes.byref(o), _stream(stream), ctypes.byref(h)))
            self.handles.append(h)
        self.depth = [torch.empty(self.n, dtype=torch.int32, device="cuda") for _ in range(nparts)]
        self.parent = torch.empty(self.n, dtype=torch.int32, device="cuda")
        self.stats = [new_stats() for _ in range(nparts)]

    def info(self, p):
        i = DupInfo()
        _check(lib().fg_dup_info(self.handles[p], ctypes.byref(i)))
        return i

    def run(self, src, poll_every=4, stream=None):
        """The whole traversal (fg_dup_run); enqueued on `stream`, whose
        stop-flag reads synchronise it."""
        P = self.nparts
        hs = (_P * P)(*[h.value for h in self.handles])
        ds = (_P * P)(*[d.data_ptr() for d in self.depth])
        ps = (_P * P)(*([self.parent.data_ptr()] * P))
        ss = (_P * P)(*[s.data_ptr() for s in self.stats])
        _check(lib().fg_dup_run(hs, P, int(src), ds, ps, ss, int(poll_every), _stream(stream)))

    # the per-iteration calls, for callers that drive the rounds themselves
    def seed(self, src, stream=None):
        for p in range(self.nparts):
            _check(lib().fg_dup_seed(self.handles[p], int(src), _ptr(self.depth[p]),
                                     _ptr(self.parent), _ptr(self.stats[p]), _stream(stream)))

    def round(self, stream=None):
        L, sp = lib(), _stream(stream)
        for h in self.handles:
            _check(L.fg_dup_step(h, sp))
        for p, hp in enumerate(self.handles):
            for q, hq in enumerate(self.handles):
                if p != q:
                    _check(L.fg_dup_send(hp, hq, sp))
        for h in self.handles:
            _check(L.fg_dup_combine(h, sp))

    def poll(self, p=0, stream=None):
        done, it = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().fg_dup_poll(self.handles[p], ctypes.byref(done), ctypes.byref(it),
                                 _stream(stream)))
        return bool(done.value), int(it.value)

    def read_stats(self, p, stream=None):
        return read_stats(self.stats[p], stream)

    def close(self):
        for h in getattr(self, "handles", []):
            if h:
                lib().fg_dup_destroy(h)
        self.handles = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
