"""Serial CPU oracle (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU path:
the C source ``oracle.c`` is built with gcc into ``oracle/liborc.so`` and
wrapped here with ctypes over numpy arrays.

Pins (what fixes each function independently of itself) are listed in the
test modules ``tests/test_oracle_pins.py`` and ``tests/test_oracle_pins_next.py``.
Parity unpinned: none of the
functions below; the R-MAT generator that feeds them (``synth``) is pinned
only by determinism and a dedup-survival sanity bound.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liborc.so")
_lib = None

PUSH, PULL = 0, 1
INF32 = 0xFFFFFFFF


def build_cmd(src=None, out=None):
    return ["gcc", "-O2", "-fPIC", "-shared", "-std=gnu11",
            src or os.path.join(_HERE, "oracle.c"), "-o", out or _LIB_PATH]


def load(path=None):
    """Load the oracle library (or a variant built at `path`, for mutation tests)."""
    global _lib
    if path is None and _lib is not None:
        return _lib
    p = path or _LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(p)
    P = ctypes.c_void_p
    i32, i64, u32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    lib.orc_csr_from_edges.restype = i64
    lib.orc_csr_from_edges.argtypes = [i32, i64, P, P, P, P]
    lib.orc_bfs.restype = i32
    lib.orc_bfs.argtypes = [i32, P, P, i32, P, P, P, P]
    lib.orc_do_schedule.restype = i32
    lib.orc_do_schedule.argtypes = [i32, P, i64, i64, u32, u32, u32, u32, P]
    lib.orc_edges_inspected.restype = None
    lib.orc_edges_inspected.argtypes = [i32, P, P, P, i32, P, P]
    lib.orc_dijkstra.restype = i32
    lib.orc_dijkstra.argtypes = [i32, P, P, P, i32, P, P]
    lib.orc_floyd_warshall.restype = None
    lib.orc_floyd_warshall.argtypes = [i32, P, P, P, P]
    lib.orc_check_bfs.restype = i32
    lib.orc_check_bfs.argtypes = [i32, P, P, i32, P, P, ctypes.c_char_p, i32]
    lib.orc_check_sssp.restype = i32
    lib.orc_check_sssp.argtypes = [i32, P, P, P, i32, P, P, ctypes.c_char_p, i32]
    lib.orc_share_build.restype = i64
    lib.orc_share_build.argtypes = [i32, P, P, P, i32, P, P, P, P, P, P, P]
    lib.orc_package.restype = None
    lib.orc_package.argtypes = [i32, P, i32, P, P, P, P, P, i32, i32, P, P, P, P, P, P]
    lib.orc_bfs_partitioned.restype = i32
    lib.orc_bfs_partitioned.argtypes = [i32, P, P, P, i32, i32, P]
    lib.orc_dobfs_dupall.restype = i32
    lib.orc_dobfs_dupall.argtypes = [i32, P, P, P, i32, i32, u32, u32, u32, u32, P, P]
    lib.orc_cc.restype = i32
    lib.orc_cc.argtypes = [i32, P, P, P]
    lib.orc_pagerank.restype = i32
    lib.orc_pagerank.argtypes = [i32, P, P, ctypes.c_double, ctypes.c_double, i32, P]
    if path is None:
        _lib = lib
    return lib


def _csr(off, col):
    return (np.ascontiguousarray(off, np.int32), np.ascontiguousarray(col, np.int32))


class Oracle:
    """Thin numpy front end; `lib` may be a mutated build in mutation tests."""

    def __init__(self, lib=None):
        self.lib = lib or load()

    @staticmethod
    def _p(a):
        return None if a is None else ctypes.c_void_p(a.ctypes.data)

    def csr_from_edges(self, n, eu, ev):
        eu = np.ascontiguousarray(eu, np.int32)
        ev = np.ascontiguousarray(ev, np.int32)
        off = np.empty(n + 1, np.int32)
        cols = np.empty(max(2 * len(eu), 1), np.int32)
        m = self.lib.orc_csr_from_edges(n, len(eu), self._p(eu), self._p(ev),
                                        self._p(off), self._p(cols))
        return off, cols[:m].copy()

    def bfs(self, off, col, src):
        """Returns (depth, parent, level_cnt, m_comp)."""
        off, col = _csr(off, col)
        n = len(off) - 1
        depth = np.empty(n, np.int32)
        parent = np.empty(n, np.int32)
        cnt = np.empty(max(n, 1), np.int64)
        mc = np.zeros(1, np.int64)
        levels = self.lib.orc_bfs(n, self._p(off), self._p(col), int(src),
                                  self._p(depth), self._p(parent), self._p(cnt),
                                  self._p(mc))
        return depth, parent, cnt[:levels].copy(), int(mc[0])

    def do_schedule(self, level_cnt, n, m, do_a=(1, 100), do_b=(1, 10)):
        level_cnt = np.ascontiguousarray(level_cnt, np.int64)
        L = len(level_cnt)
        d = np.empty(max(L, 1), np.int8)
        self.lib.orc_do_schedule(L, self._p(level_cnt), int(n), int(m),
                                 do_a[0], do_a[1], do_b[0], do_b[1], self._p(d))
        return d[:L].copy()

    def edges_inspected(self, off, col, depth, dirs):
        off, col = _csr(off, col)
        n = len(off) - 1
        dirs = np.ascontiguousarray(dirs, np.int8)
        out = np.empty(max(len(dirs), 1), np.int64)
        depth = np.ascontiguousarray(depth, np.int32)
        self.lib.orc_edges_inspected(n, self._p(off), self._p(col), self._p(depth),
                                     len(dirs), self._p(dirs), self._p(out))
        return out[:len(dirs)].copy()

    def dijkstra(self, off, col, w, src):
        off, col = _csr(off, col)
        n = len(off) - 1
        dist = np.empty(n, np.uint32)
        parent = np.empty(n, np.int32)
        w = np.ascontiguousarray(w, np.uint32)
        rc = self.lib.orc_dijkstra(n, self._p(off), self._p(col), self._p(w),
                                   int(src), self._p(dist), self._p(parent))
        if rc != 0:
            raise OverflowError("shortest-path weight does not fit in uint32")
        return dist, parent

    def floyd_warshall(self, off, col, w=None):
        off, col = _csr(off, col)
        n = len(off) - 1
        D = np.empty(n * n, np.uint64)
        wp = None if w is None else np.ascontiguousarray(w, np.uint32)
        self.lib.orc_floyd_warshall(n, self._p(off), self._p(col), self._p(wp),
                                    self._p(D))
        return D.reshape(n, n)

    def check_bfs(self, off, col, src, depth, parent=None):
        off, col = _csr(off, col)
        n = len(off) - 1
        buf = ctypes.create_string_buffer(256)
        depth = np.ascontiguousarray(depth, np.int32)
        parent = None if parent is None else np.ascontiguousarray(parent, np.int32)
        rc = self.lib.orc_check_bfs(n, self._p(off), self._p(col), int(src),
                                    self._p(depth), self._p(parent), buf, 256)
        return None if rc == 0 else buf.value.decode()

    def check_sssp(self, off, col, w, src, dist, parent=None):
        off, col = _csr(off, col)
        n = len(off) - 1
        buf = ctypes.create_string_buffer(256)
        w = np.ascontiguousarray(w, np.uint32)
        dist = np.ascontiguousarray(dist, np.uint32)
        parent = None if parent is None else np.ascontiguousarray(parent, np.int32)
        rc = self.lib.orc_check_sssp(n, self._p(off), self._p(col), self._p(w),
                                     int(src), self._p(dist), self._p(parent),
                                     buf, 256)
        return None if rc == 0 else buf.value.decode()

    def share_build(self, off, col, owner, part):
        """Returns dict with n_local, n_total, off, col, owner, conv, l2g."""
        off, col = _csr(off, col)
        n = len(off) - 1
        m = len(col)
        nl = np.zeros(1, np.int32)
        nt = np.zeros(1, np.int32)
        loff = np.empty(n + 1, np.int32)
        lcol = np.empty(max(m, 1), np.int32)
        lown = np.empty(max(n, 1), np.uint8)
        lconv = np.empty(max(n, 1), np.int32)
        l2g = np.empty(max(n, 1), np.int32)
        owner = np.ascontiguousarray(owner, np.uint8)
        lm = self.lib.orc_share_build(n, self._p(off), self._p(col), self._p(owner),
                                      int(part), self._p(nl), self._p(nt),
                                      self._p(loff), self._p(lcol), self._p(lown),
                                      self._p(lconv), self._p(l2g))
        t = int(nt[0])
        return dict(n_local=int(nl[0]), n_total=t, off=loff[:t + 1].copy(),
                    col=lcol[:lm].copy(), owner=lown[:t].copy(),
                    conv=lconv[:t].copy(), l2g=l2g[:t].copy())

    def package(self, frontier, n_local, owner, conv, depth, parent=None,
                l2g=None, nparts=4):
        frontier = np.ascontiguousarray(frontier, np.int32)
        L = len(frontier)
        cap = max(L, 1)
        ids = np.full(nparts * cap, -7, np.int32)
        dep = np.full(nparts * cap, -7, np.int32)
        par = np.full(nparts * cap, -7, np.int32) if parent is not None else None
        counts = np.zeros(nparts, np.int32)
        local = np.empty(cap, np.int32)
        lc = np.zeros(1, np.int32)
        owner = np.ascontiguousarray(owner, np.uint8)
        conv = np.ascontiguousarray(conv, np.int32)
        depth = np.ascontiguousarray(depth, np.int32)
        parent = None if parent is None else np.ascontiguousarray(parent, np.int32)
        l2g = None if l2g is None else np.ascontiguousarray(l2g, np.int32)
        self.lib.orc_package(L, self._p(frontier), int(n_local), self._p(owner),
                             self._p(conv), self._p(depth), self._p(parent),
                             self._p(l2g), nparts, cap, self._p(ids), self._p(dep), self._p(par),
                             self._p(counts), self._p(local), self._p(lc))
        bufs = []
        for p in range(nparts):
            c = int(counts[p])
            s = slice(p * cap, p * cap + c)
            bufs.append(dict(ids=ids[s].copy(), depth=dep[s].copy(),
                             parent=None if par is None else par[s].copy()))
        return bufs, local[:int(lc[0])].copy()

    def bfs_partitioned(self, off, col, owner, nparts, src):
        off, col = _csr(off, col)
        n = len(off) - 1
        depth = np.empty(n, np.int32)
        owner = np.ascontiguousarray(owner, np.uint8)
        self.lib.orc_bfs_partitioned(n, self._p(off), self._p(col), self._p(owner),
                                     nparts, int(src), self._p(depth))
        return depth


    def dobfs_dupall(self, off, col, owner, nparts, src, do_a=(1, 100), do_b=(1, 10)):
        """O11: returns (depth, direction trace, iterations); raises if the
        partitions' labels disagree."""
        off, col = _csr(off, col)
        n = len(off) - 1
        depth = np.empty(n, np.int32)
        dirs = np.zeros(max(n, 1), np.int8)
        owner = np.ascontiguousarray(owner, np.uint8)
        it = self.lib.orc_dobfs_dupall(n, self._p(off), self._p(col), self._p(owner), nparts,
                                       int(src), do_a[0], do_a[1], do_b[0], do_b[1],
                                       self._p(depth), self._p(dirs))
        if it < 0:
            raise AssertionError("partitions disagree on the labels")
        return depth, dirs[:it].copy(), it

    def cc(self, off, col):
        """O12: (label = smallest vertex id of the component, number of components)."""
        off, col = _csr(off, col)
        n = len(off) - 1
        label = np.empty(n, np.int32)
        c = self.lib.orc_cc(n, self._p(off), self._p(col), self._p(label))
        return label, int(c)

    def pagerank(self, off, col, damping=0.85, tol=0.0, max_iter=20):
        """O13: (rank float64[n], iterations run)."""
        off, col = _csr(off, col)
        n = len(off) - 1
        rank = np.empty(n, np.float64)
        it = self.lib.orc_pagerank(n, self._p(off), self._p(col), float(damping), float(tol),
                                   int(max_iter), self._p(rank))
        return rank, int(it)


_default = None


def oracle():
    global _default
    if _default is None:
        _default = Oracle()
    return _default
