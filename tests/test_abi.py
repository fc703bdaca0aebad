"""C ABI checks that need no GPU: every symbol of include/fg.h is exported,
and argument errors are reported synchronously with the documented codes."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "fg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fg_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def fg():
    import paper_1504_04804_amd as fg
    return fg


def test_header_symbols_exported(fg):
    L = fg.lib()
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), f"{name} declared in fg.h but not exported"
    # the binding knows every declared symbol
    assert set(names) <= set(fg.SIGNATURES), set(names) - set(fg.SIGNATURES)


def test_argument_errors_without_gpu(fg):
    L = fg.lib()
    h = ctypes.c_void_p()
    assert L.fg_graph_create_csr(0, 0, None, None, None, 0, None, ctypes.byref(h)) == fg.FG_EINVAL
    assert "n=0" in fg.last_error()
    assert L.fg_graph_create_csr(4, -1, None, None, None, 0, None, ctypes.byref(h)) == fg.FG_EINVAL
    assert L.fg_graph_create_csr(4, 1 << 31, None, None, None, 0, None, ctypes.byref(h)) == fg.FG_EINVAL
    assert L.fg_graph_create_csr(4, 3, None, None, None, 0, None, ctypes.byref(h)) == fg.FG_EINVAL
    arr = (ctypes.c_int32 * 8)()
    assert L.fg_graph_create_csr(4, 3, arr, arr, None, fg.FG_BORROW, None,
                                 ctypes.byref(h)) == fg.FG_EINVAL
    assert L.fg_graph_create_csr(4, 3, arr, arr, None, 0, None, None) == fg.FG_EINVAL
    assert L.fg_bfs(None, 0, None, None, 0, None, None, None, None) == fg.FG_EINVAL
    assert L.fg_workspace_bytes(None, 0, 0) == 0
    assert L.fg_advance(None, None, 0, None, None, None, 0, None, None, 0, None) == fg.FG_EINVAL
    assert L.fg_filter(None, None, None, 0, None, None, 0, None, None, None, None, None) == fg.FG_EINVAL
    assert L.fg_stats_read(None, None, None) == fg.FG_EINVAL
    assert L.fg_graph_destroy(None) == fg.FG_OK
    assert fg.lib().fg_version().decode().count(".") == 2


def test_new_entry_points_argument_errors(fg):
    import numpy as np
    L = fg.lib()
    h = ctypes.c_void_p()
    off = np.array([0, 1, 2], np.int32)
    col = np.array([1, 0], np.int32)
    own = np.array([0, 1], np.uint8)
    P = lambda a: a.ctypes.data
    # share: bad n, bad nparts / part, owner out of range (all before any HIP call)
    assert L.fg_share_create(0, 0, P(off), P(col), P(own), 2, 0, None, ctypes.byref(h)) == fg.FG_EINVAL
    assert L.fg_share_create(2, 2, P(off), P(col), P(own), 0, 0, None, ctypes.byref(h)) == fg.FG_EINVAL
    assert L.fg_share_create(2, 2, P(off), P(col), P(own), 2, 2, None, ctypes.byref(h)) == fg.FG_EINVAL
    assert L.fg_share_create(2, 2, P(off), P(col), P(own), 17, 0, None, ctypes.byref(h)) == fg.FG_EINVAL
    bad_own = np.array([0, 3], np.uint8)
    assert L.fg_share_create(2, 2, P(off), P(col), P(bad_own), 2, 0, None, ctypes.byref(h)) == fg.FG_EINVAL
    assert "owner" in fg.last_error()
    bad_off = np.array([0, 1, 3], np.int32)
    assert L.fg_share_create(2, 2, P(bad_off), P(col), P(own), 2, 0, None, ctypes.byref(h)) == fg.FG_EINVAL
    assert L.fg_share_destroy(None) == fg.FG_OK
    assert L.fg_package(None, None, 0, None, None, None, None, None, 0, None) == fg.FG_EINVAL
    assert L.fg_combine(None, None, None, None, 0, None, None, None, None, None, None,
                        None) == fg.FG_EINVAL
    assert L.fg_share_seed(None, 0, None, None, None, None, None, None) == fg.FG_EINVAL
    assert L.fg_bfs_noalloc(None, 0, None, None, None, None, None) == fg.FG_EINVAL
    assert L.fg_package_workspace_bytes(None, 10) == 0
    # sssp / batched BFS
    assert L.fg_sssp(None, 0, None, None, 0, None, None, None, None) == fg.FG_EINVAL
    assert L.fg_msbfs_open(None, 64, None, 0, None, None, ctypes.byref(h)) == fg.FG_EINVAL
    assert L.fg_msbfs_admit(None, 0, 0) == fg.FG_EINVAL
    assert L.fg_msbfs_step(None, 1, None) == fg.FG_EINVAL
    assert L.fg_msbfs_read(None, 0, None, None) == fg.FG_EINVAL
    assert L.fg_msbfs_close(None) == fg.FG_OK
    assert L.fg_graph_csr(None, None, None, None) == fg.FG_EINVAL
    assert L.fg_share_graph(None) is None


def test_dup_argument_errors_without_gpu(fg):
    import numpy as np
    L = fg.lib()
    h = ctypes.c_void_p()
    off = np.array([0, 1, 2], np.int32)
    col = np.array([1, 0], np.int32)
    own = np.array([0, 1], np.uint8)
    p = lambda a: a.ctypes.data  # noqa: E731
    assert L.fg_dup_create(2, 2, p(off), p(col), p(own), 0, 0, None, None,
                           ctypes.byref(h)) == fg.FG_EINVAL
    assert L.fg_dup_create(2, 2, p(off), p(col), p(own), 2, 2, None, None,
                           ctypes.byref(h)) == fg.FG_EINVAL
    assert L.fg_dup_create(2, 2, p(off), p(col), p(own), 1, 0, None, None,
                           ctypes.byref(h)) == fg.FG_EINVAL
    assert "owner" in fg.last_error()
    bad = np.array([0, 2, 1], np.int32)
    assert L.fg_dup_create(2, 2, p(bad), p(col), p(own), 2, 0, None, None,
                           ctypes.byref(h)) == fg.FG_EINVAL
    assert L.fg_dup_create(2, 2, p(off), p(col), p(own), 2, 0, None, None, None) == fg.FG_EINVAL
    assert L.fg_dup_step(None, None) == fg.FG_EINVAL
    assert L.fg_dup_send(None, None, None) == fg.FG_EINVAL
    assert L.fg_dup_combine(None, None) == fg.FG_EINVAL
    assert L.fg_dup_seed(None, 0, None, None, None, None) == fg.FG_EINVAL
    assert L.fg_dup_poll(None, None, None, None) == fg.FG_EINVAL
    assert L.fg_dup_info(None, None) == fg.FG_EINVAL
    assert L.fg_dup_run(None, 0, 0, None, None, None, 0, None) == fg.FG_EINVAL
    assert L.fg_dup_destroy(None) == fg.FG_OK


def test_corun_argument_errors_without_gpu(fg):
    """fg_bfs_corun checks its second query first, then the list, before any
    device work."""
    L = fg.lib()
    o2 = fg.bfs_opts(mode=fg.FG_MODE_PUSH, async_levels=8)
    rc = L.fg_bfs_corun(None, None, 0, None, None, 0, None, None, 0, None,
                        None, 0, ctypes.byref(o2), None, 0, None, None, None, None)
    assert rc == fg.FG_EINVAL
    assert "fg_bfs_corun" in fg.last_error() and "graph is NULL" in fg.last_error()


def test_serving_single_query_options(fg):
    """Both serving paths run a single BFS with the same options: the
    asynchronous push team on graphs of mean degree <= 8, direction-optimizing
    on other undirected graphs, push on directed ones."""
    from paper_1504_04804_amd import serve

    class G:
        def __init__(self, n, m, symmetric):
            self.n, self.m, self.symmetric = n, m, symmetric

    o = serve.single_bfs_opts(G(100, 360, True))
    assert o.mode == fg.FG_MODE_PUSH and o.async_levels == 64 and o.team_blocks == 64
    o = serve.single_bfs_opts(G(100, 800, True))
    assert o.mode == fg.FG_MODE_PUSH and o.async_levels == 64
    o = serve.single_bfs_opts(G(100, 3000, True))
    assert o.mode == fg.FG_MODE_DO and o.async_levels == 0
    o = serve.single_bfs_opts(G(100, 3000, False))
    assert o.mode == fg.FG_MODE_PUSH and o.async_levels == 0
