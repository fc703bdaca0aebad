"""Multi-partition BFS (Alg. 1) emulated on one GPU.

All `nparts` shares (duplicate-1-hop, random owners) live on the same device.
Per iteration every share runs the advance and filter operators on its
frontier (fg_advance, fg_filter), splits and packages its output frontier
(fg_package), and each receiving share combines the buffers addressed to it
(fg_combine): a received vertex that is not yet visited takes the received
label and joins that share's next frontier.  The loop ends when every
frontier is empty (the global stop condition).  Device-to-device reads of
the peers' buffers stand in for the inter-GPU pushes.

Every frontier length stays on the device: each operator reads its input
length from device memory (the `len_dev` arguments) with a host-side upper
bound, and the source is set by fg_share_seed.  The host reads the next
frontier lengths of all shares once per iteration, for the stop test, and
does no arithmetic of the method.  This is the device side of the paper's
multi-GPU loop on one GPU, a correctness emulation rather than a
performance path (every launch is sized for the share's whole vertex set).
"""
import ctypes

import numpy as np
import torch

import paper_1504_04804_amd as fg


class _Part:
    def __init__(self, share, dev):
        self.s = share
        nt, ml = share.n_total, max(share.m_local, 1)
        self.visited = torch.zeros((nt + 31) // 32 + 1, dtype=torch.int32, device=dev)
        self.depth = torch.full((nt,), -1, dtype=torch.int32, device=dev)
        self.qin = torch.empty(max(nt, 1), dtype=torch.int32, device=dev)
        self.qout = torch.empty(max(nt, 1), dtype=torch.int32, device=dev)
        self.edst = torch.empty(ml, dtype=torch.int32, device=dev)
        self.esrc = torch.empty(ml, dtype=torch.int32, device=dev)
        self.etot = torch.zeros(1, dtype=torch.int64, device=dev)
        self.out_len = torch.zeros(1, dtype=torch.int32, device=dev)
        nb = int(fg.lib().fg_workspace_bytes(share.graph_handle, fg.FG_PRIM_BFS_UNFUSED, 0))
        self.ws = torch.zeros(max(nb, 256), dtype=torch.uint8, device=dev)
        self.pws = share.workspace(nt)
        P = share.nparts
        self.cap = max(nt, 1)
        self.ids = torch.empty(P * self.cap, dtype=torch.int32, device=dev)
        self.dep = torch.empty(P * self.cap, dtype=torch.int32, device=dev)
        self.counts = torch.zeros(P, dtype=torch.int32, device=dev)


class PartitionedBFS:
    def __init__(self, row_offsets, col_idx, owner, nparts, device="cuda"):
        self.owner = np.ascontiguousarray(owner, np.uint8)
        self.nparts = nparts
        self.n = len(row_offsets) - 1
        self.parts = [_Part(fg.Share(row_offsets, col_idx, self.owner, nparts, p), device)
                      for p in range(nparts)]
        self.l2g = [p.s.tables()[2] for p in self.parts]
        # frontier lengths of every share, two rows used alternately as the
        # input and the next length of an iteration
        self.lens = torch.zeros((2, nparts), dtype=torch.int32, device=device)

    def run(self, src):
        """Global depths (numpy int32[n]) and the number of iterations."""
        L = fg.lib()
        stream = fg._stream()
        P = self.nparts
        lens = self.lens
        row = 0
        for i, p in enumerate(self.parts):
            fg._check(L.fg_share_seed(p.s.handle, int(src), fg._ptr(p.visited), fg._ptr(p.depth),
                                      None, fg._ptr(p.qin), fg._ptr(lens[row, i]), stream))
        it = 0
        while True:
            cur, nxt = lens[row], lens[row ^ 1]
            for i, p in enumerate(self.parts):
                g = p.s.graph_handle
                # local advance + filter on the share's input frontier
                fg._check(L.fg_advance(g, fg._ptr(p.qin), p.cap, fg._ptr(cur[i]), fg._ptr(p.edst),
                                       fg._ptr(p.esrc), p.edst.numel(), fg._ptr(p.etot),
                                       fg._ptr(p.ws), p.ws.numel(), stream))
                fg._check(L.fg_filter(g, fg._ptr(p.edst), fg._ptr(p.esrc), p.edst.numel(),
                                      fg._ptr(p.etot), fg._ptr(p.visited), it, fg._ptr(p.depth),
                                      None, fg._ptr(p.qout), fg._ptr(p.out_len), stream))
                # split + package; the local sub-frontier becomes the next
                # input (written over the consumed one), its length the
                # share's next length, which the combines below extend
                bufs = fg.PeerBufs(p.ids.data_ptr(), p.dep.data_ptr(), None, p.counts.data_ptr(),
                                   p.qin.data_ptr(), nxt[i].data_ptr(), p.cap)
                fg._check(L.fg_package(p.s.handle, fg._ptr(p.qout), p.cap, fg._ptr(p.out_len),
                                       fg._ptr(p.depth), None, ctypes.byref(bufs), fg._ptr(p.pws),
                                       p.pws.numel(), stream))
            # each share combines what the others packaged for it
            for i, p in enumerate(self.parts):
                for j, q in enumerate(self.parts):
                    if j == i:
                        continue
                    off = j * p.cap
                    fg._check(L.fg_combine(q.s.graph_handle, fg._ptr(p.ids[off:]),
                                           fg._ptr(p.dep[off:]), None, p.cap,
                                           fg._ptr(p.counts[j:]), fg._ptr(q.visited),
                                           fg._ptr(q.depth), None, fg._ptr(q.qin),
                                           fg._ptr(nxt[j:]), stream))
            it += 1
            # the global stop condition: one read-back per iteration
            if not nxt.cpu().numpy().any():
                break
            row ^= 1
        out = np.full(self.n, -1, np.int32)
        for p, l2g in zip(self.parts, self.l2g):
            nl = p.s.n_local
            out[l2g[:nl]] = p.depth[:nl].cpu().numpy()
        return out, it
