"""Multi-partition BFS (Alg. 1) emulated on one GPU.

All `nparts` shares (duplicate-1-hop, random owners) live on the same device.
Per iteration every share runs the advance and filter operators on its
frontier (fg_advance, fg_filter), splits and packages its output frontier
(fg_package), and each receiving share combines the buffers addressed to it
(fg_combine): a received vertex that is not yet visited takes the received
label and joins that share's next frontier.  The loop ends when every
frontier is empty (the global stop condition).  Device-to-device reads of
the peers' buffers stand in for the inter-GPU pushes.

This is the device side of the paper's multi-GPU loop; it is a correctness
emulation driven from the host (one synchronisation per share and
iteration), not a performance path.
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
        self.q = [torch.empty(max(nt, 1), dtype=torch.int32, device=dev) for _ in range(2)]
        self.qlen = 0
        self.edst = torch.empty(ml, dtype=torch.int32, device=dev)
        self.esrc = torch.empty(ml, dtype=torch.int32, device=dev)
        self.etot = torch.zeros(1, dtype=torch.int64, device=dev)
        self.out_len = torch.zeros(1, dtype=torch.int32, device=dev)
        self.next_len = torch.zeros(1, dtype=torch.int32, device=dev)
        nb = int(fg.lib().fg_workspace_bytes(share.graph_handle, fg.FG_PRIM_BFS_UNFUSED, 0))
        self.ws = torch.zeros(max(nb, 256), dtype=torch.uint8, device=dev)
        self.pws = share.workspace(nt)
        P = share.nparts
        self.cap = max(nt, 1)
        self.ids = torch.empty(P * self.cap, dtype=torch.int32, device=dev)
        self.dep = torch.empty(P * self.cap, dtype=torch.int32, device=dev)
        self.counts = torch.zeros(P, dtype=torch.int32, device=dev)
        self.lcount = torch.zeros(1, dtype=torch.int32, device=dev)


class PartitionedBFS:
    def __init__(self, row_offsets, col_idx, owner, nparts, device="cuda"):
        self.owner = np.ascontiguousarray(owner, np.uint8)
        self.nparts = nparts
        self.n = len(row_offsets) - 1
        self.parts = [_Part(fg.Share(row_offsets, col_idx, self.owner, nparts, p), device)
                      for p in range(nparts)]
        self.l2g = [p.s.tables()[2] for p in self.parts]

    def run(self, src):
        """Global depths (numpy int32[n]) and the number of iterations."""
        L = fg.lib()
        stream = fg._stream()
        for p in self.parts:
            p.visited.zero_()
            p.depth.fill_(-1)
            p.qlen = 0
        sp = int(self.owner[src])
        tsrc = int(np.count_nonzero(self.owner[:src] == sp))
        P0 = self.parts[sp]
        P0.depth[tsrc] = 0
        P0.visited[tsrc >> 5] = int(np.int32(np.uint32(1 << (tsrc & 31))))
        P0.q[0][0] = tsrc
        P0.qlen = 1
        sel = 0
        it = 0
        while any(p.qlen for p in self.parts):
            # local advance + filter, then split + package
            for p in self.parts:
                if p.qlen:
                    fg._check(L.fg_advance(p.s.graph_handle, fg._ptr(p.q[sel]), p.qlen,
                                           fg._ptr(p.edst), fg._ptr(p.esrc), p.edst.numel(),
                                           fg._ptr(p.etot), fg._ptr(p.ws), p.ws.numel(), stream))
                    torch.cuda.synchronize()
                    ne = int(p.etot.item())
                    fg._check(L.fg_filter(p.s.graph_handle, fg._ptr(p.edst), fg._ptr(p.esrc), ne,
                                          fg._ptr(p.visited), it, fg._ptr(p.depth), None,
                                          fg._ptr(p.q[sel ^ 1]), fg._ptr(p.out_len), stream))
                    torch.cuda.synchronize()
                    nout = int(p.out_len.item())
                else:
                    nout = 0
                bufs = fg.PeerBufs(p.ids.data_ptr(), p.dep.data_ptr(), None, p.counts.data_ptr(),
                                   p.q[sel].data_ptr(), p.lcount.data_ptr(), p.cap)
                # the local sub-frontier is written over the consumed input queue
                fg._check(L.fg_package(p.s.handle, fg._ptr(p.q[sel ^ 1]), nout,
                                       fg._ptr(p.depth), None, ctypes.byref(bufs),
                                       fg._ptr(p.pws), p.pws.numel(), stream))
            torch.cuda.synchronize()
            # combine what each share received; local sub-frontier first
            for q in self.parts:
                q.next_len.copy_(q.lcount)
            for p in self.parts:
                counts = p.counts.cpu().numpy()
                for qi, q in enumerate(self.parts):
                    c = int(counts[qi])
                    if qi == p.s.part or c == 0:
                        continue
                    off = qi * p.cap
                    fg._check(L.fg_combine(q.s.graph_handle, fg._ptr(p.ids[off:off + c]),
                                           fg._ptr(p.dep[off:off + c]), None, c,
                                           fg._ptr(q.visited), fg._ptr(q.depth), None,
                                           fg._ptr(q.q[sel]), fg._ptr(q.next_len), stream))
            torch.cuda.synchronize()
            for q in self.parts:
                q.qlen = int(q.next_len.item())
            it += 1
        out = np.full(self.n, -1, np.int32)
        for p, l2g in zip(self.parts, self.l2g):
            nl = p.s.n_local
            out[l2g[:nl]] = p.depth[:nl].cpu().numpy()
        return out, it
