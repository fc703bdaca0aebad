// Multi-GPU direction-optimizing BFS with duplicate-all vertices and
// broadcast communication (Alg. 2; the duplicate-all vertex model and the
// broadcast strategy of Sec. III-C; the newly-discovered set as the
// direction-independent view of Sec. VI-A), one partition per fg_dup.
//
// Every partition holds all n vertices under their global ids but only the
// rows of the vertices it hosts.  One iteration on partition p:
//   step     the direction rule of Sec. VI-A from the global counts (the
//            same on every partition), then either a forward step over the
//            hosted frontier vertices' rows (advance + visited test-and-set)
//            or a backward step over the hosted unvisited vertices (scan
//            the row, stop at the first neighbour already labelled).  Its
//            output is the partition's newly-discovered set, the message:
//            an id list after a forward step (sparse), a bitmap of n bits
//            after a backward step (dense).
//   send     the broadcast leg: the message is copied into a receive slot
//            of every other partition (on one GPU a device copy stands in
//            for the transfer over the GPU links).
//   combine  received vertices not yet labelled take the next depth; the
//            union of all messages is the next frontier, kept as the list
//            of its hosted vertices (list iterations) or as a bitmap
//            (bitmap iterations); the last workgroup advances the control
//            block (counts, direction state, trace, convergence).
// The host enqueues step / send / combine for every partition per
// iteration without reading anything back: directions, lengths and the
// stop flag live in device memory, and kernels of a finished traversal
// return at once.
#include <string.h>

#include <vector>

#include "fg_common.h"

namespace {

typedef unsigned long long ull;
typedef unsigned __int128 u128;

constexpr int DUP_BT = 256;       // threads per workgroup
constexpr int DUP_WAVES = DUP_BT / FG_WAVE;
constexpr int DUP_BIG = 4096;     // forward: rows at least this long go to the chunked pass
constexpr int DUP_CHUNK = 1024;   // row entries per workgroup task in that pass
constexpr int MSG_LIST = 0, MSG_BITS = 1;
constexpr int DIR_FWD = 0, DIR_BWD = 1;

struct DupCtl {
  int32_t k;            // iteration: level of the input frontier
  int32_t cur;          // direction of iteration k (written by the step)
  int32_t prev;         // direction of iteration k - 1
  int32_t switched;     // the forward -> backward switch has been taken
  int32_t ffmt;         // frontier held as MSG_LIST (fq[sel]) or MSG_BITS (fbits)
  int32_t sel;          // list buffer holding the frontier
  int32_t flen;         // its length
  int32_t nflen;        // entries appended to the other list buffer
  int32_t done;         // traversal finished
  int32_t big_len;      // forward: rows deferred to the chunked pass
  uint32_t blocks_done; // combine: workgroups finished (the last one advances)
  int32_t status;
  int64_t qcount;       // |Q_k|, global
  int64_t pcount;       // |P|: labelled vertices, frontier included
  int64_t recv_new;     // combine: vertices it labelled (list) / union size (bitmap)
  int64_t inspected;    // CSR entries read by this partition in iteration k
  int64_t insp_total;
};

struct MsgHdr {
  int32_t fmt;    // MSG_LIST or MSG_BITS
  int32_t pad;
  int64_t count;  // vertices in the message
};

struct DupArgs {
  int32_t n, nwords, part, nparts;
  int64_t m_total;
  const int32_t* off;
  const int32_t* col;
  const uint64_t* nz;  // hosted vertices with a nonempty row
  DupCtl* ctl;
  MsgHdr* hdr;         // outgoing message header
  MsgHdr* rhdr;        // received headers, slot = sender
  uint64_t* visited;
  uint64_t* fbits;     // frontier bitmap after bitmap iterations
  uint64_t* mbits;     // outgoing bitmap message
  uint64_t* rbits;     // received bitmaps, nparts slots of bits_stride words
  int64_t ids_stride;  // slot strides, multiples of 64 entries (16-byte
  int64_t bits_stride; //   aligned slots for the vector copies)
  int32_t* fq0;
  int32_t* fq1;
  int32_t* mids;       // outgoing id list
  int32_t* rids;       // received lists, nparts slots of ids_stride entries
  int32_t* big;        // forward: deferred long rows
  int32_t* depth;
  int32_t* parent;
  fg_run_stats* stats;
  uint32_t a_num, a_den, b_num, b_den;
  int32_t clock_khz;
};

// Sec. VI-A direction rule with FV = |Q| m / n and BV = |U| n / |P| under
// duplicate-all (|V_i| = n, |E_i| summed over the partitions = m), compared
// exactly in 128-bit integers: forward first, forward -> backward at most
// once when FV > do_a BV, backward -> forward when FV < do_b BV.
__device__ __forceinline__ int32_t dup_direction(const DupCtl& c, const DupArgs& A) {
  if (c.k == 0) return DIR_FWD;
  const u128 lhs = (u128)(ull)c.qcount * (ull)A.m_total * (ull)c.pcount;
  const u128 rhs = (u128)(ull)((int64_t)A.n - c.pcount) * (ull)A.n * (ull)A.n;
  if (c.prev == DIR_FWD) return (!c.switched && lhs * A.a_den > rhs * A.a_num) ? DIR_BWD : DIR_FWD;
  return (lhs * A.b_den < rhs * A.b_num) ? DIR_FWD : DIR_BWD;
}

__device__ __forceinline__ void load_ctl(const DupCtl* C, DupCtl* s) {
  if (threadIdx.x == 0) *s = *C;
  __syncthreads();
}

__device__ __forceinline__ bool hosted(const DupArgs& A, int32_t v) {
  return (A.nz[v >> 6] >> (v & 63)) & 1ull;
}

// Wave-aggregated append of `keep` lanes' x to out[atomicAdd(counter)].
template <class CT>
__device__ __forceinline__ void wave_append(bool keep, int32_t x, CT* counter, int32_t* out) {
  const uint64_t mask = __ballot(keep);
  if (!mask) return;
  CT pos = 0;
  if (fg_lane() == 0) pos = atomicAdd(counter, (CT)__popcll(mask));
  pos = __shfl(pos, 0, FG_WAVE);
  if (keep) out[pos + fg_mbcnt(mask)] = x;
}

// Forward visit of v (or nothing for v < 0) from frontier vertex pu: the
// visited test-and-set (filter), then depth / parent for the winner, which
// joins the outgoing message and, if this partition hosts its row, the
// next frontier list.
__device__ __forceinline__ void fwd_visit(const DupArgs& A, int32_t v, int32_t pu, int32_t d_new,
                                          int32_t* nq) {
  bool won = false;
  if (v >= 0) {
    uint32_t* wp = (uint32_t*)A.visited + (v >> 5);
    const uint32_t bit = 1u << (v & 31);
    if (!(*wp & bit)) won = !(atomicOr(wp, bit) & bit);
    if (won) {
      A.depth[v] = d_new;
      if (A.parent) A.parent[v] = pu;
    }
  }
  wave_append(won, v, (unsigned long long*)&A.hdr->count, A.mids);
  wave_append(won ? hosted(A, v) : false, v, &A.ctl->nflen, nq);
}

// ------------------------------------------------------------------ seed

__global__ __launch_bounds__(DUP_BT) void dup_seed_kernel(DupArgs A, int32_t src) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = tid; v < A.n; v += nth) {
    A.depth[v] = v == src ? 0 : -1;
    if (A.parent) A.parent[v] = v == src ? src : -1;
  }
  for (int64_t w = tid; w < A.nwords; w += nth)
    A.visited[w] = (w == (src >> 6)) ? (1ull << (src & 63)) : 0ull;
  if (tid == 0) {
    DupCtl c;
    memset(&c, 0, sizeof(c));
    c.ffmt = MSG_LIST;
    c.qcount = 1;
    c.pcount = 1;
    if (hosted(A, src)) {
      A.fq0[0] = src;
      c.flen = 1;
    }
    *A.ctl = c;
    A.hdr->fmt = MSG_LIST;
    A.hdr->count = 0;
    if (A.stats) {
      fg_run_stats* st = A.stats;
      st->status = FG_OK;
      st->iterations = 0;
      st->reached = 1;
      st->edges_inspected = 0;
      st->direction_switches = 0;
      st->grid_blocks = gridDim.x;
      st->clock_khz = A.clock_khz;
      st->t_start = (int64_t)wall_clock64();
    }
  }
}

// ------------------------------------------------------------------ step

__global__ __launch_bounds__(DUP_BT) void dup_step_kernel(DupArgs A) {
  __shared__ DupCtl sc;
  __shared__ int32_t s_incl[DUP_WAVES][FG_WAVE];
  __shared__ int32_t s_row[DUP_WAVES][FG_WAVE];
  __shared__ int32_t s_src[DUP_WAVES][FG_WAVE];
  load_ctl(A.ctl, &sc);
  if (sc.done) return;
  const int32_t dir = dup_direction(sc, A);
  const int lane = fg_lane();
  const int wid = threadIdx.x / FG_WAVE;
  const int64_t gwave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / FG_WAVE;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / FG_WAVE;
  const int32_t d_new = sc.k + 1;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    A.ctl->cur = dir;
    A.hdr->fmt = dir == DIR_BWD ? MSG_BITS : MSG_LIST;
  }
  int64_t insp = 0;
  if (dir == DIR_FWD) {
    const bool from_list = sc.ffmt == MSG_LIST;
    const int32_t* q = sc.sel ? A.fq1 : A.fq0;
    int32_t* nq = sc.sel ? A.fq0 : A.fq1;
    const int64_t items = from_list ? ((int64_t)sc.flen + FG_WAVE - 1) / FG_WAVE : A.nwords;
    for (int64_t it = gwave; it < items; it += nwaves) {
      // up to 64 frontier vertices per wave: 64 list entries or one bitmap word
      int32_t u = -1;
      if (from_list) {
        const int64_t i = it * FG_WAVE + lane;
        if (i < sc.flen) u = q[i];
      } else {
        const uint64_t bits = A.fbits[it] & A.nz[it];
        if ((bits >> lane) & 1ull) u = (int32_t)(it * FG_WAVE + lane);
      }
      int32_t b = 0, deg = 0;
      if (u >= 0) {
        b = A.off[u];
        deg = A.off[u + 1] - b;
      }
      // long rows: the chunked pass, every workgroup a share of each
      wave_append(deg >= DUP_BIG, u, &A.ctl->big_len, A.big);
      // medium rows: one at a time, the whole wave across the row
      uint64_t med = __ballot(deg >= FG_WAVE && deg < DUP_BIG);
      while (med) {
        const int l = __builtin_ctzll(med);
        med &= med - 1;
        const int32_t ub = __shfl(b, l, FG_WAVE);
        const int32_t ud = __shfl(deg, l, FG_WAVE);
        const int32_t uu = __shfl(u, l, FG_WAVE);
        for (int32_t e0 = 0; e0 < ud; e0 += FG_WAVE) {
          const int32_t e = e0 + lane;
          fwd_visit(A, e < ud ? A.col[ub + e] : -1, uu, d_new, nq);
        }
        insp += (lane == 0) ? ud : 0;
      }
      // short rows: scan-gather, 64 row entries of the wave's rows per round
      const int32_t sd = deg < FG_WAVE ? deg : 0;
      const int32_t incl = fg_wave_incl_scan(sd);
      const int32_t total = __shfl(incl, FG_WAVE - 1, FG_WAVE);
      if (total == 0) continue;
      s_incl[wid][lane] = incl;
      s_row[wid][lane] = b;
      s_src[wid][lane] = u;
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      for (int32_t t0 = 0; t0 < total; t0 += FG_WAVE) {
        const int32_t t = t0 + lane;
        int32_t v = -1, pu = -1;
        if (t < total) {
          // owner: the first lane whose inclusive sum exceeds t
          int32_t lo = 0, hi = FG_WAVE - 1;
          while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            if (s_incl[wid][mid] > t) hi = mid; else lo = mid + 1;
          }
          const int32_t ex = lo ? s_incl[wid][lo - 1] : 0;
          pu = s_src[wid][lo];
          v = A.col[s_row[wid][lo] + (t - ex)];
        }
        fwd_visit(A, v, pu, d_new, nq);
      }
      insp += (lane == 0) ? total : 0;
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
  } else {
    // backward: hosted unvisited vertices scan their rows for a neighbour
    // labelled k.  Every labelled vertex has depth <= k and an unlabelled
    // one depth >= k + 1, so a labelled neighbour has depth exactly k: the
    // visited bitmap is the frontier test.  visited is not changed here
    // (the combine adds the union), so every row sees level k only.
    int64_t cnt = 0;
    for (int64_t w = gwave; w < A.nwords; w += nwaves) {
      const uint64_t cand = A.nz[w] & ~A.visited[w];
      uint64_t nb = 0;
      if (cand) {
        const int32_t v = (int32_t)(w * FG_WAVE + lane);
        bool found = false;
        int32_t pu = -1;
        if ((cand >> lane) & 1ull) {
          // four entries per step, their column and visited-word loads in
          // flight together (a row is otherwise a chain of dependent
          // loads); the entries read still stop at the first hit
          const int32_t e = A.off[v + 1];
          for (int32_t i0 = A.off[v]; i0 < e && !found; i0 += 4) {
            int32_t u[4];
            uint64_t wv[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) u[k] = A.col[i0 + k < e ? i0 + k : e - 1];
#pragma unroll
            for (int k = 0; k < 4; ++k) wv[k] = A.visited[u[k] >> 6];
            int32_t h = -1;
#pragma unroll
            for (int k = 3; k >= 0; --k)
              if (i0 + k < e && ((wv[k] >> (u[k] & 63)) & 1ull)) h = k;
            if (h >= 0) {
              found = true;
              pu = u[h];
              insp += h + 1;
            } else {
              insp += e - i0 < 4 ? e - i0 : 4;
            }
          }
        }
        nb = __ballot(found);
        if (found) {
          A.depth[v] = d_new;
          if (A.parent) A.parent[v] = pu;
        }
      }
      if (lane == 0) {
        A.mbits[w] = nb;
        cnt += __popcll(nb);
      }
    }
    cnt = fg_wave_sum(cnt);
    if (lane == 0 && cnt) atomicAdd((ull*)&A.hdr->count, (ull)cnt);
  }
  insp = fg_wave_sum(insp);
  if (lane == 0 && insp) atomicAdd((ull*)&A.ctl->inspected, (ull)insp);
}

// Forward rows of at least DUP_BIG entries, cut into DUP_CHUNK-entry tasks
// dealt round-robin over the workgroups (task numbering continues across
// rows, so short lists of long rows still spread over the grid).
__global__ __launch_bounds__(DUP_BT) void dup_big_kernel(DupArgs A) {
  __shared__ DupCtl sc;
  load_ctl(A.ctl, &sc);
  if (sc.done || sc.cur != DIR_FWD || sc.big_len == 0) return;
  int32_t* nq = sc.sel ? A.fq0 : A.fq1;
  const int32_t d_new = sc.k + 1;
  const int lane = fg_lane();
  int64_t base = 0, insp = 0;
  for (int32_t i = 0; i < sc.big_len; ++i) {
    const int32_t u = A.big[i];
    const int32_t b = A.off[u];
    const int32_t deg = A.off[u + 1] - b;
    const int64_t ntask = (deg + DUP_CHUNK - 1) / DUP_CHUNK;
    int64_t first = ((int64_t)blockIdx.x - base) % (int64_t)gridDim.x;
    if (first < 0) first += gridDim.x;
    for (int64_t t = first; t < ntask; t += gridDim.x) {
      const int32_t e_end = (int32_t)((t + 1) * DUP_CHUNK < deg ? (t + 1) * DUP_CHUNK : deg);
      for (int32_t e0 = (int32_t)(t * DUP_CHUNK); e0 < e_end; e0 += DUP_BT) {
        const int32_t e = e0 + threadIdx.x;
        fwd_visit(A, e < e_end ? A.col[b + e] : -1, u, d_new, nq);
        insp += e < e_end;
      }
    }
    base += ntask;
  }
  insp = fg_wave_sum(insp);
  if (lane == 0 && insp) atomicAdd((ull*)&A.ctl->inspected, (ull)insp);
}

// ------------------------------------------------------------------ send

__global__ __launch_bounds__(DUP_BT) void dup_send_kernel(const DupCtl* __restrict__ sctl,
                                                          const MsgHdr* __restrict__ hdr,
                                                          const int32_t* __restrict__ ids,
                                                          const uint64_t* __restrict__ bits,
                                                          int32_t nwords, MsgHdr* dhdr,
                                                          int32_t* __restrict__ dids,
                                                          uint64_t* __restrict__ dbits) {
  if (sctl->done) return;
  const MsgHdr h = *hdr;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  if (tid == 0) *dhdr = h;
  if (h.fmt == MSG_LIST) {
    const int64_t n4 = h.count / 4;
    for (int64_t i = tid; i < n4; i += nth) ((int4*)dids)[i] = ((const int4*)ids)[i];
    for (int64_t i = n4 * 4 + tid; i < h.count; i += nth) dids[i] = ids[i];
  } else {
    const int64_t n2 = nwords / 2;
    for (int64_t i = tid; i < n2; i += nth) ((int4*)dbits)[i] = ((const int4*)bits)[i];
    for (int64_t i = n2 * 2 + tid; i < nwords; i += nth) dbits[i] = bits[i];
  }
}

// --------------------------------------------------------------- combine

__global__ __launch_bounds__(DUP_BT) void dup_combine_kernel(DupArgs A) {
  __shared__ DupCtl sc;
  __shared__ int s_last;
  load_ctl(A.ctl, &sc);
  if (sc.done) return;
  const int lane = fg_lane();
  const int64_t gwave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / FG_WAVE;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / FG_WAVE;
  const int32_t d_new = sc.k + 1;
  const int32_t fmt = sc.cur == DIR_BWD ? MSG_BITS : MSG_LIST;
  int64_t cnt = 0;
  if (fmt == MSG_LIST) {
    int32_t* nq = sc.sel ? A.fq0 : A.fq1;
    for (int32_t q = 0; q < A.nparts; ++q) {
      if (q == A.part) continue;
      const int64_t len = A.rhdr[q].count;
      const int32_t* ids = A.rids + (int64_t)q * A.ids_stride;
      for (int64_t i0 = gwave * FG_WAVE; i0 < len; i0 += nwaves * FG_WAVE) {
        const int64_t i = i0 + lane;
        bool won = false;
        int32_t v = -1;
        if (i < len) {
          v = ids[i];
          uint32_t* wp = (uint32_t*)A.visited + (v >> 5);
          const uint32_t bit = 1u << (v & 31);
          if (!(*wp & bit)) won = !(atomicOr(wp, bit) & bit);
          if (won) A.depth[v] = d_new;
        }
        cnt += won;
        wave_append(won ? hosted(A, v) : false, v, &A.ctl->nflen, nq);
      }
    }
  } else {
    // 64 words per wave: lane l ORs word w0 + l of every message; then the
    // wave writes the depths of each word's received vertices, lane b
    // taking bit b (one coalesced row of 64 depths per word).
    for (int64_t w0 = gwave * FG_WAVE; w0 < A.nwords; w0 += nwaves * FG_WAVE) {
      const int64_t w = w0 + lane;
      uint64_t newr = 0;
      if (w < A.nwords) {
        const uint64_t own = A.mbits[w];
        uint64_t un = own;
        for (int32_t q = 0; q < A.nparts; ++q)
          if (q != A.part) un |= A.rbits[(int64_t)q * A.bits_stride + w];
        const uint64_t vis = A.visited[w];
        newr = un & ~own & ~vis;
        A.visited[w] = vis | un;
        A.fbits[w] = un;
        cnt += __popcll(un);
      }
      const int32_t nw = (int32_t)((A.nwords - w0) < FG_WAVE ? (A.nwords - w0) : FG_WAVE);
      for (int32_t j = 0; j < nw; ++j) {
        const ull r = fg_readlane64(newr, j);
        if (r && ((r >> lane) & 1ull)) A.depth[(w0 + j) * FG_WAVE + lane] = d_new;
      }
    }
  }
  cnt = fg_wave_sum(cnt);
  if (lane == 0 && cnt) atomicAdd((ull*)&A.ctl->recv_new, (ull)cnt);

  // the last workgroup to finish advances the control block
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0)
    s_last = atomicAdd(&A.ctl->blocks_done, 1u) == gridDim.x - 1;
  __syncthreads();
  if (!s_last || threadIdx.x != 0) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  DupCtl* C = A.ctl;
  const int64_t own = __hip_atomic_load(&A.hdr->count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const int64_t recv = __hip_atomic_load(&C->recv_new, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const int64_t insp = __hip_atomic_load(&C->inspected, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const int32_t nflen = __hip_atomic_load(&C->nflen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const int64_t newq = fmt == MSG_LIST ? own + recv : recv;
  const int32_t k = sc.k;
  if (A.stats) {
    fg_run_stats* st = A.stats;
    if (k < FG_TRACE_MAX) {
      st->dir[k] = (int8_t)sc.cur;
      st->frontier[k] = sc.qcount;
      st->inspected[k] = insp;
      st->t_end[k] = (int64_t)wall_clock64();
    }
    st->edges_inspected += insp;
    st->reached = sc.pcount + newq;
    st->iterations = k + 1;
    if (sc.cur != sc.prev) st->direction_switches++;
  }
  C->insp_total = sc.insp_total + insp;
  C->prev = sc.cur;
  if (sc.cur == DIR_BWD) C->switched = 1;
  C->pcount = sc.pcount + newq;
  C->qcount = newq;
  if (fmt == MSG_LIST) {
    C->sel = sc.sel ^ 1;
    C->flen = nflen;
    C->ffmt = MSG_LIST;
  } else {
    C->ffmt = MSG_BITS;
  }
  C->nflen = 0;
  C->k = k + 1;
  C->done = newq == 0;
  C->recv_new = 0;
  C->inspected = 0;
  C->big_len = 0;
  A.hdr->count = 0;
  C->blocks_done = 0;
}

int dup_grid(const fg_graph* g) {
  const int cus = fg_props(g->device).cus;
  return (cus > 0 ? cus : 256) * 4;
}

}  // namespace

struct fg_dup {
  int32_t n = 0, nparts = 0, part = 0, nwords = 0;
  int64_t m_local = 0, m_total = 0;
  int32_t nhosted = 0;
  fg_graph* g = nullptr;
  void* mem = nullptr;
  DupArgs args;
  int32_t grid = 0;
  int32_t device = 0;
  int64_t resident_bytes = 0;
  bool seeded = false;
};

extern "C" fg_status fg_dup_create(int32_t n, int64_t m, const int32_t* row_offsets,
                                   const int32_t* col_idx, const uint8_t* owner, int32_t nparts,
                                   int32_t part, const fg_bfs_opts* opts, void* stream,
                                   fg_dup** out) {
  if (!out) return fg_set_error(FG_EINVAL, "fg_dup_create: out is NULL");
  *out = nullptr;
  if (n < 1 || !row_offsets || !owner || (m > 0 && !col_idx))
    return fg_set_error(FG_EINVAL, "fg_dup_create: bad graph arguments");
  if (m < 0 || m >= (int64_t(1) << 31))
    return fg_set_error(FG_EINVAL, "fg_dup_create: m=%lld outside [0, 2^31)", (long long)m);
  if (nparts < 1 || nparts > 16 || part < 0 || part >= nparts)
    return fg_set_error(FG_EINVAL, "fg_dup_create: part %d of %d (1 <= nparts <= 16)", part,
                        nparts);
  if (row_offsets[0] != 0 || (int64_t)row_offsets[n] != m)
    return fg_set_error(FG_EINVAL, "fg_dup_create: invalid CSR offsets");
  fg_bfs_opts o;
  if (opts) {
    o = *opts;
  } else {
    memset(&o, 0, sizeof(o));
    o.do_a_num = 1;
    o.do_a_den = 100;
    o.do_b_num = 1;
    o.do_b_den = 10;
  }
  if (o.do_a_den == 0 || o.do_b_den == 0)
    return fg_set_error(FG_EINVAL, "fg_dup_create: zero threshold denominator");
  // the partition's CSR: every vertex, rows of the hosted ones only
  std::vector<int32_t> poff((size_t)n + 1);
  int64_t ml = 0;
  int32_t nh = 0;
  poff[0] = 0;
  for (int32_t v = 0; v < n; ++v) {
    const int32_t a = row_offsets[v], b = row_offsets[v + 1];
    if (b < a || b > m) return fg_set_error(FG_EINVAL, "fg_dup_create: offsets not monotone at %d", v);
    if (owner[v] >= nparts)
      return fg_set_error(FG_EINVAL, "fg_dup_create: owner[%d]=%d >= nparts", v, owner[v]);
    if (owner[v] == part) {
      ml += b - a;
      nh++;
    }
    poff[v + 1] = (int32_t)ml;
  }
  std::vector<int32_t> pcol((size_t)(ml > 0 ? ml : 1));
  for (int32_t v = 0; v < n; ++v) {
    if (owner[v] != part) continue;
    const int32_t a = row_offsets[v], b = row_offsets[v + 1];
    for (int32_t i = a; i < b; ++i) {
      const int32_t c = col_idx[i];
      if (c < 0 || c >= n) return fg_set_error(FG_EINVAL, "fg_dup_create: column %d out of range", c);
      pcol[poff[v] + (i - a)] = c;
    }
  }
  fg_dup* d = new fg_dup();
  fg_status st = fg_graph_create_csr(n, ml, poff.data(), pcol.data(), nullptr, 0, stream, &d->g);
  if (st != FG_OK) {
    delete d;
    return st;
  }
  d->n = n;
  d->nparts = nparts;
  d->part = part;
  d->nwords = (n + 63) / 64;
  d->m_local = ml;
  d->m_total = m;
  d->nhosted = nh;
  hipGetDevice(&d->device);
  d->grid = dup_grid(d->g);

  // device state: one allocation
  fg_carver c(nullptr);
  const int64_t nw = d->nwords;
  const int64_t ids_stride = ((int64_t)n + 63) & ~(int64_t)63;
  const int64_t bits_stride = (nw + 63) & ~(int64_t)63;
  c.take<DupCtl>(1);
  c.take<MsgHdr>(1);
  c.take<MsgHdr>(nparts);
  c.take<uint64_t>(nw);
  c.take<uint64_t>(nw);
  c.take<uint64_t>(nw);
  c.take<uint64_t>(bits_stride * nparts);
  c.take<int32_t>(n);
  c.take<int32_t>(n);
  c.take<int32_t>(n);
  c.take<int32_t>(ids_stride * nparts);
  c.take<int32_t>(n);
  if (hipMalloc(&d->mem, c.used) != hipSuccess) {
    fg_graph_destroy(d->g);
    delete d;
    return fg_set_error(FG_ENOMEM, "fg_dup_create: hipMalloc of %zu bytes", c.used);
  }
  if (hipMemsetAsync(d->mem, 0, c.used, (hipStream_t)stream) != hipSuccess) {
    hipFree(d->mem);
    fg_graph_destroy(d->g);
    delete d;
    return fg_set_error(FG_EDEVICE, "fg_dup_create: clearing the state failed");
  }
  fg_carver k(d->mem);
  DupArgs& A = d->args;
  memset(&A, 0, sizeof(A));
  A.ctl = k.take<DupCtl>(1);
  A.hdr = k.take<MsgHdr>(1);
  A.rhdr = k.take<MsgHdr>(nparts);
  A.visited = k.take<uint64_t>(nw);
  A.fbits = k.take<uint64_t>(nw);
  A.mbits = k.take<uint64_t>(nw);
  A.rbits = k.take<uint64_t>(bits_stride * nparts);
  A.fq0 = k.take<int32_t>(n);
  A.fq1 = k.take<int32_t>(n);
  A.mids = k.take<int32_t>(n);
  A.rids = k.take<int32_t>(ids_stride * nparts);
  A.ids_stride = ids_stride;
  A.bits_stride = bits_stride;
  A.big = k.take<int32_t>(n);
  A.n = n;
  A.nwords = d->nwords;
  A.part = part;
  A.nparts = nparts;
  A.m_total = m;
  A.off = d->g->off;
  A.col = d->g->col;
  A.nz = d->g->nzmask;
  A.a_num = o.do_a_num;
  A.a_den = o.do_a_den;
  A.b_num = o.do_b_num;
  A.b_den = o.do_b_den;
  A.clock_khz = fg_props(d->device).clock_khz;
  d->resident_bytes = d->g->resident_bytes + (int64_t)c.used;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) {
    fg_dup_destroy(d);
    return fg_set_error(FG_EDEVICE, "fg_dup_create: device set-up failed");
  }
  *out = d;
  return FG_OK;
}

extern "C" fg_status fg_dup_destroy(fg_dup* d) {
  if (!d) return FG_OK;
  hipSetDevice(d->device);
  hipDeviceSynchronize();
  if (d->mem) hipFree(d->mem);
  if (d->g) fg_graph_destroy(d->g);
  delete d;
  return FG_OK;
}

extern "C" fg_status fg_dup_info(const fg_dup* d, fg_dup_info_t* info) {
  if (!d || !info) return fg_set_error(FG_EINVAL, "fg_dup_info: NULL argument");
  info->n = d->n;
  info->nparts = d->nparts;
  info->part = d->part;
  info->hosted = d->nhosted;
  info->m_local = d->m_local;
  info->m_total = d->m_total;
  info->resident_bytes = d->resident_bytes;
  return FG_OK;
}

extern "C" const fg_graph* fg_dup_graph(const fg_dup* d) { return d ? d->g : nullptr; }

extern "C" fg_status fg_dup_seed(fg_dup* d, int32_t src, int32_t* depth, int32_t* parent,
                                 fg_run_stats* stats, void* stream) {
  if (!d || !depth) return fg_set_error(FG_EINVAL, "fg_dup_seed: NULL argument");
  if (src < 0 || src >= d->n)
    return fg_set_error(FG_EINVAL, "fg_dup_seed: src=%d outside [0, %d)", src, d->n);
  d->args.depth = depth;
  d->args.parent = parent;
  d->args.stats = stats;
  d->seeded = true;
  dup_seed_kernel<<<d->grid, DUP_BT, 0, (hipStream_t)stream>>>(d->args, src);
  FG_HIP_TRY(hipGetLastError());
  return FG_OK;
}

extern "C" fg_status fg_dup_step(fg_dup* d, void* stream) {
  if (!d) return fg_set_error(FG_EINVAL, "fg_dup_step: NULL argument");
  if (!d->seeded) return fg_set_error(FG_EINVAL, "fg_dup_step: no source set (fg_dup_seed)");
  hipStream_t s = (hipStream_t)stream;
  dup_step_kernel<<<d->grid, DUP_BT, 0, s>>>(d->args);
  dup_big_kernel<<<d->grid, DUP_BT, 0, s>>>(d->args);
  FG_HIP_TRY(hipGetLastError());
  return FG_OK;
}

extern "C" fg_status fg_dup_send(const fg_dup* from, fg_dup* to, void* stream) {
  if (!from || !to) return fg_set_error(FG_EINVAL, "fg_dup_send: NULL argument");
  if (from == to || from->part == to->part || from->nparts != to->nparts || from->n != to->n)
    return fg_set_error(FG_EINVAL, "fg_dup_send: partitions %d -> %d do not belong together",
                        from->part, to->part);
  const DupArgs& F = from->args;
  const DupArgs& T = to->args;
  const int32_t q = from->part;
  dup_send_kernel<<<from->grid, DUP_BT, 0, (hipStream_t)stream>>>(
      F.ctl, F.hdr, F.mids, F.mbits, F.nwords, T.rhdr + q, T.rids + (int64_t)q * T.ids_stride,
      T.rbits + (int64_t)q * T.bits_stride);
  FG_HIP_TRY(hipGetLastError());
  return FG_OK;
}

extern "C" fg_status fg_dup_combine(fg_dup* d, void* stream) {
  if (!d) return fg_set_error(FG_EINVAL, "fg_dup_combine: NULL argument");
  if (!d->seeded) return fg_set_error(FG_EINVAL, "fg_dup_combine: no source set (fg_dup_seed)");
  dup_combine_kernel<<<d->grid, DUP_BT, 0, (hipStream_t)stream>>>(d->args);
  FG_HIP_TRY(hipGetLastError());
  return FG_OK;
}

extern "C" fg_status fg_dup_poll(const fg_dup* d, int32_t* done, int32_t* iterations,
                                 void* stream) {
  if (!d) return fg_set_error(FG_EINVAL, "fg_dup_poll: NULL argument");
  DupCtl c;
  hipStream_t s = (hipStream_t)stream;
  FG_HIP_TRY(hipMemcpyAsync(&c, d->args.ctl, sizeof(c), hipMemcpyDeviceToHost, s));
  FG_HIP_TRY(hipStreamSynchronize(s));
  if (done) *done = c.done;
  if (iterations) *iterations = c.k;
  return FG_OK;
}

extern "C" fg_status fg_dup_run(fg_dup* const* parts, int32_t nparts, int32_t src,
                                int32_t* const* depth, int32_t* const* parent,
                                fg_run_stats* const* stats, int32_t poll_every, void* stream) {
  if (!parts || !depth || nparts < 1 || nparts > 16)
    return fg_set_error(FG_EINVAL, "fg_dup_run: bad arguments");
  uint32_t seen = 0;
  for (int32_t p = 0; p < nparts; ++p) {
    const fg_dup* d = parts[p];
    if (!d || !depth[p]) return fg_set_error(FG_EINVAL, "fg_dup_run: NULL partition %d", p);
    if (d->nparts != nparts || d->n != parts[0]->n || d->part != p)
      return fg_set_error(FG_EINVAL, "fg_dup_run: parts[%d] is partition %d of %d", p, d->part,
                          d->nparts);
    seen |= 1u << d->part;
  }
  if (seen != (nparts == 32 ? 0xffffffffu : (1u << nparts) - 1))
    return fg_set_error(FG_EINVAL, "fg_dup_run: partitions missing");
  if (poll_every < 1) poll_every = 4;
  for (int32_t p = 0; p < nparts; ++p) {
    fg_status st = fg_dup_seed(parts[p], src, depth[p], parent ? parent[p] : nullptr,
                               stats ? stats[p] : nullptr, stream);
    if (st != FG_OK) return st;
  }
  // every iteration labels at least one vertex, so n + 1 iterations bound
  // any traversal
  const int64_t max_iter = (int64_t)parts[0]->n + 1;
  for (int64_t it = 0; it < max_iter;) {
    for (int32_t r = 0; r < poll_every; ++r, ++it) {
      for (int32_t p = 0; p < nparts; ++p) {
        fg_status st = fg_dup_step(parts[p], stream);
        if (st != FG_OK) return st;
      }
      for (int32_t p = 0; p < nparts; ++p)
        for (int32_t q = 0; q < nparts; ++q) {
          if (q == p) continue;
          fg_status st = fg_dup_send(parts[p], parts[q], stream);
          if (st != FG_OK) return st;
        }
      for (int32_t p = 0; p < nparts; ++p) {
        fg_status st = fg_dup_combine(parts[p], stream);
        if (st != FG_OK) return st;
      }
    }
    int32_t done = 0;
    fg_status st = fg_dup_poll(parts[0], &done, nullptr, stream);
    if (st != FG_OK) return st;
    if (done) return FG_OK;
  }
  return fg_set_error(FG_EDEVICE, "fg_dup_run: no convergence after %lld iterations",
                      (long long)max_iter);
}
