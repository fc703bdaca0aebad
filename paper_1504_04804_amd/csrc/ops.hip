// Standalone frontier operators (Sec. II-B): advance with a deterministic
// edge-frontier layout, filter with the visited test-and-set, one backward
// (pull) step (Sec. VI-A), queue <-> bitmap conversions, and the unfused
// push BFS that chains advance and filter kernels (Alg. 1 as an advance
// kernel followed by a filter kernel).
#include <string.h>

#include <vector>

#include "fg_common.h"

namespace {

constexpr int TB = 1024;          // tile of the scans (one block, one element per thread)
constexpr int EXP_PER_BLOCK = 2048;

// ------------------------------------------------------------ scan helpers

// Block sums of `val(i)` over tiles of TB elements.
template <class F>
__global__ void tile_sum_kernel(int64_t len, F val, int64_t* __restrict__ sums) {
  __shared__ int64_t red[TB / FG_WAVE + 1];
  const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
  int64_t x = i < len ? val(i) : 0;
  int64_t s = fg_block_sum<TB>(x, red);
  if (threadIdx.x == 0) sums[blockIdx.x] = s;
}

// Exclusive scan of `cnt` tile sums in place (single block), total -> *total.
__global__ void scan_sums_kernel(int64_t cnt, int64_t* __restrict__ sums,
                                 int64_t* __restrict__ total) {
  __shared__ int64_t red[TB / FG_WAVE + 1];
  int64_t carry = 0;
  for (int64_t c0 = 0; c0 < cnt; c0 += TB) {
    const int64_t i = c0 + threadIdx.x;
    int64_t x = i < cnt ? sums[i] : 0;
    int64_t tot = 0;
    int64_t ex = fg_block_excl_scan<TB>(x, red, &tot);
    if (i < cnt) sums[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) *total = carry;
}

// Exclusive scan of val(i) using the scanned tile sums; out[i] for i < len.
template <class F>
__global__ void tile_scan_kernel(int64_t len, F val, const int64_t* __restrict__ sums,
                                 int64_t* __restrict__ out) {
  __shared__ int64_t red[TB / FG_WAVE + 1];
  const int64_t i = (int64_t)blockIdx.x * TB + threadIdx.x;
  int64_t x = i < len ? val(i) : 0;
  int64_t tot = 0;
  int64_t ex = fg_block_excl_scan<TB>(x, red, &tot);
  if (i < len) out[i] = sums[blockIdx.x] + ex;
}

// Degree of frontier entry i; entries at or past the device-resident
// length *dlen (when given) count as degree 0.
struct DegOf {
  const int32_t* off;
  const int32_t* q;
  const int32_t* dlen;
  __device__ int64_t operator()(int64_t i) const {
    if (dlen && i >= (int64_t)*dlen) return 0;
    int32_t u = q[i];
    return (int64_t)(off[u + 1] - off[u]);
  }
};

struct PopOf {
  const uint64_t* bits;
  __device__ int64_t operator()(int64_t i) const { return __popcll(bits[i]); }
};

// Scan workspace: tile sums + scanned values + total.
struct ScanWs {
  int64_t* sums;   // ceil(len / TB)
  int64_t* scan;   // len
  int64_t* total;  // 1
};

template <class F>
void run_scan(int64_t len, F f, ScanWs w, hipStream_t s) {
  const int64_t tiles = (len + TB - 1) / TB;
  if (tiles > 0) tile_sum_kernel<<<(unsigned)tiles, TB, 0, s>>>(len, f, w.sums);
  scan_sums_kernel<<<1, TB, 0, s>>>(tiles, w.sums, w.total);
  if (tiles > 0) tile_scan_kernel<<<(unsigned)tiles, TB, 0, s>>>(len, f, w.sums, w.scan);
}

// -------------------------------------------------------------- advance

// Largest i in [lo, hi] with scan[i] <= t.
__device__ __forceinline__ int64_t scan_upper(const int64_t* scan, int64_t lo, int64_t hi,
                                              int64_t t) {
  while (lo < hi) {
    int64_t mid = (lo + hi + 1) >> 1;
    if (scan[mid] <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Each block writes EXP_PER_BLOCK consecutive slots of the edge frontier.
// Slot t belongs to frontier entry i = last index with scan[i] <= t.
__global__ void advance_expand_kernel(int64_t len, const int32_t* __restrict__ q,
                                      const int32_t* __restrict__ off,
                                      const int32_t* __restrict__ col,
                                      const int64_t* __restrict__ scan,
                                      const int64_t* __restrict__ total, int64_t capacity,
                                      int32_t* __restrict__ out_dst,
                                      int32_t* __restrict__ out_src,
                                      int64_t* __restrict__ out_len) {
  __shared__ int64_t s_scan[EXP_PER_BLOCK + 1];
  __shared__ int64_t s_lo, s_cnt;
  const int64_t T = *total;
  if (blockIdx.x == 0 && threadIdx.x == 0 && out_len) *out_len = T;
  const int64_t lim = T < capacity ? T : capacity;
  for (int64_t t0 = (int64_t)blockIdx.x * EXP_PER_BLOCK; t0 < lim;
       t0 += (int64_t)gridDim.x * EXP_PER_BLOCK) {
    const int64_t t1 = (t0 + EXP_PER_BLOCK < lim ? t0 + EXP_PER_BLOCK : lim) - 1;
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t lo = scan_upper(scan, 0, len - 1, t0);
      int64_t hi = scan_upper(scan, lo, len - 1, t1);
      s_lo = lo;
      s_cnt = hi - lo + 1;
    }
    __syncthreads();
    const int64_t lo = s_lo, cnt = s_cnt;
    const bool in_lds = cnt <= EXP_PER_BLOCK + 1;
    if (in_lds)
      for (int64_t j = threadIdx.x; j < cnt; j += blockDim.x) s_scan[j] = scan[lo + j];
    __syncthreads();
    for (int64_t t = t0 + threadIdx.x; t <= t1; t += blockDim.x) {
      int64_t i;
      if (in_lds) {
        int64_t a = 0, b = cnt - 1;
        while (a < b) {
          int64_t mid = (a + b + 1) >> 1;
          if (s_scan[mid] <= t) a = mid; else b = mid - 1;
        }
        i = lo + a;
      } else {
        i = scan_upper(scan, lo, lo + cnt - 1, t);
      }
      const int32_t u = q[i];
      const int64_t base = in_lds ? s_scan[i - lo] : scan[i];
      out_dst[t] = col[off[u] + (t - base)];
      out_src[t] = u;
    }
  }
}

// --------------------------------------------------------------- filter

__global__ void fill_i32_kernel(int32_t* p, int64_t count, int32_t value) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

// Test-and-set of dst's visited bit; winners take depth / parent and are
// appended to out_q.  The edge-frontier length is read from device memory
// (`d_len`, clamped to `cap`) or taken from `h_len` when d_len is NULL.
__global__ void filter_kernel(const int32_t* __restrict__ dst, const int32_t* __restrict__ src,
                              const int64_t* __restrict__ d_len, int64_t h_len, int64_t cap,
                              uint32_t* __restrict__ visited, int32_t d_new,
                              int32_t* __restrict__ depth, int32_t* __restrict__ parent,
                              int32_t* __restrict__ out_q, int32_t* __restrict__ out_len) {
  int64_t len = d_len ? *d_len : h_len;
  if (len > cap) len = cap;
  const int lane = fg_lane();
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x - lane; k0 < len; k0 += nth) {
    const int64_t k = k0 + lane;
    bool won = false;
    int32_t v = 0;
    if (k < len) {
      v = dst[k];
      const uint32_t bit = 1u << (v & 31);
      if (!(visited[v >> 5] & bit)) {
        const uint32_t old = atomicOr(&visited[v >> 5], bit);
        if (!(old & bit)) {
          won = true;
          depth[v] = d_new;
          if (parent) parent[v] = src[k];
        }
      }
    }
    const uint64_t mask = __ballot(won);
    if (mask) {
      int32_t pos = 0;
      if (lane == 0) pos = atomicAdd(out_len, __popcll(mask));
      pos = __shfl(pos, 0, FG_WAVE);
      if (won) out_q[pos + fg_mbcnt(mask)] = v;
    }
  }
}

// ------------------------------------------------------------ pull step

__global__ void pull_step_kernel(int32_t nwords, const int32_t* __restrict__ off,
                                 const int32_t* __restrict__ col,
                                 const uint64_t* __restrict__ nz,
                                 const uint64_t* __restrict__ fbits,
                                 uint64_t* __restrict__ visited,
                                 uint64_t* __restrict__ next_bits, int32_t d_new,
                                 int32_t* __restrict__ depth, int32_t* __restrict__ parent,
                                 int32_t* __restrict__ out_q, int32_t* __restrict__ out_len,
                                 int64_t* __restrict__ inspected) {
  const int lane = fg_lane();
  const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / FG_WAVE;
  const int64_t W = ((int64_t)gridDim.x * blockDim.x) / FG_WAVE;
  int64_t insp = 0;
  for (int64_t w = gw; w < nwords; w += W) {
    const uint64_t vis = visited[w];
    const uint64_t act = nz[w] & ~vis;
    uint64_t nb = 0;
    if (act) {
      const int32_t v = (int32_t)(w * 64 + lane);
      bool found = false;
      int32_t pu = -1;
      if ((act >> lane) & 1ull) {
        const int32_t e = off[v + 1];
        for (int32_t i = off[v]; i < e; ++i) {
          const int32_t u = col[i];
          insp++;
          if ((fbits[u >> 6] >> (u & 63)) & 1ull) {
            found = true;
            pu = u;
            break;
          }
        }
      }
      nb = __ballot(found);
      if (found) {
        depth[v] = d_new;
        if (parent) parent[v] = pu;
      }
      if (nb) {
        int32_t pos = 0;
        if (lane == 0) pos = atomicAdd(out_len, __popcll(nb));
        pos = __shfl(pos, 0, FG_WAVE);
        if (found) out_q[pos + fg_mbcnt(nb)] = v;
        if (lane == 0) visited[w] = vis | nb;
      }
    }
    if (lane == 0) next_bits[w] = nb;
  }
  insp = fg_wave_sum(insp);
  if (lane == 0 && inspected && insp) atomicAdd((unsigned long long*)inspected, (unsigned long long)insp);
}

__global__ void zero_i64_kernel(int64_t* p) {
  if (threadIdx.x == 0) *p = 0;
}

// ---------------------------------------------------------- conversions

__global__ void queue_to_bitmap_kernel(const int32_t* __restrict__ q, int64_t len,
                                       unsigned long long* __restrict__ bits) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = q[i];
    atomicOr(&bits[v >> 6], 1ull << (v & 63));
  }
}

__global__ void bitmap_to_queue_kernel(int64_t nwords, const uint64_t* __restrict__ bits,
                                       const int64_t* __restrict__ scan,
                                       const int64_t* __restrict__ total,
                                       int32_t* __restrict__ out_q, int32_t* __restrict__ out_len) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *out_len = (int32_t)*total;
  if (i >= nwords) return;
  uint64_t w = bits[i];
  int64_t pos = scan[i];
  while (w) {
    const int b = __builtin_ctzll(w);
    w &= w - 1;
    out_q[pos++] = (int32_t)(i * 64 + b);
  }
}

// ------------------------------------------------------------- layouts

struct OpsLayout {
  int64_t* sums;
  int64_t* scan;
  int64_t* total;
  int64_t* misc;     // [0] edge-frontier length, [1] inspected
  int32_t* len32;    // [0] out length
  uint32_t* visited; // unfused BFS
  int32_t* q[2];
  int32_t* edst;
  int32_t* esrc;
  size_t bytes;
};

OpsLayout ops_layout(const fg_graph* g, void* ws, bool with_bfs) {
  fg_carver c(ws);
  OpsLayout L;
  const int64_t n = g->n;
  const int64_t maxlen = n > g->nwords ? n : g->nwords;
  L.sums = c.take<int64_t>((maxlen + TB - 1) / TB + 1);
  L.scan = c.take<int64_t>(maxlen + 1);
  L.total = c.take<int64_t>(1);
  L.misc = c.take<int64_t>(4);
  L.len32 = c.take<int32_t>(4);
  if (with_bfs) {
    L.visited = c.take<uint32_t>((n + 31) / 32 + 2);
    L.q[0] = c.take<int32_t>(n);
    L.q[1] = c.take<int32_t>(n);
    L.edst = c.take<int32_t>(g->m > 0 ? g->m : 1);
    L.esrc = c.take<int32_t>(g->m > 0 ? g->m : 1);
  } else {
    L.visited = nullptr;
    L.q[0] = L.q[1] = nullptr;
    L.edst = L.esrc = nullptr;
  }
  L.bytes = c.used;
  return L;
}

int grid_for(int64_t work, int per_block, int cap) {
  int64_t b = (work + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

}  // namespace

size_t fg_ops_workspace_bytes(const fg_graph* g, bool with_bfs) {
  return ops_layout(g, nullptr, with_bfs).bytes;
}


extern "C" size_t fg_workspace_bytes(const fg_graph* g, int32_t primitive, int32_t lanes) {
  if (!g) return 0;
  switch (primitive) {
    case FG_PRIM_BFS: return fg_bfs_workspace_bytes(g);
    case FG_PRIM_BFS_UNFUSED: return fg_ops_workspace_bytes(g, true);
    case FG_PRIM_SSSP: return fg_sssp_workspace_bytes(g);
    case FG_PRIM_MSBFS:
      if (lanes < 1 || lanes > 64) return 0;
      return fg_msbfs_workspace_bytes(g, lanes);
    case FG_PRIM_MSSSP:
      if (lanes < 1 || lanes > 64) return 0;
      return fg_mssp_workspace_bytes(g);
    case FG_PRIM_PR: return fg_pr_workspace_bytes(g);
    case FG_PRIM_CC: return fg_cc_workspace_bytes(g);
    default: return 0;
  }
}

static fg_status advance_impl(const fg_graph* g, const int32_t* frontier, int64_t len,
                              const int32_t* len_dev, int32_t* out_dst, int32_t* out_src,
                              int64_t capacity, int64_t* out_len, const OpsLayout& L,
                              hipStream_t s) {
  ScanWs sw{L.sums, L.scan, L.total};
  // with a device-resident length the scan runs over the host bound `len`,
  // entries past the device length contributing no edges
  run_scan(len, DegOf{g->off, frontier, len_dev}, sw, s);
  int blocks = grid_for(g->m > 0 ? g->m : 1, EXP_PER_BLOCK, 4096);
  advance_expand_kernel<<<blocks, 256, 0, s>>>(len, frontier, g->off, g->col, L.scan, L.total,
                                               capacity, out_dst, out_src, out_len);
  FG_HIP_TRY(hipGetLastError());
  return FG_OK;
}

extern "C" fg_status fg_advance(const fg_graph* g, const int32_t* frontier, int32_t len,
                                const int32_t* len_dev, int32_t* out_dst, int32_t* out_src,
                                int64_t capacity, int64_t* out_len, void* ws, size_t ws_bytes,
                                void* stream) {
  if (!g || !out_dst || !out_src || !out_len || !ws)
    return fg_set_error(FG_EINVAL, "fg_advance: NULL argument");
  if (len < 0 || len > g->n) return fg_set_error(FG_EINVAL, "fg_advance: len=%d outside [0, n]", len);
  if (len > 0 && !frontier) return fg_set_error(FG_EINVAL, "fg_advance: frontier is NULL");
  if (capacity < 0) return fg_set_error(FG_EINVAL, "fg_advance: negative capacity");
  OpsLayout L = ops_layout(g, ws, false);
  FG_CHECK_WS_ALIGN(ws, "fg_advance");
  if (ws_bytes < L.bytes)
    return fg_set_error(FG_ENOMEM, "fg_advance: workspace of %zu bytes < required %zu", ws_bytes,
                        L.bytes);
  return advance_impl(g, frontier, len, len_dev, out_dst, out_src, capacity, out_len, L,
                      (hipStream_t)stream);
}

extern "C" fg_status fg_filter(const fg_graph* g, const int32_t* dst, const int32_t* src,
                               int64_t len, const int64_t* len_dev, uint32_t* visited,
                               int32_t iter, int32_t* depth, int32_t* parent, int32_t* out_q,
                               int32_t* out_len, void* stream) {
  if (!g || !visited || !depth || !out_q || !out_len)
    return fg_set_error(FG_EINVAL, "fg_filter: NULL argument");
  if (len < 0) return fg_set_error(FG_EINVAL, "fg_filter: negative len");
  if (len > 0 && (!dst || (parent && !src))) return fg_set_error(FG_EINVAL, "fg_filter: NULL edge frontier");
  if (iter < 0) return fg_set_error(FG_EINVAL, "fg_filter: negative iteration");
  hipStream_t s = (hipStream_t)stream;
  fill_i32_kernel<<<1, 64, 0, s>>>(out_len, 1, 0);
  if (len > 0)
    filter_kernel<<<grid_for(len, 256, 8192), 256, 0, s>>>(dst, src, len_dev, len, len, visited,
                                                           iter + 1, depth, parent, out_q, out_len);
  FG_HIP_TRY(hipGetLastError());
  return FG_OK;
}

extern "C" fg_status fg_pull_step(const fg_graph* g, const uint64_t* frontier_bits,
                                  uint64_t* visited, uint64_t* next_bits, int32_t iter,
                                  int32_t* depth, int32_t* parent, int32_t* out_q,
                                  int32_t* out_len, int64_t* inspected, void* stream) {
  if (!g || !frontier_bits || !visited || !next_bits || !depth || !out_q || !out_len)
    return fg_set_error(FG_EINVAL, "fg_pull_step: NULL argument");
  if (!g->symmetric)
    return fg_set_error(FG_EUNSUPPORTED, "fg_pull_step: needs an undirected graph (FG_SYMMETRIC)");
  if (iter < 0) return fg_set_error(FG_EINVAL, "fg_pull_step: negative iteration");
  hipStream_t s = (hipStream_t)stream;
  fill_i32_kernel<<<1, 64, 0, s>>>(out_len, 1, 0);
  if (inspected) zero_i64_kernel<<<1, 64, 0, s>>>(inspected);
  pull_step_kernel<<<grid_for(g->nwords, 4, 8192), 256, 0, s>>>(
      g->nwords, g->off, g->col, g->nzmask, frontier_bits, visited, next_bits, iter + 1, depth,
      parent, out_q, out_len, inspected);
  FG_HIP_TRY(hipGetLastError());
  return FG_OK;
}

extern "C" fg_status fg_queue_to_bitmap(const fg_graph* g, const int32_t* queue, int32_t len,
                                        uint64_t* bits, void* stream) {
  if (!g || !bits) return fg_set_error(FG_EINVAL, "fg_queue_to_bitmap: NULL argument");
  if (len < 0 || len > g->n) return fg_set_error(FG_EINVAL, "fg_queue_to_bitmap: bad len %d", len);
  if (len > 0 && !queue) return fg_set_error(FG_EINVAL, "fg_queue_to_bitmap: queue is NULL");
  if (len == 0) return FG_OK;
  queue_to_bitmap_kernel<<<grid_for(len, 256, 4096), 256, 0, (hipStream_t)stream>>>(
      queue, len, (unsigned long long*)bits);
  FG_HIP_TRY(hipGetLastError());
  return FG_OK;
}

extern "C" fg_status fg_bitmap_to_queue(const fg_graph* g, const uint64_t* bits, int32_t* out_q,
                                        int32_t* out_len, void* ws, size_t ws_bytes,
                                        void* stream) {
  if (!g || !bits || !out_q || !out_len || !ws)
    return fg_set_error(FG_EINVAL, "fg_bitmap_to_queue: NULL argument");
  OpsLayout L = ops_layout(g, ws, false);
  FG_CHECK_WS_ALIGN(ws, "fg_bitmap_to_queue");
  if (ws_bytes < L.bytes)
    return fg_set_error(FG_ENOMEM, "fg_bitmap_to_queue: workspace of %zu bytes < required %zu",
                        ws_bytes, L.bytes);
  hipStream_t s = (hipStream_t)stream;
  ScanWs sw{L.sums, L.scan, L.total};
  run_scan(g->nwords, PopOf{bits}, sw, s);
  bitmap_to_queue_kernel<<<grid_for(g->nwords, 256, 1 << 30), 256, 0, s>>>(
      g->nwords, bits, L.scan, L.total, out_q, out_len);
  FG_HIP_TRY(hipGetLastError());
  return FG_OK;
}

// Unfused push BFS (Alg. 1: an advance kernel followed by a filter kernel),
// driven from the host one iteration at a time.  Kept as the baseline that
// kernel fusion (Sec. VI-C) is measured against.

fg_status fg_bfs_unfused(const fg_graph* g, int32_t src, void* ws, size_t ws_bytes,
                         int32_t* depth, int32_t* parent, fg_run_stats* stats, hipStream_t s) {
  OpsLayout L = ops_layout(g, ws, true);
  FG_CHECK_WS_ALIGN(ws, "fg_bfs_unfused");
  if (ws_bytes < L.bytes)
    return fg_set_error(FG_ENOMEM, "fg_bfs: workspace of %zu bytes < required %zu (unfused)",
                        ws_bytes, L.bytes);
  fg_bfs_launch_init(g, src, depth, parent, (uint64_t*)L.visited, L.q[0], stats, s, nullptr, 0);
  std::vector<int8_t> dir;
  std::vector<int64_t> front, insp;
  int64_t len = 1, reached = 1, insp_sum = 0;
  int32_t k = 0, sel = 0;
  while (len > 0) {
    front.push_back(len);
    fg_status st = advance_impl(g, L.q[sel], len, nullptr, L.edst, L.esrc, g->m, L.misc, L, s);
    if (st != FG_OK) return st;
    fill_i32_kernel<<<1, 64, 0, s>>>(L.len32, 1, 0);
    filter_kernel<<<grid_for(g->m > 0 ? g->m : 1, 256, 8192), 256, 0, s>>>(
        L.edst, L.esrc, L.misc, 0, g->m, L.visited, k + 1, depth, parent, L.q[sel ^ 1], L.len32);
    int64_t h[1];
    int32_t nl = 0;
    FG_HIP_TRY(hipMemcpyAsync(h, L.misc, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    FG_HIP_TRY(hipMemcpyAsync(&nl, L.len32, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    FG_HIP_TRY(hipStreamSynchronize(s));
    insp.push_back(h[0]);
    insp_sum += h[0];
    len = nl;
    reached += nl;
    sel ^= 1;
    k++;
  }
  if (stats) {
    fg_run_stats hs;
    memset(&hs, 0, sizeof(hs));
    hs.status = FG_OK;
    hs.iterations = k;
    hs.reached = reached;
    hs.edges_inspected = insp_sum;
    for (int32_t i = 0; i < k && i < FG_TRACE_MAX; ++i) {
      hs.dir[i] = 0;
      hs.frontier[i] = front[i];
      hs.inspected[i] = insp[i];
    }
    FG_HIP_TRY(hipMemcpyAsync(stats, &hs, sizeof(hs), hipMemcpyHostToDevice, s));
    FG_HIP_TRY(hipStreamSynchronize(s));
  }
  return FG_OK;
}
