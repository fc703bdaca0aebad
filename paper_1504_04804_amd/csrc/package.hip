// One GPU's share of a partitioned graph and the per-iteration package step
// of the multi-GPU framework (Sec. III-B: split the output frontier into
// local and remote sub-frontiers, package the remote ones with their
// associated data per receiving GPU).
//
// The share is built on the host with duplicate-1-hop proxies (Sec. III-C):
// hosted vertices get local ids 0..n_local-1 in ascending global order,
// remote neighbours of hosted vertices become proxies n_local..n_total-1 in
// ascending global order; a hosted row keeps the global order of its
// neighbours (renamed); proxies have no out-edges.  conv[v] is the id of v
// on its owner (its rank among the owner's hosted vertices), l2g[v] its
// global id.  On the device the owner and conv tables are fused into one
// 32-bit route word (owner << 28 | conv), so splitting and id conversion cost
// one gather per frontier vertex.
//
// fg_package is stable: each peer buffer lists its vertices in frontier
// order.  Three kernels: per-tile bucket counts, a scan of the tile counts,
// and a scatter that ranks entries inside each tile with wave ballots.
#include <string.h>

#include <vector>

#include "fg_common.h"

struct fg_share {
  int32_t n = 0, n_local = 0, n_total = 0, nparts = 0, part = 0;
  int64_t m_local = 0;
  fg_graph* graph = nullptr;   // the local CSR (n_total vertices)
  uint8_t* owner = nullptr;    // device uint8[n_total]
  int32_t* conv = nullptr;     // device int32[n_total]
  int32_t* l2g = nullptr;      // device int32[n_total]
  uint32_t* route = nullptr;   // device uint32[n_total]: owner << 28 | conv
  void* owned = nullptr;
};

namespace {

constexpr int KB = 1024;        // threads per block
constexpr int TILE = 4 * KB;    // frontier entries per tile
constexpr int MAXP = 16;        // partitions (owner fits 4 bits)

// Frontier length: the host value, or the smaller of it and the device-
// resident length when one is given.
__device__ __forceinline__ int32_t eff_len(int32_t len, const int32_t* len_dev) {
  if (!len_dev) return len;
  const int32_t d = *len_dev;
  return d < len ? (d < 0 ? 0 : d) : len;
}

__global__ void pkg_count_kernel(const int32_t* __restrict__ frontier, int32_t hlen,
                                 const int32_t* __restrict__ len_dev,
                                 const uint32_t* __restrict__ route, int32_t n_local,
                                 int32_t part, int32_t nparts, int32_t* __restrict__ tile_cnt) {
  __shared__ int32_t cnt[MAXP];
  const int32_t len = eff_len(hlen, len_dev);
  if (threadIdx.x < MAXP) cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t t0 = (int64_t)blockIdx.x * TILE;
  for (int j = 0; j < TILE / KB; ++j) {
    const int64_t i = t0 + j * KB + threadIdx.x;
    if (i < len) {
      const int32_t v = frontier[i];
      const int32_t b = v < n_local ? part : (int32_t)(route[v] >> 28);
      atomicAdd(&cnt[b], 1);
    }
  }
  __syncthreads();
  if (threadIdx.x < nparts) tile_cnt[(int64_t)blockIdx.x * nparts + threadIdx.x] = cnt[threadIdx.x];
}

// In place exclusive scan of tile counts per bucket; totals to counts[].
__global__ void pkg_scan_kernel(int32_t tiles, int32_t nparts, int32_t* __restrict__ tile_cnt,
                                int32_t* __restrict__ counts, int32_t part,
                                int32_t* __restrict__ local_count) {
  __shared__ int32_t red[KB / FG_WAVE + 1];
  for (int b = 0; b < nparts; ++b) {
    int32_t carry = 0;
    for (int32_t c0 = 0; c0 < tiles; c0 += KB) {
      const int32_t t = c0 + threadIdx.x;
      const int32_t x = t < tiles ? tile_cnt[(int64_t)t * nparts + b] : 0;
      int32_t tot = 0;
      const int32_t ex = fg_block_excl_scan<KB>(x, red, &tot);
      if (t < tiles) tile_cnt[(int64_t)t * nparts + b] = carry + ex;
      carry += tot;
    }
    if (threadIdx.x == 0) {
      if (b == part) {
        counts[b] = 0;
        if (local_count) *local_count = carry;
      } else {
        counts[b] = carry;
      }
    }
  }
}

__global__ void pkg_scatter_kernel(const int32_t* __restrict__ frontier, int32_t hlen,
                                   const int32_t* __restrict__ len_dev,
                                   const uint32_t* __restrict__ route,
                                   const int32_t* __restrict__ l2g, int32_t n_local, int32_t part,
                                   int32_t nparts, const int32_t* __restrict__ depth,
                                   const int32_t* __restrict__ parent,
                                   const int32_t* __restrict__ tile_base, int64_t cap,
                                   int32_t* __restrict__ ids_out, int32_t* __restrict__ depth_out,
                                   int32_t* __restrict__ parent_out,
                                   int32_t* __restrict__ local_out) {
  __shared__ int32_t wcnt[KB / FG_WAVE][MAXP];
  __shared__ int32_t run[MAXP];
  const int32_t len = eff_len(hlen, len_dev);
  const int lane = fg_lane();
  const int wid = threadIdx.x / FG_WAVE;
  if (threadIdx.x < MAXP) run[threadIdx.x] = threadIdx.x < nparts
                                                 ? tile_base[(int64_t)blockIdx.x * nparts + threadIdx.x]
                                                 : 0;
  const int64_t t0 = (int64_t)blockIdx.x * TILE;
  for (int j = 0; j < TILE / KB; ++j) {
    const int64_t i = t0 + j * KB + threadIdx.x;
    int32_t v = 0, b = -1;
    uint32_t r = 0;
    if (i < len) {
      v = frontier[i];
      if (v < n_local) {
        b = part;
      } else {
        r = route[v];
        b = (int32_t)(r >> 28);
      }
    }
    // rank within the wave for this lane's bucket, and per-wave bucket totals
    int32_t in_wave = 0;
    for (int p = 0; p < nparts; ++p) {
      const uint64_t m = __ballot(b == p);
      if (b == p) in_wave = fg_mbcnt(m);
      if (lane == 0) wcnt[wid][p] = __popcll(m);
    }
    __syncthreads();
    int32_t before = 0;
    if (b >= 0) {
      for (int w = 0; w < wid; ++w) before += wcnt[w][b];
    }
    const int32_t pos = (b >= 0 ? run[b] : 0) + before + in_wave;
    if (b == part) {
      if (local_out) local_out[pos] = v;
    } else if (b >= 0) {
      const int64_t slot = (int64_t)b * cap + pos;
      ids_out[slot] = (int32_t)(r & 0x0FFFFFFFu);
      depth_out[slot] = depth[v];
      if (parent_out) {
        const int32_t pv = parent[v];
        parent_out[slot] = pv >= 0 ? l2g[pv] : -1;
      }
    }
    __syncthreads();
    if (threadIdx.x < nparts) {
      int32_t s = 0;
      for (int w = 0; w < KB / FG_WAVE; ++w) s += wcnt[w][threadIdx.x];
      run[threadIdx.x] += s;
    }
    __syncthreads();
  }
}

// Combine received vertices with the local state (the framework's merge
// step; for BFS a received vertex not yet visited takes the received label
// and joins the next input frontier).  Test-and-set on the visited bitmap,
// so a vertex received from several peers (or also found locally) is
// taken once.
__global__ void combine_kernel(const int32_t* __restrict__ ids, const int32_t* __restrict__ labels,
                               const int32_t* __restrict__ parents, int32_t hlen,
                               const int32_t* __restrict__ len_dev,
                               uint32_t* __restrict__ visited, int32_t* __restrict__ depth,
                               int32_t* __restrict__ parent, int32_t* __restrict__ out_q,
                               int32_t* __restrict__ out_len) {
  const int32_t len = eff_len(hlen, len_dev);
  const int lane = fg_lane();
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x - lane; i0 < len; i0 += nth) {
    const int64_t i = i0 + lane;
    bool won = false;
    int32_t v = 0;
    if (i < len) {
      v = ids[i];
      const uint32_t bit = 1u << (v & 31);
      if (!(visited[v >> 5] & bit) && !(atomicOr(&visited[v >> 5], bit) & bit)) {
        won = true;
        depth[v] = labels[i];
        if (parent && parents) parent[v] = parents[i];
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

__global__ void route_kernel(int32_t n, const uint8_t* __restrict__ owner,
                             const int32_t* __restrict__ conv, uint32_t* __restrict__ route) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    route[i] = ((uint32_t)owner[i] << 28) | (uint32_t)conv[i];
}

// a1 on a share: visited cleared, depth (and parent) -1; if the share
// hosts global vertex `src` (l2g is ascending over the hosted vertices,
// found by binary search), its local id is marked visited at depth 0 and
// becomes the one-entry frontier; *qlen receives the frontier length.
__global__ void share_clear_kernel(int32_t n_total, uint32_t* __restrict__ visited,
                                   int32_t* __restrict__ depth, int32_t* __restrict__ parent) {
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = t; i < n_total; i += nth) {
    depth[i] = -1;
    if (parent) parent[i] = -1;
  }
  const int64_t nwords = ((int64_t)n_total + 31) / 32;
  for (int64_t w = t; w < nwords; w += nth) visited[w] = 0u;
}

__global__ void share_seed_src_kernel(int32_t n_local, const int32_t* __restrict__ l2g, int32_t src,
                                      uint32_t* __restrict__ visited, int32_t* __restrict__ depth,
                                      int32_t* __restrict__ parent, int32_t* __restrict__ queue,
                                      int32_t* __restrict__ qlen) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int32_t lo = 0, hi = n_local;  // first hosted local id with l2g >= src
  while (lo < hi) {
    const int32_t mid = lo + (hi - lo) / 2;
    if (l2g[mid] < src) lo = mid + 1; else hi = mid;
  }
  if (lo < n_local && l2g[lo] == src) {
    depth[lo] = 0;
    if (parent) parent[lo] = src;
    visited[lo >> 5] |= 1u << (lo & 31);
    queue[0] = lo;
    *qlen = 1;
  } else {
    *qlen = 0;
  }
}

}  // namespace

extern "C" fg_status fg_share_seed(const fg_share* s, int32_t src, uint32_t* visited,
                                   int32_t* depth, int32_t* parent, int32_t* queue, int32_t* qlen,
                                   void* stream) {
  if (!s || !visited || !depth || !queue || !qlen)
    return fg_set_error(FG_EINVAL, "fg_share_seed: NULL argument");
  if (src < 0 || src >= s->n)
    return fg_set_error(FG_EINVAL, "fg_share_seed: src=%d outside [0, %d)", src, s->n);
  hipStream_t hs = (hipStream_t)stream;
  int blocks = (int)((s->n_total + 1023) / 1024);
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  share_clear_kernel<<<blocks, 256, 0, hs>>>(s->n_total, visited, depth, parent);
  share_seed_src_kernel<<<1, 64, 0, hs>>>(s->n_local, s->l2g, src, visited, depth, parent, queue,
                                          qlen);
  FG_HIP_TRY(hipGetLastError());
  return FG_OK;
}

extern "C" fg_status fg_share_destroy(fg_share* s) {
  if (!s) return FG_OK;
  if (s->graph) fg_graph_destroy(s->graph);
  if (s->owned) hipFree(s->owned);
  delete s;
  return FG_OK;
}

extern "C" fg_status fg_share_create(int32_t n, int64_t m, const int32_t* row_offsets,
                                     const int32_t* col_idx, const uint8_t* owner,
                                     int32_t nparts, int32_t part, void* stream,
                                     fg_share** out) {
  if (!out) return fg_set_error(FG_EINVAL, "fg_share_create: out is NULL");
  *out = nullptr;
  if (n < 1 || m < 0 || m >= (int64_t(1) << 31) || !row_offsets || (m > 0 && !col_idx) || !owner)
    return fg_set_error(FG_EINVAL, "fg_share_create: bad graph arguments");
  if (nparts < 1 || nparts > MAXP || part < 0 || part >= nparts)
    return fg_set_error(FG_EINVAL, "fg_share_create: nparts=%d part=%d (1 <= nparts <= %d)",
                        nparts, part, MAXP);
  if (n >= (1 << 28))
    return fg_set_error(FG_EUNSUPPORTED, "fg_share_create: n >= 2^28 does not fit the route word");
  if (row_offsets[0] != 0 || (int64_t)row_offsets[n] != m)
    return fg_set_error(FG_EINVAL, "fg_share_create: invalid CSR offsets");
  for (int32_t v = 0; v < n; ++v)
    if (owner[v] >= nparts)
      return fg_set_error(FG_EINVAL, "fg_share_create: owner[%d]=%d >= nparts", v, owner[v]);

  // ranks among each owner's vertices, hosted ids, proxies (ascending)
  std::vector<int32_t> rank(n), g2l(n, -1);
  int32_t per[MAXP] = {0};
  for (int32_t v = 0; v < n; ++v) rank[v] = per[owner[v]]++;
  int32_t nl = 0;
  for (int32_t v = 0; v < n; ++v)
    if (owner[v] == part) g2l[v] = nl++;
  std::vector<uint8_t> proxy(n, 0);
  for (int32_t v = 0; v < n; ++v) {
    if (owner[v] != part) continue;
    for (int32_t e = row_offsets[v]; e < row_offsets[v + 1]; ++e) {
      const int32_t u = col_idx[e];
      if (u < 0 || u >= n) return fg_set_error(FG_EINVAL, "fg_share_create: column out of range");
      if (owner[u] != part) proxy[u] = 1;
    }
  }
  int32_t nt = nl;
  for (int32_t v = 0; v < n; ++v)
    if (proxy[v]) g2l[v] = nt++;
  std::vector<int32_t> l2g(nt), conv(nt);
  std::vector<uint8_t> lown(nt);
  for (int32_t v = 0; v < n; ++v) {
    const int32_t l = g2l[v];
    if (l < 0) continue;
    l2g[l] = v;
    conv[l] = rank[v];
    lown[l] = owner[v];
  }
  std::vector<int32_t> loff((size_t)nt + 1);
  int64_t lm = 0;
  for (int32_t l = 0; l < nl; ++l) {
    const int32_t v = l2g[l];
    lm += row_offsets[v + 1] - row_offsets[v];
  }
  std::vector<int32_t> lcol((size_t)(lm > 0 ? lm : 1));
  int64_t k = 0;
  for (int32_t l = 0; l < nt; ++l) {
    loff[l] = (int32_t)k;
    if (l < nl) {
      const int32_t v = l2g[l];
      for (int32_t e = row_offsets[v]; e < row_offsets[v + 1]; ++e) lcol[k++] = g2l[col_idx[e]];
    }
  }
  loff[nt] = (int32_t)k;

  fg_share* s = new fg_share();
  s->n = n;
  s->n_local = nl;
  s->n_total = nt;
  s->nparts = nparts;
  s->part = part;
  s->m_local = lm;
  fg_status st = fg_graph_create_csr(nt, lm, loff.data(), lcol.data(), nullptr, 0u, stream,
                                     &s->graph);
  if (st != FG_OK) {
    fg_share_destroy(s);
    return st;
  }
  const size_t b_own = fg_align((size_t)nt), b_i32 = fg_align(sizeof(int32_t) * (size_t)nt);
  if (hipMalloc(&s->owned, b_own + 3 * b_i32) != hipSuccess) {
    fg_share_destroy(s);
    return fg_set_error(FG_ENOMEM, "fg_share_create: hipMalloc tables");
  }
  char* base = (char*)s->owned;
  s->owner = (uint8_t*)base;
  s->conv = (int32_t*)(base + b_own);
  s->l2g = (int32_t*)(base + b_own + b_i32);
  s->route = (uint32_t*)(base + b_own + 2 * b_i32);
  hipStream_t hs = (hipStream_t)stream;
  if (hipMemcpyAsync(s->owner, lown.data(), (size_t)nt, hipMemcpyHostToDevice, hs) != hipSuccess ||
      hipMemcpyAsync(s->conv, conv.data(), 4 * (size_t)nt, hipMemcpyHostToDevice, hs) != hipSuccess ||
      hipMemcpyAsync(s->l2g, l2g.data(), 4 * (size_t)nt, hipMemcpyHostToDevice, hs) != hipSuccess) {
    fg_share_destroy(s);
    return fg_set_error(FG_EDEVICE, "fg_share_create: copy tables");
  }
  int blocks = (int)((nt + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  route_kernel<<<blocks, 256, 0, hs>>>(nt, s->owner, s->conv, s->route);
  if (hipStreamSynchronize(hs) != hipSuccess) {
    fg_share_destroy(s);
    return fg_set_error(FG_EDEVICE, "fg_share_create: route table");
  }
  *out = s;
  return FG_OK;
}

extern "C" fg_status fg_share_info(const fg_share* s, fg_share_info_t* info) {
  if (!s || !info) return fg_set_error(FG_EINVAL, "fg_share_info: NULL argument");
  info->n_global = s->n;
  info->n_local = s->n_local;
  info->n_total = s->n_total;
  info->nparts = s->nparts;
  info->part = s->part;
  info->m_local = s->m_local;
  return FG_OK;
}

extern "C" const fg_graph* fg_share_graph(const fg_share* s) { return s ? s->graph : nullptr; }

extern "C" fg_status fg_share_tables(const fg_share* s, const uint8_t** owner,
                                     const int32_t** conv, const int32_t** l2g) {
  if (!s) return fg_set_error(FG_EINVAL, "fg_share_tables: share is NULL");
  if (owner) *owner = s->owner;
  if (conv) *conv = s->conv;
  if (l2g) *l2g = s->l2g;
  return FG_OK;
}

extern "C" size_t fg_package_workspace_bytes(const fg_share* s, int32_t max_len) {
  if (!s || max_len < 0) return 0;
  const int64_t tiles = ((int64_t)max_len + TILE - 1) / TILE + 1;
  return fg_align(sizeof(int32_t) * (size_t)(tiles * s->nparts));
}

extern "C" fg_status fg_package(const fg_share* s, const int32_t* frontier, int32_t len,
                                const int32_t* len_dev, const int32_t* depth,
                                const int32_t* parent, const fg_peer_bufs* out, void* ws,
                                size_t ws_bytes, void* stream) {
  if (!s || !out || !depth || !out->ids || !out->depth || !out->counts)
    return fg_set_error(FG_EINVAL, "fg_package: NULL argument");
  if (len < 0 || len > s->n_total)
    return fg_set_error(FG_EINVAL, "fg_package: len=%d outside [0, n_total=%d]", len, s->n_total);
  if (len > 0 && !frontier) return fg_set_error(FG_EINVAL, "fg_package: frontier is NULL");
  if (out->capacity < len)
    return fg_set_error(FG_EINVAL, "fg_package: capacity %lld < len %d",
                        (long long)out->capacity, len);
  if (parent && !out->parent)
    return fg_set_error(FG_EINVAL, "fg_package: parent given without an output buffer");
  const size_t need = fg_package_workspace_bytes(s, len);
  FG_CHECK_WS_ALIGN(ws, "fg_package");
  if (!ws || ws_bytes < need)
    return fg_set_error(FG_ENOMEM, "fg_package: workspace of %zu bytes < required %zu", ws_bytes,
                        need);
  hipStream_t hs = (hipStream_t)stream;
  const int32_t tiles = (int32_t)(((int64_t)len + TILE - 1) / TILE);
  int32_t* tile_cnt = (int32_t*)ws;
  if (tiles > 0)
    pkg_count_kernel<<<tiles, KB, 0, hs>>>(frontier, len, len_dev, s->route, s->n_local,
                                           s->part, s->nparts, tile_cnt);
  pkg_scan_kernel<<<1, KB, 0, hs>>>(tiles, s->nparts, tile_cnt, out->counts, s->part,
                                    out->local_count);
  if (tiles > 0)
    pkg_scatter_kernel<<<tiles, KB, 0, hs>>>(frontier, len, len_dev, s->route, s->l2g, s->n_local,
                                             s->part, s->nparts, depth, parent, tile_cnt, out->capacity,
                                             out->ids, out->depth, parent ? out->parent : nullptr,
                                             out->local);
  FG_HIP_TRY(hipGetLastError());
  return FG_OK;
}

extern "C" fg_status fg_combine(const fg_graph* g, const int32_t* ids, const int32_t* labels,
                                const int32_t* parents, int32_t len, const int32_t* len_dev,
                                uint32_t* visited, int32_t* depth, int32_t* parent,
                                int32_t* out_q, int32_t* out_len, void* stream) {
  if (!g || !visited || !depth || !out_q || !out_len)
    return fg_set_error(FG_EINVAL, "fg_combine: NULL argument");
  if (len < 0) return fg_set_error(FG_EINVAL, "fg_combine: negative len");
  if (len > 0 && (!ids || !labels)) return fg_set_error(FG_EINVAL, "fg_combine: NULL input");
  if (len == 0) return FG_OK;
  int blocks = (len + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  combine_kernel<<<blocks, 256, 0, (hipStream_t)stream>>>(ids, labels, parents, len, len_dev,
                                                          visited, depth, parent, out_q, out_len);
  FG_HIP_TRY(hipGetLastError());
  return FG_OK;
}
