// Graph loading (Sec. III-B initialisation step): CSR upload, validation,
// and the per-graph nonzero-degree mask used by the pull step.
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "fg_common.h"

namespace {

enum : uint32_t {
  VAL_OK = 0,
  VAL_OFF0 = 1,
  VAL_MONO = 2,
  VAL_LAST = 4,
  VAL_COL = 8,
  VAL_SORT = 16,
  VAL_SYM = 32,
  VAL_WSYM = 64,
};

// One wave per vertex: offsets monotone, columns in range, and (if `sym`)
// strictly ascending rows whose every edge u->v has v->u (same weight).
__global__ void validate_kernel(int32_t n, int64_t m, const int32_t* __restrict__ off,
                                const int32_t* __restrict__ col,
                                const uint32_t* __restrict__ w, int sym,
                                uint32_t* __restrict__ flags) {
  const int lane = fg_lane();
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / FG_WAVE;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / FG_WAVE;
  uint32_t bad = 0;
  if (wave == 0 && lane == 0) {
    if (off[0] != 0) bad |= VAL_OFF0;
    if ((int64_t)off[n] != m) bad |= VAL_LAST;
  }
  for (int64_t u = wave; u < n; u += nwaves) {
    int32_t b = off[u], e = off[u + 1];
    if (e < b) {
      bad |= VAL_MONO;
      continue;
    }
    if (b < 0 || (int64_t)e > m) {
      bad |= VAL_MONO;
      continue;
    }
    for (int32_t i = b + lane; i < e; i += FG_WAVE) {
      int32_t v = col[i];
      if (v < 0 || v >= n) {
        bad |= VAL_COL;
        continue;
      }
      if (!sym) continue;
      if (i > b && col[i - 1] >= v) bad |= VAL_SORT;
      // binary search u in row v
      int32_t lo = off[v], hi = off[v + 1];
      if (hi < lo) continue;
      int32_t lo0 = lo;
      while (lo < hi) {
        int32_t mid = lo + ((hi - lo) >> 1);
        if (col[mid] < (int32_t)u) lo = mid + 1; else hi = mid;
      }
      if (lo >= off[v + 1] || col[lo] != (int32_t)u) bad |= VAL_SYM;
      else if (w && w[lo] != w[i]) bad |= VAL_WSYM;
      (void)lo0;
    }
  }
  if (bad) atomicOr(flags, bad);
}

// nzmask words, maximum degree, count of nonzero-degree vertices, and the
// head table: the first four CSR entries of every vertex, contiguous by
// vertex id (entries past the degree repeat the last one; -1 for degree 0).
// An early-exit pull reads a vertex's first neighbours from it with one
// coalesced 16-byte load instead of one random cache line of the column
// array per vertex.
__global__ void degree_summary_kernel(int32_t n, int32_t nwords,
                                      const int32_t* __restrict__ off,
                                      const int32_t* __restrict__ col,
                                      uint64_t* __restrict__ nz,
                                      int4* __restrict__ head,
                                      int32_t* __restrict__ maxdeg,
                                      int32_t* __restrict__ nzcount) {
  const int lane = fg_lane();
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / FG_WAVE;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / FG_WAVE;
  int32_t mx = 0, cnt = 0;
  for (int64_t wd = wave; wd < nwords; wd += nwaves) {
    int64_t v = wd * 64 + lane;
    int32_t d = 0;
    if (v < n) {
      const int32_t b = off[v];
      d = off[v + 1] - b;
      int4 h = make_int4(-1, -1, -1, -1);
      if (d > 0) {
        const int32_t l = b + d - 1;
        h = make_int4(col[b], col[b + 1 < l ? b + 1 : l], col[b + 2 < l ? b + 2 : l],
                      col[b + 3 < l ? b + 3 : l]);
      }
      head[v] = h;
    }
    uint64_t bits = __ballot(d > 0);
    if (lane == 0) nz[wd] = bits;
    mx = d > mx ? d : mx;
    cnt += d > 0;
  }
  for (int s = 32; s > 0; s >>= 1) {
    int32_t o = __shfl_xor(mx, s, 64);
    mx = o > mx ? o : mx;
    cnt += __shfl_xor(cnt, s, 64);
  }
  if (lane == 0) {
    atomicMax(maxdeg, mx);
    atomicAdd(nzcount, cnt);
  }
}

// Sum and maximum of the edge weights (the SSSP kernel's default near-far
// step uses the mean).
__global__ void weight_summary_kernel(int64_t m, const uint32_t* __restrict__ w,
                                      unsigned long long* __restrict__ sum,
                                      uint32_t* __restrict__ mx) {
  unsigned long long s = 0;
  uint32_t x = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t v = w[i];
    s += v;
    x = v > x ? v : x;
  }
  for (int d = 32; d > 0; d >>= 1) {
    s += __shfl_xor(s, d, 64);
    const uint32_t o = __shfl_xor(x, d, 64);
    x = o > x ? o : x;
  }
  if (fg_lane() == 0) {
    atomicAdd(sum, s);
    atomicMax(mx, x);
  }
}

const char* describe(uint32_t f) {
  if (f & VAL_OFF0) return "row_offsets[0] != 0";
  if (f & VAL_LAST) return "row_offsets[n] != m";
  if (f & VAL_MONO) return "row_offsets not monotone / out of [0, m]";
  if (f & VAL_COL) return "column index outside [0, n)";
  if (f & VAL_SORT) return "FG_SYMMETRIC validation needs strictly ascending rows";
  if (f & VAL_SYM) return "graph is not symmetric (u->v without v->u)";
  if (f & VAL_WSYM) return "weights differ between u->v and v->u";
  return "unknown";
}

}  // namespace

extern "C" fg_status fg_graph_destroy(fg_graph* g) {
  if (!g) return FG_OK;
  hipSetDevice(g->device);
  hipDeviceSynchronize();
  for (void* p : g->owned)
    if (p) hipFree(p);
  delete g;
  return FG_OK;
}

extern "C" fg_status fg_graph_create_csr(int32_t n, int64_t m, const int32_t* row_offsets,
                                         const int32_t* col_idx, const uint32_t* weights,
                                         uint32_t flags, void* stream, fg_graph** out) {
  if (!out) return fg_set_error(FG_EINVAL, "fg_graph_create_csr: out is NULL");
  *out = nullptr;
  if (n < 1) return fg_set_error(FG_EINVAL, "fg_graph_create_csr: n=%d < 1", n);
  if (m < 0 || m >= (int64_t(1) << 31))
    return fg_set_error(FG_EINVAL, "fg_graph_create_csr: m=%lld outside [0, 2^31)", (long long)m);
  if (!row_offsets || (m > 0 && !col_idx))
    return fg_set_error(FG_EINVAL, "fg_graph_create_csr: NULL CSR array");
  if ((flags & FG_BORROW) && !(flags & FG_DEVICE_PTRS))
    return fg_set_error(FG_EINVAL, "fg_graph_create_csr: FG_BORROW needs FG_DEVICE_PTRS");
  hipStream_t s = (hipStream_t)stream;
  fg_graph* g = new fg_graph();
  g->n = n;
  g->m = m;
  g->nwords = (n + 63) / 64;
  g->symmetric = (flags & FG_SYMMETRIC) ? 1 : 0;
  hipGetDevice(&g->device);

  auto fail = [&](fg_status st) {
    fg_graph_destroy(g);
    return st;
  };
  const bool dev = (flags & FG_DEVICE_PTRS) != 0;
  const size_t ob = sizeof(int32_t) * ((size_t)n + 1);
  const size_t cb = sizeof(int32_t) * (size_t)(m > 0 ? m : 1);
  const size_t wb = sizeof(uint32_t) * (size_t)(m > 0 ? m : 1);

  if (flags & FG_BORROW) {
    g->off = row_offsets;
    g->col = col_idx;
    g->w = weights;
  } else {
    void *po = nullptr, *pc = nullptr, *pw = nullptr;
    if (hipMalloc(&po, ob) != hipSuccess) return fail(fg_set_error(FG_ENOMEM, "hipMalloc offsets"));
    g->owned[0] = po;
    if (hipMalloc(&pc, cb) != hipSuccess) return fail(fg_set_error(FG_ENOMEM, "hipMalloc cols"));
    g->owned[1] = pc;
    hipMemcpyKind kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if (hipMemcpyAsync(po, row_offsets, ob, kind, s) != hipSuccess)
      return fail(fg_set_error(FG_EDEVICE, "copy offsets"));
    if (m > 0 && hipMemcpyAsync(pc, col_idx, sizeof(int32_t) * (size_t)m, kind, s) != hipSuccess)
      return fail(fg_set_error(FG_EDEVICE, "copy cols"));
    if (weights) {
      if (hipMalloc(&pw, wb) != hipSuccess) return fail(fg_set_error(FG_ENOMEM, "hipMalloc weights"));
      g->owned[2] = pw;
      if (m > 0 && hipMemcpyAsync(pw, weights, sizeof(uint32_t) * (size_t)m, kind, s) != hipSuccess)
        return fail(fg_set_error(FG_EDEVICE, "copy weights"));
    }
    g->off = (const int32_t*)po;
    g->col = (const int32_t*)pc;
    g->w = (const uint32_t*)pw;
    g->resident_bytes += (int64_t)(fg_align(ob) + fg_align(cb) + (weights ? fg_align(wb) : 0));
  }

  // Host-side check of the offsets before any kernel walks them.
  if (flags & FG_VALIDATE) {
    if (!dev) {
      if (row_offsets[0] != 0) return fail(fg_set_error(FG_EINVAL, "invalid CSR: row_offsets[0] != 0"));
      for (int32_t i = 0; i < n; ++i)
        if (row_offsets[i + 1] < row_offsets[i] || row_offsets[i + 1] > m)
          return fail(fg_set_error(FG_EINVAL, "invalid CSR: row_offsets not monotone at %d", i));
      if ((int64_t)row_offsets[n] != m)
        return fail(fg_set_error(FG_EINVAL, "invalid CSR: row_offsets[n] != m"));
    }
  }

  void* aux = nullptr;
  const size_t nzb = sizeof(uint64_t) * (size_t)g->nwords;
  const size_t hb = sizeof(int4) * (size_t)n;
  if (hipMalloc(&aux, fg_align(nzb) + 256 + fg_align(hb)) != hipSuccess)
    return fail(fg_set_error(FG_ENOMEM, "hipMalloc aux"));
  g->owned[3] = aux;
  g->nzmask = (uint64_t*)aux;
  int32_t* dsum = (int32_t*)((char*)aux + fg_align(nzb));  // maxdeg, nzcount, flags
  g->head = (int4*)((char*)aux + fg_align(nzb) + 256);
  g->resident_bytes += (int64_t)(fg_align(nzb) + 256 + fg_align(hb));
  if (hipMemsetAsync(dsum, 0, 32, s) != hipSuccess) return fail(fg_set_error(FG_EDEVICE, "memset"));

  if (flags & FG_VALIDATE) {
    if (dev) {
      // offsets must be sane before the row walk: check them first on device
      std::vector<int32_t> hoff((size_t)n + 1);
      if (hipMemcpyAsync(hoff.data(), g->off, ob, hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return fail(fg_set_error(FG_EDEVICE, "read back offsets"));
      if (hoff[0] != 0) return fail(fg_set_error(FG_EINVAL, "invalid CSR: row_offsets[0] != 0"));
      for (int32_t i = 0; i < n; ++i)
        if (hoff[i + 1] < hoff[i] || hoff[i + 1] > m)
          return fail(fg_set_error(FG_EINVAL, "invalid CSR: row_offsets not monotone at %d", i));
      if ((int64_t)hoff[n] != m) return fail(fg_set_error(FG_EINVAL, "invalid CSR: row_offsets[n] != m"));
    }
    validate_kernel<<<1024, 256, 0, s>>>(n, m, g->off, g->col, g->w, g->symmetric,
                                         (uint32_t*)(dsum + 2));
    uint32_t f = 0;
    if (hipMemcpyAsync(&f, dsum + 2, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail(fg_set_error(FG_EDEVICE, "validation kernel failed"));
    if (f) return fail(fg_set_error(FG_EINVAL, "invalid CSR: %s", describe(f)));
  }

  int blocks = (int)((g->nwords + 3) / 4);
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  degree_summary_kernel<<<blocks, 256, 0, s>>>(n, g->nwords, g->off, g->col, g->nzmask, g->head,
                                               dsum, dsum + 1);
  if (g->w && m > 0) {
    int wb = (int)((m + 1023) / 1024);
    if (wb > 4096) wb = 4096;
    weight_summary_kernel<<<wb, 256, 0, s>>>(m, g->w, (unsigned long long*)(dsum + 4),
                                             (uint32_t*)(dsum + 6));
  }
  int32_t hs[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (hipMemcpyAsync(hs, dsum, 32, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(fg_set_error(FG_EDEVICE, "degree summary failed"));
  g->max_degree = hs[0];
  g->nonzero_degree = hs[1];
  memcpy(&g->w_sum, &hs[4], 8);
  g->w_max = (uint32_t)hs[6];
  *out = g;
  return FG_OK;
}

extern "C" fg_status fg_graph_info(const fg_graph* g, fg_graph_info_t* info) {
  if (!g || !info) return fg_set_error(FG_EINVAL, "fg_graph_info: NULL argument");
  info->n = g->n;
  info->m = g->m;
  info->has_weights = g->w != nullptr;
  info->symmetric = g->symmetric;
  info->max_degree = g->max_degree;
  info->nonzero_degree = g->nonzero_degree;
  info->device = g->device;
  info->resident_bytes = g->resident_bytes;
  return FG_OK;
}

extern "C" fg_status fg_graph_csr(const fg_graph* g, const int32_t** row_offsets,
                                  const int32_t** col_idx, const uint32_t** weights) {
  if (!g) return fg_set_error(FG_EINVAL, "fg_graph_csr: graph is NULL");
  if (row_offsets) *row_offsets = g->off;
  if (col_idx) *col_idx = g->col;
  if (weights) *weights = g->w;
  return FG_OK;
}
