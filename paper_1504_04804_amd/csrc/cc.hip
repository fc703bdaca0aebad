// Connected components (Table I's CC primitive; the hooking and
// pointer-jumping scheme of Soman et al. that the paper cites): every
// vertex is labelled with the smallest vertex id of its component.
//
// The label array itself holds a forest in which every vertex points to a
// smaller (or equal) vertex of its own component:
//   init     label[v] = min(v, first neighbour of v)
//   hook     every undirected edge {u, v} (the CSR entry with v < u) joins
//            the trees of u and v: both roots are found (with path halving,
//            the pointer jumping), and the larger root is linked under the
//            smaller one by a compare-and-swap that succeeds only while it
//            is still a root (a failed swap returns the new parent, from
//            which the search continues)
//   compress label[v] = the root of v's tree.
// Links only ever point to a smaller root, so the smallest vertex of a
// component is never linked and ends as the root of the whole component:
// the labels are the component minima whatever the order of the hooks.
// The hook pass is edge-balanced: each task is a fixed range of CSR
// entries whose rows are found with a binary search over the offsets
// (staged in LDS), so a row of any length costs its share of the range.
#include <string.h>

#include "fg_common.h"

namespace {

constexpr int CC_BT = 256;
constexpr int CC_TASK = 4096;           // CSR entries per workgroup task
constexpr int CC_LDS_OFF = 4096 + 2;    // offsets staged per task

// Root of x with path halving: each visited vertex is re-pointed at its
// grandparent.  Every value read (even a stale one) is an ancestor, because
// parents only move to ancestors, so the walk always ends at a vertex that
// was a root when it was read.
__device__ __forceinline__ int32_t cc_find(int32_t* __restrict__ p, int32_t x) {
  int32_t cur = p[x];
  if (cur == x) return x;
  int32_t prev = x;
  int32_t next;
  while (cur > (next = p[cur])) {
    p[prev] = next;
    prev = cur;
    cur = next;
  }
  return cur;
}

// Joins the trees of a and b (hooking): the larger root goes under the
// smaller one while it is still a root.
__device__ __forceinline__ void cc_unite(int32_t* __restrict__ p, int32_t a, int32_t b) {
  int32_t ra = cc_find(p, a);
  int32_t rb = cc_find(p, b);
  while (ra != rb) {
    if (ra < rb) {
      const int32_t t = ra;
      ra = rb;
      rb = t;
    }
    const int32_t old = atomicCAS(&p[ra], ra, rb);
    if (old == ra) return;
    ra = cc_find(p, old);
  }
}

__global__ __launch_bounds__(CC_BT) void cc_init_kernel(int32_t n, const int4* __restrict__ head,
                                                        int32_t* __restrict__ label) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t f = head[v].x;  // first neighbour, -1 for degree 0
    label[v] = (f >= 0 && f < (int32_t)v) ? f : (int32_t)v;
  }
}

// Largest u in [lo, hi] with off[u] <= e.
__device__ __forceinline__ int32_t row_of(const int32_t* __restrict__ off, int32_t lo, int32_t hi,
                                          int64_t e) {
  while (lo < hi) {
    const int32_t mid = lo + ((hi - lo + 1) >> 1);
    if ((int64_t)off[mid] <= e) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(CC_BT) void cc_hook_kernel(int32_t n, int64_t m,
                                                        const int32_t* __restrict__ off,
                                                        const int32_t* __restrict__ col,
                                                        int32_t* __restrict__ label) {
  __shared__ int32_t s_off[CC_LDS_OFF];
  __shared__ int32_t s_u0, s_u1;
  const int64_t ntasks = (m + CC_TASK - 1) / CC_TASK;
  for (int64_t t = blockIdx.x; t < ntasks; t += gridDim.x) {
    const int64_t e0 = t * CC_TASK;
    const int64_t e1 = (e0 + CC_TASK < m ? e0 + CC_TASK : m);
    __syncthreads();
    if (threadIdx.x == 0) {
      // rows holding entries e0 and e1 - 1 (rows with no entries are skipped
      // by the search: it returns the last row starting at or before e)
      s_u0 = row_of(off, 0, n - 1, e0);
      s_u1 = row_of(off, s_u0, n - 1, e1 - 1);
    }
    __syncthreads();
    const int32_t u0 = s_u0, u1 = s_u1;
    const int32_t span = u1 - u0 + 2;  // offsets u0 .. u1 + 1
    const bool staged = span <= CC_LDS_OFF;
    if (staged)
      for (int32_t i = threadIdx.x; i < span; i += CC_BT) s_off[i] = off[u0 + i];
    __syncthreads();
    for (int64_t e = e0 + threadIdx.x; e < e1; e += CC_BT) {
      int32_t u;
      if (staged) {
        int32_t lo = 0, hi = u1 - u0;
        while (lo < hi) {
          const int32_t mid = (lo + hi + 1) >> 1;
          if ((int64_t)s_off[mid] <= e) lo = mid; else hi = mid - 1;
        }
        u = u0 + lo;
      } else {
        u = row_of(off, u0, u1, e);
      }
      const int32_t v = col[e];
      if (v < u) cc_unite(label, u, v);
    }
  }
}

// The final pass walks without re-pointing: once a vertex holds its root,
// a path-halving store from a walk that passed it earlier could put an
// intermediate vertex back.  Concurrent walks only ever see parents or
// roots, so each still ends at its root.
__device__ __forceinline__ int32_t cc_root(const int32_t* p, int32_t x) {
  int32_t cur = p[x];
  while (cur != x) {
    x = cur;
    cur = p[x];
  }
  return cur;
}

__global__ __launch_bounds__(CC_BT) void cc_compress_kernel(int32_t n, int32_t* __restrict__ label,
                                                            unsigned long long* __restrict__ ncomp) {
  unsigned long long roots = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t r = cc_root(label, (int32_t)v);
    label[v] = r;
    roots += r == (int32_t)v;
  }
  roots = fg_wave_sum(roots);
  if (fg_lane() == 0 && roots && ncomp) atomicAdd(ncomp, roots);
}

__global__ void cc_zero_kernel(unsigned long long* p) {
  if (threadIdx.x == 0) *p = 0;
}

}  // namespace

extern "C" fg_status fg_cc(const fg_graph* g, int32_t* label, int64_t* components,
                           void* stream) {
  if (!g || !label) return fg_set_error(FG_EINVAL, "fg_cc: NULL argument");
  if (!g->symmetric)
    return fg_set_error(FG_EUNSUPPORTED, "fg_cc: needs an undirected graph (FG_SYMMETRIC)");
  hipStream_t s = (hipStream_t)stream;
  const int cus = fg_props(g->device).cus;
  const int grid = (cus > 0 ? cus : 256) * 8;
  unsigned long long* nc = (unsigned long long*)components;
  if (nc) cc_zero_kernel<<<1, 64, 0, s>>>(nc);
  cc_init_kernel<<<grid, CC_BT, 0, s>>>(g->n, g->head, label);
  if (g->m > 0) cc_hook_kernel<<<grid, CC_BT, 0, s>>>(g->n, g->m, g->off, g->col, label);
  cc_compress_kernel<<<grid, CC_BT, 0, s>>>(g->n, label, nc);
  FG_HIP_TRY(hipGetLastError());
  return FG_OK;
}
