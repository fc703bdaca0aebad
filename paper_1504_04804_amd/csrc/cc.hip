// Connected components (Table I's CC primitive; the hooking and
// pointer-jumping scheme of Soman et al. that the paper cites): every
// vertex is labelled with the smallest vertex id of its component.
//
// The label array itself holds a forest in which every vertex points to a
// smaller (or equal) vertex of its own component.  Hooking an edge {u, v}
// finds both roots (with path halving: the pointer jumping) and links the
// larger root under the smaller one by a compare-and-swap that succeeds
// only while it is still a root (a failed swap returns the new parent, from
// which the search continues).  Links only ever point to a smaller root, so
// the smallest vertex of a component is never linked and ends as the root
// of the whole component: the labels are the component minima whatever the
// order of the hooks.
//
// The order of the hooks is free, which the passes use (the neighbour
// sampling of Sutton, Ben-Nun and Barak's Afforest):
//   link     every vertex hooks its first two neighbours (the graph's head
//            table: one coalesced 16-byte load per vertex); on graphs with
//            hubs the first one while the labels are initialised, by
//            pointing the vertex at its first neighbour when that is
//            smaller (a forest already, no atomics)
//   compress every label becomes its root
//   sample   the most frequent root of 1024 sampled vertices, c: on graphs
//            with a giant component, that component's root
//   hook     every row of a vertex outside c's tree is hooked in full
//            (entries after the first two); rows of c's members are
//            skipped: each of their edges either stays inside c's tree or
//            is hooked from the other end's row
//   compress every label becomes its root (walks without re-pointing).
// The hook pass is edge-balanced: each task is a fixed range of CSR
// entries whose rows are found with a binary search over the offsets
// (staged in LDS), so a row of any length costs its share of the range,
// and the entries of skipped rows cost no column read; a task none of whose
// rows has work is left after one label read per row.
#include <string.h>

#include "fg_common.h"

namespace {

constexpr int CC_BT = 256;
constexpr int CC_TASK = 4096;           // CSR entries per workgroup task
constexpr int CC_LDS_OFF = 4096 + 2;    // offsets staged per task
constexpr int CC_SAMPLES = 1024;
constexpr int CC_SKIP = 2;              // entries per row hooked by the link pass

struct CcCtl {
  int32_t giant;                // the sampled most frequent root
  int32_t pad;
  unsigned long long comps;     // number of components
};

// Root of x with path halving: each visited vertex is re-pointed at its
// grandparent.  A vertex only ever points to a smaller vertex of its own
// tree (stale reads included: trees only merge), so the walk always ends
// at a vertex that was a root when it was read.
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

// Root of x without re-pointing (for passes that publish roots): once a
// vertex holds its root, a path-halving store from a walk that passed it
// earlier could put an intermediate vertex back.
__device__ __forceinline__ int32_t cc_root(const int32_t* p, int32_t x) {
  int32_t cur = p[x];
  while (cur != x) {
    x = cur;
    cur = p[x];
  }
  return cur;
}

// label[v] = v, or v's first neighbour where that one is smaller: already
// a forest of pointers to smaller vertices of the same component, written
// without atomics (the first link of the link pass).
__global__ __launch_bounds__(CC_BT) void cc_init_kernel(int32_t n, const int4* __restrict__ head,
                                                        const int32_t* __restrict__ off,
                                                        int32_t* __restrict__ label,
                                                        CcCtl* __restrict__ ctl) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    int32_t l = (int32_t)v;
    if (head && off[v + 1] > off[v]) {
      const int32_t u = head[v].x;
      if (u < l) l = u;
    }
    label[v] = l;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ctl->giant = -1;
    ctl->comps = 0;
  }
}

// Hooks from the head table: the first entry of every row (LINK_FIRST),
// the second (LINK_SECOND), or the second and, where the init pass did not
// link it (a first neighbour larger than the vertex), the first
// (LINK_REST).  After the passes run, both first entries of every row are
// hooked.
constexpr int LINK_FIRST = 0, LINK_SECOND = 1, LINK_REST = 2;
__global__ __launch_bounds__(CC_BT) void cc_link_kernel(int32_t n, const int4* __restrict__ head,
                                                        const int32_t* __restrict__ off,
                                                        int32_t what, int32_t* __restrict__ label) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    const int4 h = head[v];
    const int32_t deg = off[v + 1] - off[v];
    if (what != LINK_SECOND && deg > 0 && (what == LINK_FIRST ? h.x != (int32_t)v : h.x > (int32_t)v))
      cc_unite(label, (int32_t)v, h.x);
    if (what != LINK_FIRST && deg > 1 && h.y != (int32_t)v) cc_unite(label, (int32_t)v, h.y);
  }
}

// label[v] = root of v; counts the roots when `ctl` is given.
__global__ __launch_bounds__(CC_BT) void cc_compress_kernel(int32_t n, int32_t* __restrict__ label,
                                                            CcCtl* __restrict__ ctl) {
  unsigned long long roots = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t r = cc_root(label, (int32_t)v);
    label[v] = r;
    roots += r == (int32_t)v;
  }
  if (!ctl) return;
  roots = fg_wave_sum(roots);
  if (fg_lane() == 0 && roots) atomicAdd(&ctl->comps, roots);
}

// The most frequent label among CC_SAMPLES spread-out vertices (one
// workgroup of CC_SAMPLES threads; ties go to the smaller label).
__global__ __launch_bounds__(CC_SAMPLES) void cc_sample_kernel(int32_t n,
                                                               const int32_t* __restrict__ label,
                                                               CcCtl* __restrict__ ctl) {
  __shared__ int32_t s_lab[CC_SAMPLES];
  __shared__ unsigned long long s_best[CC_SAMPLES / FG_WAVE];
  const int t = threadIdx.x;
  const uint64_t v = ((uint64_t)t * 0x9E3779B97F4A7C15ull + 0x5851F42D4C957F2Dull) % (uint64_t)n;
  const int32_t mine = label[v];
  s_lab[t] = mine;
  __syncthreads();
  int32_t cnt = 0;
  for (int j = 0; j < CC_SAMPLES; ++j) cnt += s_lab[j] == mine;
  // key: count high, then the smaller label
  unsigned long long key = ((unsigned long long)cnt << 32) | (uint32_t)(0x7fffffff - mine);
  for (int s = FG_WAVE / 2; s > 0; s >>= 1) {
    const unsigned long long o = __shfl_xor(key, s, FG_WAVE);
    key = o > key ? o : key;
  }
  if (fg_lane() == 0) s_best[t / FG_WAVE] = key;
  __syncthreads();
  if (t == 0) {
    unsigned long long b = 0;
    for (int w = 0; w < CC_SAMPLES / FG_WAVE; ++w) b = s_best[w] > b ? s_best[w] : b;
    ctl->giant = 0x7fffffff - (int32_t)(uint32_t)b;
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
                                                        int32_t* __restrict__ label,
                                                        const CcCtl* __restrict__ ctl) {
  __shared__ int32_t s_off[CC_LDS_OFF];
  __shared__ int32_t s_u0, s_u1;
  const int32_t giant = ctl->giant;
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
    // a task whose rows all lie in the sampled tree (or have no entry past
    // the first two) has nothing to hook: one look at each row's label
    // instead of a search per entry
    int todo = 0;
    for (int32_t i = threadIdx.x; i <= u1 - u0 && !todo; i += CC_BT) {
      const int32_t u = u0 + i;
      const int32_t deg = staged ? s_off[i + 1] - s_off[i] : off[u + 1] - off[u];
      todo = deg > CC_SKIP && label[u] != giant;
    }
    if (!__syncthreads_or(todo)) continue;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += CC_BT) {
      int32_t u, first;
      if (staged) {
        int32_t lo = 0, hi = u1 - u0;
        while (lo < hi) {
          const int32_t mid = (lo + hi + 1) >> 1;
          if ((int64_t)s_off[mid] <= e) lo = mid; else hi = mid - 1;
        }
        u = u0 + lo;
        first = s_off[lo];
      } else {
        u = row_of(off, u0, u1, e);
        first = off[u];
      }
      if (e - first < CC_SKIP) continue;      // hooked by the link pass
      if (label[u] == giant) continue;        // a member of the sampled tree
      const int32_t v = col[e];
      if (v != u) cc_unite(label, u, v);
    }
  }
}

}  // namespace

size_t fg_cc_workspace_bytes(const fg_graph*) { return fg_align(sizeof(CcCtl)); }

extern "C" fg_status fg_cc(const fg_graph* g, int32_t* label, int64_t* components, void* ws,
                           size_t ws_bytes, void* stream) {
  if (!g || !label || !ws) return fg_set_error(FG_EINVAL, "fg_cc: NULL argument");
  if (!g->symmetric)
    return fg_set_error(FG_EUNSUPPORTED, "fg_cc: needs an undirected graph (FG_SYMMETRIC)");
  FG_CHECK_WS_ALIGN(ws, "fg_cc");
  if (ws_bytes < sizeof(CcCtl))
    return fg_set_error(FG_ENOMEM, "fg_cc: workspace of %zu bytes < required %zu", ws_bytes,
                        sizeof(CcCtl));
  hipStream_t s = (hipStream_t)stream;
  CcCtl* ctl = (CcCtl*)ws;
  const int cus = fg_props(g->device).cus;
  const int grid = (cus > 0 ? cus : 256) * 8;
  // On graphs with hubs (mean degree above 8) a vertex's first neighbour is
  // usually a smaller hub, and the init pass links it for free; on grids
  // and road-like graphs that would chain every vertex to the one before
  // it, so they hook both first entries by compare-and-swap.
  const bool init_link = g->m > 8 * (int64_t)g->n;
  cc_init_kernel<<<grid, CC_BT, 0, s>>>(g->n, init_link ? g->head : nullptr, g->off, label, ctl);
  if (g->m > 0) {
    if (init_link) {
      cc_link_kernel<<<grid, CC_BT, 0, s>>>(g->n, g->head, g->off, LINK_REST, label);
    } else {
      cc_link_kernel<<<grid, CC_BT, 0, s>>>(g->n, g->head, g->off, LINK_FIRST, label);
      cc_link_kernel<<<grid, CC_BT, 0, s>>>(g->n, g->head, g->off, LINK_SECOND, label);
    }
    cc_compress_kernel<<<grid, CC_BT, 0, s>>>(g->n, label, nullptr);
    cc_sample_kernel<<<1, CC_SAMPLES, 0, s>>>(g->n, label, ctl);
    cc_hook_kernel<<<grid, CC_BT, 0, s>>>(g->n, g->m, g->off, g->col, label, ctl);
  }
  cc_compress_kernel<<<grid, CC_BT, 0, s>>>(g->n, label, ctl);
  if (components)
    FG_HIP_TRY(hipMemcpyAsync(components, &ctl->comps, sizeof(int64_t), hipMemcpyDeviceToDevice, s));
  FG_HIP_TRY(hipGetLastError());
  return FG_OK;
}
