// PageRank by power iteration in double precision (Table I's PR primitive;
// the rank update and the accumulation over edges of Alg. 3), on an
// undirected CSR where every edge carries rank both ways.
//
// rank_0(v) = 1/n.  Iteration i reads contrib_i(u) = rank_i(u) / deg(u) and
// writes, for every vertex v,
//   acc(v)         = sum over the neighbours u of v of contrib_i(u)
//   rank_{i+1}(v)  = (1 - d)/n + d acc(v)
//   contrib_{i+1}(v) = rank_{i+1}(v) / deg(v)   (0 for degree 0)
// in one pass: the accumulation is a gather over v's own row (a pull, no
// atomics), so each vertex's new rank is final when its row is done.  Rows
// of fewer than 64 entries are laid end to end over a wave's lanes (64
// entries per step, segmented sums), rows up to PR_LONG entries are summed
// by one wave each and longer rows by one workgroup (listed once per call
// and taken first); every row's sum is formed in a fixed order.  Convergence (the threshold ratio): the run stops
// after an iteration in which every vertex changed by at most tol times its
// previous rank; tol = 0 runs max_iter iterations.  Every iteration is a
// launch that returns at once when the run has already stopped, so the
// host enqueues all of them without reading anything back.
#include <math.h>
#include <string.h>

#include "fg_common.h"
#include "frontier.h"

namespace {

constexpr int PR_BT = 256;
constexpr int PR_LONG = 4096;  // rows at least this long are summed by a workgroup

struct PrCtl {
  uint32_t next_item[2];  // work counters, slot = iteration parity
  uint32_t blocks_done;
  int32_t nlong;          // rows of at least PR_LONG entries
  int32_t done;           // converged (tol > 0)
  int32_t iterations;
  unsigned long long notconv[2];  // vertices above the threshold, slot = parity
};

struct PrArgs {
  int32_t n;
  int64_t m;
  const int32_t* off;
  const int32_t* col;
  double d;      // damping
  double base;   // (1 - d) / n
  double tol;
  double* rank;
  double* contrib[2];
  int32_t* longrows;
  PrCtl* ctl;
  fg_run_stats* stats;
  int32_t clock_khz;
};

__device__ __forceinline__ double wave_sum_f64(double x) {
#pragma unroll
  for (int s = FG_WAVE / 2; s > 0; s >>= 1) x += __shfl_xor(x, s, FG_WAVE);
  return x;
}

// The update of one vertex from its accumulated sum (no contraction into
// fused multiply-adds: the products and sums round as written).
__device__ __forceinline__ unsigned long long pr_update(const PrArgs& A, double* nxt, int32_t v,
                                                        int32_t deg, double acc) {
  const double nr = __dadd_rn(A.base, __dmul_rn(A.d, acc));
  const double old = A.rank[v];
  const double diff = nr > old ? __dsub_rn(nr, old) : __dsub_rn(old, nr);
  A.rank[v] = nr;
  nxt[v] = deg > 0 ? nr / (double)deg : 0.0;
  return diff > __dmul_rn(A.tol, old) ? 1ull : 0ull;
}

__global__ __launch_bounds__(PR_BT) void pr_setup_kernel(PrArgs A, double inv_n) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = tid; v < A.n; v += nth) {
    const int32_t deg = A.off[v + 1] - A.off[v];
    A.rank[v] = inv_n;
    A.contrib[0][v] = deg > 0 ? inv_n / (double)deg : 0.0;
    if (deg >= PR_LONG) A.longrows[atomicAdd(&A.ctl->nlong, 1)] = (int32_t)v;
  }
  if (tid == 0 && A.stats) {
    fg_run_stats* st = A.stats;
    st->status = FG_OK;
    st->iterations = 0;
    st->reached = A.n;
    st->edges_inspected = 0;
    st->direction_switches = 0;
    st->grid_blocks = 0;
    st->clock_khz = A.clock_khz;
    st->t_start = (int64_t)wall_clock64();
  }
}

__global__ void pr_reset_kernel(PrCtl* c) {
  if (threadIdx.x == 0) {
    PrCtl z;
    memset(&z, 0, sizeof(z));
    *c = z;
  }
}

// Sum of x over the lanes of this lane's run of equal `key` up to this
// lane (runs are adjacent lanes; `start` = the run's first lane), in a
// fixed order.
__device__ __forceinline__ double seg_incl_sum(double x, int lane, int start) {
#pragma unroll
  for (int dd = 1; dd < FG_WAVE; dd <<= 1) {
    const double y = __shfl_up(x, dd, FG_WAVE);
    if (lane - dd >= start) x += y;
  }
  return x;
}

// Sum of cur[col[i]] for i = first, first + stride, ... < end, with four
// independent partial sums so that four gathers per thread are in flight
// (a long row is otherwise a chain of dependent column-then-value loads,
// and the longest row held its workgroup for most of an iteration; eight
// partial sums measured no faster); the order of the additions is fixed.
__device__ __forceinline__ double strided_gather_sum(const double* cur, const int32_t* col,
                                                     int32_t first, int32_t end, int32_t stride) {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int32_t i = first;
  // every index of a round is below `end`: i < end - 3 * stride (no
  // overflow: end >= 0 and 3 * stride is small)
  for (; i < end - 3 * stride; i += 4 * stride) {
    const int32_t c0 = col[i];
    const int32_t c1 = col[i + stride];
    const int32_t c2 = col[i + 2 * stride];
    const int32_t c3 = col[i + 3 * stride];
    a0 += cur[c0];
    a1 += cur[c1];
    a2 += cur[c2];
    a3 += cur[c3];
  }
  for (; i < end; i += stride) a0 += cur[col[i]];
  return (a0 + a1) + (a2 + a3);
}

__global__ __launch_bounds__(PR_BT) void pr_iter_kernel(PrArgs A, int32_t it) {
  __shared__ int32_t s_item;
  __shared__ int s_last;
  __shared__ double s_red[PR_BT / FG_WAVE];
  // short rows of each wave's 64 vertices: exclusive prefix of their
  // lengths, their first entries, their sums
  __shared__ int32_t s_sc[PR_BT / FG_WAVE][FG_WAVE];
  __shared__ int32_t s_sb[PR_BT / FG_WAVE][FG_WAVE];
  __shared__ double s_acc[PR_BT / FG_WAVE][FG_WAVE];
  PrCtl* C = A.ctl;
  if (C->done) return;
  const int par = it & 1;
  const double* cur = A.contrib[par];
  double* nxt = A.contrib[par ^ 1];
  const int lane = fg_lane();
  const int wid = threadIdx.x / FG_WAVE;
  const int32_t nlong = C->nlong;
  const int64_t ngroups = ((int64_t)A.n + PR_BT - 1) / PR_BT;
  const int64_t items = (int64_t)nlong + ngroups;
  unsigned long long nc = 0;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_item = (int32_t)atomicAdd(&C->next_item[par], 1u);
    __syncthreads();
    const int64_t item = s_item;
    if (item >= items) break;
    if (item < nlong) {
      // one long row, the whole workgroup
      const int32_t v = A.longrows[item];
      const int32_t b = A.off[v], e = A.off[v + 1];
      double acc = strided_gather_sum(cur, A.col, b + (int32_t)threadIdx.x, e, PR_BT);
      acc = wave_sum_f64(acc);
      if (lane == 0) s_red[wid] = acc;
      __syncthreads();
      if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < PR_BT / FG_WAVE; ++w) t += s_red[w];
        nc += pr_update(A, nxt, v, e - b, t);
      }
      continue;
    }
    // 256 consecutive vertices, 64 per wave
    const int64_t v64 = (item - nlong) * PR_BT + threadIdx.x;
    const int32_t v = (int32_t)v64;
    int32_t b = 0, deg = 0;
    if (v64 < A.n) {
      b = A.off[v];
      deg = A.off[v + 1] - b;
    }
    {
      // short rows: the wave's rows laid end to end and taken 64 entries
      // per step, one per lane (all the contribution loads of a step in
      // flight together); a step's lanes of one row (adjacent) are summed
      // by a segmented scan and its last lane adds the part to the row's
      // sum, so every row is summed in a fixed order
      const int32_t ds = (v64 < A.n && deg < FG_WAVE) ? deg : 0;
      const int32_t incl = fg_wave_incl_scan(ds);
      const int32_t T = __builtin_amdgcn_readlane(incl, FG_WAVE - 1);
      int32_t* sc = s_sc[wid];
      int32_t* sb = s_sb[wid];
      double* sacc = s_acc[wid];
      sc[lane] = incl - ds;
      sb[lane] = b;
      sacc[lane] = 0.0;
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      for (int32_t t0 = 0; t0 < T; t0 += FG_WAVE) {
        const int32_t t = t0 + lane;
        double x = 0.0;
        int32_t key = -1 - lane;  // lanes past the end: runs of their own
        if (t < T) {
          const int32_t j = fgk::upper_idx(sc, FG_WAVE, t);
          // t - sc[j] < the length of row j: the entry lies inside its row
          x = cur[A.col[sb[j] + (t - sc[j])]];
          key = j;
        }
        const int32_t kp = __shfl_up(key, 1, FG_WAVE);
        const int32_t kn = __shfl_down(key, 1, FG_WAVE);
        const bool head = lane == 0 || kp != key;
        const bool tail = lane == FG_WAVE - 1 || kn != key;
        const uint64_t H = __ballot(head);
        const uint64_t upto = lane == FG_WAVE - 1 ? ~0ull : ((2ull << lane) - 1ull);
        const int start = 63 - __builtin_clzll(H & upto);
        x = seg_incl_sum(x, lane, start);
        if (tail && key >= 0) sacc[key] += x;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
      }
      if (v64 < A.n && deg < FG_WAVE) nc += pr_update(A, nxt, v, deg, sacc[lane]);
    }
    // medium rows: one at a time, the whole wave across the row
    uint64_t med = __ballot(deg >= FG_WAVE && deg < PR_LONG);
    while (med) {
      const int l = __builtin_ctzll(med);
      med &= med - 1;
      const int32_t ub = __shfl(b, l, FG_WAVE);
      const int32_t ud = __shfl(deg, l, FG_WAVE);
      double acc = 0.0;
      acc = strided_gather_sum(cur, A.col, ub + lane, ub + ud, FG_WAVE);
      acc = wave_sum_f64(acc);
      if (lane == l) nc += pr_update(A, nxt, v, ud, acc);
    }
  }
  nc = fg_wave_sum(nc);
  if (lane == 0 && nc) atomicAdd(&C->notconv[par], nc);

  // the last workgroup closes the iteration
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) s_last = atomicAdd(&C->blocks_done, 1u) == gridDim.x - 1;
  __syncthreads();
  if (!s_last || threadIdx.x != 0) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  const unsigned long long above =
      __hip_atomic_load(&C->notconv[par], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (A.stats) {
    fg_run_stats* st = A.stats;
    if (it < FG_TRACE_MAX) {
      st->dir[it] = 0;
      st->frontier[it] = (int64_t)above;
      st->inspected[it] = A.m;
      st->t_end[it] = (int64_t)wall_clock64();
    }
    st->iterations = it + 1;
    st->edges_inspected += A.m;
  }
  C->iterations = it + 1;
  if (A.tol > 0.0 && above == 0) C->done = 1;
  C->notconv[par ^ 1] = 0;
  C->next_item[par] = 0;
  C->blocks_done = 0;
}

struct PrLayout {
  double* contrib0;
  double* contrib1;
  int32_t* longrows;
  PrCtl* ctl;
  size_t bytes;
};

PrLayout pr_layout(const fg_graph* g, void* ws) {
  fg_carver c(ws);
  PrLayout L;
  L.contrib0 = c.take<double>(g->n);
  L.contrib1 = c.take<double>(g->n);
  L.longrows = c.take<int32_t>(g->n);
  L.ctl = c.take<PrCtl>(1);
  L.bytes = c.used;
  return L;
}

}  // namespace

size_t fg_pr_workspace_bytes(const fg_graph* g) { return pr_layout(g, nullptr).bytes; }

extern "C" fg_status fg_pagerank(const fg_graph* g, double damping, double tol, int32_t max_iter,
                                 void* ws, size_t ws_bytes, double* rank, fg_run_stats* stats,
                                 void* stream) {
  if (!g || !rank || !ws) return fg_set_error(FG_EINVAL, "fg_pagerank: NULL argument");
  if (!g->symmetric)
    return fg_set_error(FG_EUNSUPPORTED, "fg_pagerank: needs an undirected graph (FG_SYMMETRIC)");
  if (!(damping >= 0.0 && damping <= 1.0))
    return fg_set_error(FG_EINVAL, "fg_pagerank: damping %g outside [0, 1]", damping);
  if (!(tol >= 0.0)) return fg_set_error(FG_EINVAL, "fg_pagerank: tol %g < 0", tol);
  if (max_iter < 0 || max_iter > 100000)
    return fg_set_error(FG_EINVAL, "fg_pagerank: max_iter %d outside [0, 100000]", max_iter);
  PrLayout L = pr_layout(g, ws);
  FG_CHECK_WS_ALIGN(ws, "fg_pagerank");
  if (ws_bytes < L.bytes)
    return fg_set_error(FG_ENOMEM, "fg_pagerank: workspace of %zu bytes < required %zu",
                        ws_bytes, L.bytes);
  hipStream_t s = (hipStream_t)stream;
  PrArgs A;
  memset(&A, 0, sizeof(A));
  A.n = g->n;
  A.m = g->m;
  A.off = g->off;
  A.col = g->col;
  A.d = damping;
  A.base = (1.0 - damping) / (double)g->n;
  A.tol = tol;
  A.rank = rank;
  A.contrib[0] = L.contrib0;
  A.contrib[1] = L.contrib1;
  A.longrows = L.longrows;
  A.ctl = L.ctl;
  A.stats = stats;
  const fg_device_props pr = fg_props(g->device);
  A.clock_khz = pr.clock_khz;
  const int cus = pr.cus > 0 ? pr.cus : 256;
  pr_reset_kernel<<<1, 64, 0, s>>>(L.ctl);
  pr_setup_kernel<<<cus * 4, PR_BT, 0, s>>>(A, 1.0 / (double)g->n);
  for (int32_t it = 0; it < max_iter; ++it) pr_iter_kernel<<<cus * 4, PR_BT, 0, s>>>(A, it);
  FG_HIP_TRY(hipGetLastError());
  return FG_OK;
}
