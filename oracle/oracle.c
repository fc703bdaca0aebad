/*
 * Serial CPU oracle for the frontier traversal path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * source with the GPU path and must never be used as a fallback for it.
 *
 * Every function is the plain textbook definition of what the GPU path must
 * produce (breadth-first hop distance, shortest-path weight), or the step of
 * the paper it restates, written serially and without blocking or fusion:
 *
 *   O1 orc_csr_from_edges    undirected simple graph from an edge list
 *                            (Sec. VII-A preprocessing), via sorted pairs.
 *   O2 orc_bfs               FIFO-queue BFS: depth, a parent, level sizes.
 *   O3 orc_do_schedule       push/pull direction trace of direction-optimizing
 *                            BFS predicted from level sizes alone (Sec. VI-A).
 *   O4 orc_edges_inspected   edges a push or an early-exit pull iteration
 *                            reads (Sec. VI-A, vertex-parallel pull).
 *   O5 orc_dijkstra          binary-heap Dijkstra, canonical parents.
 *   O6 orc_floyd_warshall    all-pairs distances for tiny graphs.
 *   O7 orc_check_bfs/_sssp   O(m) invariant and tree checkers.
 *   O8 orc_package           split + package of an output frontier (Sec. III-B).
 *      orc_share_build       one partition's subgraph with duplicate-1-hop
 *                            proxies (Sec. III-C).
 *   O9 orc_bfs_partitioned   serial BSP emulation of multi-GPU BFS (Alg. 1):
 *                            per-partition advance+filter, selective
 *                            communication, combine.
 *  O11 orc_dobfs_dupall      serial BSP emulation of multi-GPU DOBFS (Alg. 2):
 *                            duplicate-all vertices, per-partition forward or
 *                            backward step, broadcast, combine.
 *  O12 orc_cc                connected components, each vertex labelled with
 *                            the smallest vertex id of its component.
 *  O13 orc_pagerank          PageRank power iteration in double precision
 *                            (Alg. 3 computation: rank update, then
 *                            accumulation over edges), threshold-ratio or
 *                            iteration-count convergence.
 *
 * Conventions: depth -1 and parent -1 for unreached vertices, parent[src] =
 * src, SSSP distance UINT32_MAX for unreached vertices.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define ORC_INF32 0xFFFFFFFFu

/* ------------------------------------------------------------------ O1 */

static int cmp_u64(const void* a, const void* b) {
  uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
  return (x > y) - (x < y);
}

/*
 * Sec. VII-A: graphs are made undirected, self-loops and duplicate edges are
 * removed.  Every edge {u,v}, u != v, becomes the pairs (u,v) and (v,u); the
 * pairs are sorted, duplicates dropped, and rows read off in order.  Returns
 * m (number of directed entries); `cols` needs room for 2*ne entries.
 */
int64_t orc_csr_from_edges(int32_t n, int64_t ne, const int32_t* eu,
                           const int32_t* ev, int32_t* off, int32_t* cols) {
  uint64_t* pairs = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(2 * ne + 1));
  int64_t np = 0;
  for (int64_t e = 0; e < ne; ++e) {
    uint64_t u = (uint32_t)eu[e], v = (uint32_t)ev[e];
    if (u == v) continue;
    pairs[np++] = (u << 32) | v;
    pairs[np++] = (v << 32) | u;
  }
  qsort(pairs, (size_t)np, sizeof(uint64_t), cmp_u64);
  int64_t m = 0;
  for (int32_t i = 0; i <= n; ++i) off[i] = 0;
  for (int64_t i = 0; i < np; ++i) {
    if (i > 0 && pairs[i] == pairs[i - 1]) continue;
    int32_t u = (int32_t)(pairs[i] >> 32);
    cols[m++] = (int32_t)(pairs[i] & 0xFFFFFFFFu);
    off[u + 1]++;
  }
  for (int32_t i = 0; i < n; ++i) off[i + 1] += off[i];
  free(pairs);
  return m;
}

/* ------------------------------------------------------------------ O2 */

/*
 * Breadth-first search with a FIFO queue, neighbours in CSR order.
 * depth[v] = hop distance from src (-1 if unreachable); parent[v] = the
 * vertex that first discovered v (parent[src] = src).  level_cnt[k] = number
 * of vertices at depth k (needs room for n entries); m_comp = sum of degrees
 * of reached vertices (directed CSR entries in the reached component).
 * Returns the number of levels (max depth + 1).
 */
int32_t orc_bfs(int32_t n, const int32_t* off, const int32_t* col, int32_t src,
                int32_t* depth, int32_t* parent, int64_t* level_cnt,
                int64_t* m_comp) {
  int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  for (int32_t v = 0; v < n; ++v) { depth[v] = -1; parent[v] = -1; }
  int64_t head = 0, tail = 0, mc = 0;
  int32_t levels = 0;
  depth[src] = 0;
  parent[src] = src;
  queue[tail++] = src;
  while (head < tail) {
    int32_t u = queue[head++];
    int32_t du = depth[u];
    if (du + 1 > levels) levels = du + 1;
    mc += off[u + 1] - off[u];
    for (int32_t e = off[u]; e < off[u + 1]; ++e) {
      int32_t v = col[e];
      if (depth[v] == -1) {
        depth[v] = du + 1;
        parent[v] = u;
        queue[tail++] = v;
      }
    }
  }
  if (level_cnt) {
    for (int32_t k = 0; k < levels; ++k) level_cnt[k] = 0;
    for (int32_t v = 0; v < n; ++v)
      if (depth[v] >= 0) level_cnt[depth[v]]++;
  }
  if (m_comp) *m_comp = mc;
  free(queue);
  return levels;
}

/* ------------------------------------------------------------------ O3 */

/*
 * Direction trace of direction-optimizing BFS (Sec. VI-A).  Iteration k
 * expands the level-k frontier Q.  P = vertices with a depth so far (levels
 * 0..k, Q included), U = n - |P|, |E_i| = m, |V_i| = n.  FV = |Q| m / n,
 * BV = |U| n / |P|.  Iteration 0 is forward.  Afterwards, a forward
 * iteration switches to backward when FV > do_a * BV (allowed once per
 * traversal); a backward iteration switches back when FV < do_b * BV.
 * With do = num/den both tests are exact in 128-bit integers:
 *   FV > do_a BV  <=>  a_den |Q| m |P| > a_num |U| n n.
 * dir[k] = 0 forward (push), 1 backward (pull).  Returns num_levels.
 */
int32_t orc_do_schedule(int32_t num_levels, const int64_t* level_cnt,
                        int64_t n, int64_t m, uint32_t a_num, uint32_t a_den,
                        uint32_t b_num, uint32_t b_den, int8_t* dir) {
  int switched = 0;
  int8_t cur = 0;
  int64_t p = 0;
  for (int32_t k = 0; k < num_levels; ++k) {
    int64_t q = level_cnt[k];
    p += q;
    int64_t u = n - p;
    if (k > 0) {
      unsigned __int128 lhs_common = (unsigned __int128)(uint64_t)q * (uint64_t)m;
      lhs_common *= (uint64_t)p;
      unsigned __int128 rhs_common = (unsigned __int128)(uint64_t)u * (uint64_t)n;
      rhs_common *= (uint64_t)n;
      if (cur == 0) {
        if (!switched && lhs_common * a_den > rhs_common * a_num) {
          cur = 1;
          switched = 1;
        }
      } else {
        if (lhs_common * b_den < rhs_common * b_num) cur = 0;
      }
    }
    dir[k] = cur;
  }
  return num_levels;
}

/* ------------------------------------------------------------------ O4 */

/*
 * Edges read in each iteration, given final depths and the direction trace.
 * Forward iteration k: every edge of every level-k vertex.
 * Backward iteration k (vertex-parallel advance with early exit, Sec. VI-A):
 * each vertex v with deg(v) > 0 not yet discovered (depth -1 or > k) scans
 * its row in CSR order; if depth[v] == k+1 it stops at the first neighbour
 * of depth k (position + 1 edges read), otherwise it reads the whole row.
 */
void orc_edges_inspected(int32_t n, const int32_t* off, const int32_t* col,
                         const int32_t* depth, int32_t num_levels,
                         const int8_t* dir, int64_t* out) {
  for (int32_t k = 0; k < num_levels; ++k) {
    int64_t cnt = 0;
    if (dir[k] == 0) {
      for (int32_t u = 0; u < n; ++u)
        if (depth[u] == k) cnt += off[u + 1] - off[u];
    } else {
      for (int32_t v = 0; v < n; ++v) {
        int32_t deg = off[v + 1] - off[v];
        if (deg == 0) continue;
        if (depth[v] != -1 && depth[v] <= k) continue;
        if (depth[v] == k + 1) {
          int32_t j = 0;
          while (depth[col[off[v] + j]] != k) ++j;
          cnt += j + 1;
        } else {
          cnt += deg;
        }
      }
    }
    out[k] = cnt;
  }
}

/* ------------------------------------------------------------------ O5 */

typedef struct { uint64_t d; int32_t v; } heap_item;

static void heap_push(heap_item* h, int64_t* sz, heap_item x) {
  int64_t i = (*sz)++;
  while (i > 0) {
    int64_t p = (i - 1) / 2;
    if (h[p].d <= x.d) break;
    h[i] = h[p];
    i = p;
  }
  h[i] = x;
}

static heap_item heap_pop(heap_item* h, int64_t* sz) {
  heap_item top = h[0];
  heap_item last = h[--(*sz)];
  int64_t i = 0;
  for (;;) {
    int64_t c = 2 * i + 1;
    if (c >= *sz) break;
    if (c + 1 < *sz && h[c + 1].d < h[c].d) c++;
    if (last.d <= h[c].d) break;
    h[i] = h[c];
    i = c;
  }
  if (*sz > 0) h[i] = last;
  return top;
}

/*
 * Single-source shortest paths (Dijkstra, binary heap with lazy deletion,
 * 64-bit accumulation).  dist[v] = minimum total weight (UINT32_MAX if
 * unreachable).  The canonical parent of a reached v != src is the smallest
 * u with an edge u->v and dist[u] + w(u,v) == dist[v]; parent[src] = src.
 * Returns 0, or -1 if a distance does not fit below UINT32_MAX.
 */
int32_t orc_dijkstra(int32_t n, const int32_t* off, const int32_t* col,
                     const uint32_t* w, int32_t src, uint32_t* dist,
                     int32_t* parent) {
  uint64_t* d = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
  uint8_t* done = (uint8_t*)calloc((size_t)n, 1);
  int64_t cap = (int64_t)off[n] + 2, sz = 0;
  heap_item* h = (heap_item*)malloc(sizeof(heap_item) * (size_t)cap);
  for (int32_t v = 0; v < n; ++v) d[v] = UINT64_MAX;
  d[src] = 0;
  heap_item s0 = {0, src};
  heap_push(h, &sz, s0);
  while (sz > 0) {
    heap_item it = heap_pop(h, &sz);
    int32_t u = it.v;
    if (done[u]) continue;
    done[u] = 1;
    for (int32_t e = off[u]; e < off[u + 1]; ++e) {
      int32_t v = col[e];
      uint64_t nd = d[u] + (uint64_t)w[e];
      if (nd < d[v]) {
        d[v] = nd;
        heap_item x = {nd, v};
        heap_push(h, &sz, x);
      }
    }
  }
  int32_t rc = 0;
  for (int32_t v = 0; v < n; ++v) {
    if (d[v] != UINT64_MAX && d[v] >= ORC_INF32) rc = -1;
    dist[v] = d[v] == UINT64_MAX ? ORC_INF32 : (uint32_t)d[v];
  }
  if (parent) {
    for (int32_t v = 0; v < n; ++v) parent[v] = -1;
    for (int32_t u = 0; u < n; ++u) {
      if (d[u] == UINT64_MAX) continue;
      for (int32_t e = off[u]; e < off[u + 1]; ++e) {
        int32_t v = col[e];
        if (v == src) continue;
        if (d[u] + (uint64_t)w[e] == d[v] && (parent[v] == -1 || u < parent[v]))
          parent[v] = u;
      }
    }
    parent[src] = src;
  }
  free(d);
  free(done);
  free(h);
  return rc;
}

/* ------------------------------------------------------------------ O6 */

/*
 * All-pairs shortest path weights, D[i*n + j] (UINT64_MAX = no path).
 * w == NULL means every edge weighs 1 (hop distance).  For tiny n only.
 */
void orc_floyd_warshall(int32_t n, const int32_t* off, const int32_t* col,
                        const uint32_t* w, uint64_t* D) {
  for (int64_t i = 0; i < (int64_t)n * n; ++i) D[i] = UINT64_MAX;
  for (int32_t i = 0; i < n; ++i) D[(int64_t)i * n + i] = 0;
  for (int32_t u = 0; u < n; ++u)
    for (int32_t e = off[u]; e < off[u + 1]; ++e) {
      uint64_t we = w ? w[e] : 1;
      int64_t idx = (int64_t)u * n + col[e];
      if (col[e] != u && we < D[idx]) D[idx] = we;
    }
  for (int32_t k = 0; k < n; ++k)
    for (int32_t i = 0; i < n; ++i) {
      uint64_t dik = D[(int64_t)i * n + k];
      if (dik == UINT64_MAX) continue;
      for (int32_t j = 0; j < n; ++j) {
        uint64_t dkj = D[(int64_t)k * n + j];
        if (dkj == UINT64_MAX) continue;
        if (dik + dkj < D[(int64_t)i * n + j]) D[(int64_t)i * n + j] = dik + dkj;
      }
    }
}

/* ------------------------------------------------------------------ O7 */

#define FAIL(...) do { if (msg) snprintf(msg, (size_t)msglen, __VA_ARGS__); return 1; } while (0)

/*
 * BFS result check in O(m) for a symmetric CSR: depth[src] == 0; on every
 * edge both ends are unreached or both reached with |d(u) - d(v)| <= 1;
 * every reached v != src has parent[v] adjacent to v with depth d(v) - 1;
 * parent[src] == src; unreached vertices have parent -1.  Together with the
 * edge condition this fixes every depth to the hop distance.
 */
int32_t orc_check_bfs(int32_t n, const int32_t* off, const int32_t* col,
                      int32_t src, const int32_t* depth, const int32_t* parent,
                      char* msg, int32_t msglen) {
  if (depth[src] != 0) FAIL("depth[src]=%d", depth[src]);
  for (int32_t u = 0; u < n; ++u) {
    if (depth[u] < -1) FAIL("depth[%d]=%d", u, depth[u]);
    if (u != src && depth[u] == 0) FAIL("second root %d", u);
    for (int32_t e = off[u]; e < off[u + 1]; ++e) {
      int32_t v = col[e];
      int32_t a = depth[u], b = depth[v];
      if ((a < 0) != (b < 0)) FAIL("edge %d-%d crosses reach (%d,%d)", u, v, a, b);
      if (a >= 0 && (a - b > 1 || b - a > 1)) FAIL("edge %d-%d depths %d,%d", u, v, a, b);
    }
  }
  if (!parent) return 0;
  if (parent[src] != src) FAIL("parent[src]=%d", parent[src]);
  for (int32_t v = 0; v < n; ++v) {
    if (v == src) continue;
    int32_t p = parent[v];
    if (depth[v] < 0) {
      if (p != -1) FAIL("unreached %d has parent %d", v, p);
      continue;
    }
    if (p < 0 || p >= n) FAIL("parent[%d]=%d out of range", v, p);
    if (depth[p] != depth[v] - 1) FAIL("parent[%d]=%d depth %d vs %d", v, p, depth[p], depth[v]);
    int found = 0;
    for (int32_t e = off[v]; e < off[v + 1] && !found; ++e) found = col[e] == p;
    if (!found) FAIL("parent[%d]=%d not adjacent", v, p);
  }
  return 0;
}

/*
 * SSSP result check in O(m) for a CSR whose reverse edges carry the same
 * weights: dist[src] == 0; dist[v] <= dist[u] + w on every edge; every
 * reached v != src has a tight in-edge; if parent is given it must equal the
 * smallest tight predecessor.  Together these fix dist to the shortest-path
 * weights (positive weights) and parent to the canonical one.
 */
int32_t orc_check_sssp(int32_t n, const int32_t* off, const int32_t* col,
                       const uint32_t* w, int32_t src, const uint32_t* dist,
                       const int32_t* parent, char* msg, int32_t msglen) {
  if (dist[src] != 0) FAIL("dist[src]=%u", dist[src]);
  int32_t* tight = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  for (int32_t v = 0; v < n; ++v) tight[v] = -1;
  for (int32_t u = 0; u < n; ++u) {
    if (dist[u] == ORC_INF32) continue;
    for (int32_t e = off[u]; e < off[u + 1]; ++e) {
      int32_t v = col[e];
      uint64_t nd = (uint64_t)dist[u] + w[e];
      if ((uint64_t)dist[v] > nd) { free(tight); FAIL("edge %d->%d not relaxed", u, v); }
      if ((uint64_t)dist[v] == nd && (tight[v] == -1 || u < tight[v])) tight[v] = u;
    }
  }
  for (int32_t v = 0; v < n; ++v) {
    if (v == src || dist[v] == ORC_INF32) continue;
    if (tight[v] == -1) { free(tight); FAIL("no tight edge into %d", v); }
  }
  if (parent) {
    for (int32_t v = 0; v < n; ++v) {
      int32_t want = v == src ? src : (dist[v] == ORC_INF32 ? -1 : tight[v]);
      if (parent[v] != want) { free(tight); FAIL("parent[%d]=%d want %d", v, parent[v], want); }
    }
  }
  free(tight);
  return 0;
}

/* ------------------------------------------------------------------ O8 */

/*
 * One partition's subgraph under duplicate-1-hop (Sec. III-C) with the
 * random owner map.  Local ids: the hosted vertices (owner == part) in
 * ascending global order, then the proxies (remote neighbours of hosted
 * vertices) in ascending global order.  A hosted vertex keeps its global
 * row, each neighbour renamed to its local id, in the same order; proxies
 * have no out-edges.  lowner = owner of each local vertex; lconv = the id a
 * local vertex has on its owner (its rank among that owner's hosted
 * vertices); l2g = global id.  Returns the local edge count.
 */
int64_t orc_share_build(int32_t n, const int32_t* off, const int32_t* col,
                        const uint8_t* owner, int32_t part, int32_t* n_local,
                        int32_t* n_total, int32_t* loff, int32_t* lcol,
                        uint8_t* lowner, int32_t* lconv, int32_t* l2g) {
  int32_t* g2l = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* rank = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t counts[256] = {0};
  for (int32_t v = 0; v < n; ++v) rank[v] = counts[owner[v]]++;
  int32_t nl = 0;
  for (int32_t v = 0; v < n; ++v) {
    g2l[v] = -1;
    if (owner[v] == part) g2l[v] = nl++;
  }
  uint8_t* is_proxy = (uint8_t*)calloc((size_t)n, 1);
  for (int32_t v = 0; v < n; ++v) {
    if (owner[v] != part) continue;
    for (int32_t e = off[v]; e < off[v + 1]; ++e)
      if (owner[col[e]] != part) is_proxy[col[e]] = 1;
  }
  int32_t nt = nl;
  for (int32_t v = 0; v < n; ++v)
    if (is_proxy[v]) g2l[v] = nt++;
  for (int32_t v = 0; v < n; ++v) {
    if (g2l[v] < 0) continue;
    l2g[g2l[v]] = v;
    lowner[g2l[v]] = owner[v];
    lconv[g2l[v]] = rank[v];
  }
  int64_t k = 0;
  for (int32_t i = 0; i < nt; ++i) {
    loff[i] = (int32_t)k;
    if (i < nl) {
      int32_t v = l2g[i];
      for (int32_t e = off[v]; e < off[v + 1]; ++e) lcol[k++] = g2l[col[e]];
    }
  }
  loff[nt] = (int32_t)k;
  *n_local = nl;
  *n_total = nt;
  free(g2l);
  free(rank);
  free(is_proxy);
  return k;
}

/*
 * Split + package (Sec. III-B): walk the output frontier in order; a vertex
 * v >= n_local is a proxy of a remote vertex and is appended, with its
 * associated data, to the buffer of its owner: id on the owner (conv[v]),
 * depth[v], and (if parent != NULL) the parent's global id l2g[parent[v]].
 * Buffer p occupies [p*cap, p*cap + counts[p]) of each output array.
 * Local vertices (v < n_local) are appended to local_out in order.
 */
void orc_package(int32_t len, const int32_t* frontier, int32_t n_local,
                 const uint8_t* owner, const int32_t* conv, const int32_t* depth,
                 const int32_t* parent, const int32_t* l2g, int32_t nparts,
                 int32_t cap, int32_t* ids_out, int32_t* depth_out,
                 int32_t* parent_out, int32_t* counts, int32_t* local_out,
                 int32_t* local_count) {
  for (int32_t p = 0; p < nparts; ++p) counts[p] = 0;
  int32_t nlocal = 0;
  for (int32_t i = 0; i < len; ++i) {
    int32_t v = frontier[i];
    if (v < n_local) {
      if (local_out) local_out[nlocal] = v;
      nlocal++;
      continue;
    }
    int32_t p = owner[v];
    int64_t slot = (int64_t)p * cap + counts[p];
    ids_out[slot] = conv[v];
    depth_out[slot] = depth[v];
    if (parent && parent_out) parent_out[slot] = l2g[parent[v]];
    counts[p]++;
  }
  if (local_count) *local_count = nlocal;
}

/* ------------------------------------------------------------------ O9 */

typedef struct {
  int32_t nl, nt;
  int32_t *off, *col, *conv, *l2g, *label;
  uint8_t* own;
} orc_part;

/*
 * Multi-GPU BFS (Alg. 1) emulated serially on `nparts` partitions built
 * with orc_share_build.  Per iteration every partition advances its local
 * frontier and filters newly reached vertices (label -1 -> iter+1).  The
 * output frontier is split: hosted vertices feed the partition's next
 * frontier; proxies are packaged (O8) and sent to their owners.  Combine: a
 * received vertex that has no label yet takes the received label and joins
 * the receiver's next frontier.  Stops when every frontier is empty.
 * Writes global depths (label of each vertex on its owner).
 */
int32_t orc_bfs_partitioned(int32_t n, const int32_t* off, const int32_t* col,
                            const uint8_t* owner, int32_t nparts, int32_t src,
                            int32_t* depth_out) {
  int64_t m = off[n];
  orc_part* P = (orc_part*)calloc((size_t)nparts, sizeof(orc_part));
  int32_t** fr = (int32_t**)calloc((size_t)nparts, sizeof(int32_t*));
  int32_t** nx = (int32_t**)calloc((size_t)nparts, sizeof(int32_t*));
  int32_t* frl = (int32_t*)calloc((size_t)nparts, sizeof(int32_t));
  int32_t* nxl = (int32_t*)calloc((size_t)nparts, sizeof(int32_t));
  for (int32_t p = 0; p < nparts; ++p) {
    P[p].off = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
    P[p].col = (int32_t*)malloc(sizeof(int32_t) * ((size_t)m + 1));
    P[p].own = (uint8_t*)malloc((size_t)n + 1);
    P[p].conv = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
    P[p].l2g = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
    orc_share_build(n, off, col, owner, p, &P[p].nl, &P[p].nt, P[p].off,
                    P[p].col, P[p].own, P[p].conv, P[p].l2g);
    P[p].label = (int32_t*)malloc(sizeof(int32_t) * ((size_t)P[p].nt + 1));
    for (int32_t i = 0; i < P[p].nt; ++i) P[p].label[i] = -1;
    fr[p] = (int32_t*)malloc(sizeof(int32_t) * ((size_t)P[p].nt + 1));
    nx[p] = (int32_t*)malloc(sizeof(int32_t) * ((size_t)P[p].nt + 1));
  }
  /* source: host partition and its id there */
  int32_t sp = owner[src];
  int32_t tsrc = 0;
  for (int32_t v = 0; v < src; ++v) tsrc += owner[v] == sp;
  P[sp].label[tsrc] = 0;
  fr[sp][0] = tsrc;
  frl[sp] = 1;
  /* per-partition receive queues: (local id on receiver, label) */
  int32_t** rid = (int32_t**)calloc((size_t)nparts, sizeof(int32_t*));
  int32_t** rlab = (int32_t**)calloc((size_t)nparts, sizeof(int32_t*));
  int32_t* rcnt = (int32_t*)calloc((size_t)nparts, sizeof(int32_t));
  for (int32_t p = 0; p < nparts; ++p) {
    int64_t cap = 0;
    for (int32_t q = 0; q < nparts; ++q) cap += P[q].nt;
    rid[p] = (int32_t*)malloc(sizeof(int32_t) * ((size_t)cap + 1));
    rlab[p] = (int32_t*)malloc(sizeof(int32_t) * ((size_t)cap + 1));
  }
  int32_t iter = 0;
  for (;;) {
    int64_t total = 0;
    for (int32_t p = 0; p < nparts; ++p) total += frl[p];
    if (total == 0) break;
    for (int32_t p = 0; p < nparts; ++p) rcnt[p] = 0;
    for (int32_t p = 0; p < nparts; ++p) {
      orc_part* S = &P[p];
      nxl[p] = 0;
      /* advance + filter on the local frontier */
      for (int32_t i = 0; i < frl[p]; ++i) {
        int32_t u = fr[p][i];
        for (int32_t e = S->off[u]; e < S->off[u + 1]; ++e) {
          int32_t v = S->col[e];
          if (S->label[v] != -1) continue;
          S->label[v] = iter + 1;
          /* split: hosted -> next local frontier; proxy -> package to owner */
          if (v < S->nl) {
            nx[p][nxl[p]++] = v;
          } else {
            int32_t q = S->own[v];
            rid[q][rcnt[q]] = S->conv[v];
            rlab[q][rcnt[q]] = iter + 1;
            rcnt[q]++;
          }
        }
      }
    }
    /* combine received data: keep the smaller label, enqueue if improved */
    for (int32_t q = 0; q < nparts; ++q) {
      orc_part* S = &P[q];
      for (int32_t i = 0; i < rcnt[q]; ++i) {
        int32_t v = rid[q][i];
        if (S->label[v] == -1 || rlab[q][i] < S->label[v]) {
          S->label[v] = rlab[q][i];
          nx[q][nxl[q]++] = v;
        }
      }
    }
    for (int32_t p = 0; p < nparts; ++p) {
      int32_t* t = fr[p]; fr[p] = nx[p]; nx[p] = t;
      frl[p] = nxl[p];
    }
    iter++;
  }
  for (int32_t v = 0; v < n; ++v) depth_out[v] = -1;
  for (int32_t p = 0; p < nparts; ++p)
    for (int32_t i = 0; i < P[p].nl; ++i) depth_out[P[p].l2g[i]] = P[p].label[i];
  for (int32_t p = 0; p < nparts; ++p) {
    free(P[p].off); free(P[p].col); free(P[p].own); free(P[p].conv);
    free(P[p].l2g); free(P[p].label); free(fr[p]); free(nx[p]);
    free(rid[p]); free(rlab[p]);
  }
  free(P); free(fr); free(nx); free(frl); free(nxl); free(rid); free(rlab); free(rcnt);
  return iter;
}

/* ----------------------------------------------------------------- O11 */

/*
 * Multi-GPU direction-optimizing BFS (Alg. 2) with duplicate-all vertices
 * and broadcast communication (Sec. III-C), emulated serially.  Partition p
 * holds every vertex (ids unchanged) but only the rows of the vertices it
 * hosts (owner[v] == p); the other rows are empty on p.  Each partition
 * keeps its own labels.  Iteration k starts from the frontier of level k,
 * which is the same on every partition:
 *   direction   the rule of Sec. VI-A, FV = |Q| |E| / |V| against
 *               BV = |U| |V| / |P|, from the global counts (|E| the sum of
 *               the partitions' |E_i|, |V_i| = |V| under duplicate-all), so
 *               that every partition takes the same direction; forward
 *               first, forward->backward at most once, strict comparisons,
 *               do = num / den compared exactly in integers;
 *   computation forward: each frontier vertex's local row is scanned and
 *               every neighbour without a label takes k + 1 and joins the
 *               partition's newly-discovered list N_p; backward: each hosted
 *               vertex without a label scans its row in order and stops at
 *               the first neighbour labelled k, taking k + 1 and joining N_p;
 *   broadcast   every N_p is sent to every other partition;
 *   combine     a received vertex without a label takes k + 1;
 *   convergence the union of the N_p (the next frontier) is empty.
 * depth_out receives partition 0's labels and dir (room for n entries) the
 * direction of each iteration (0 forward, 1 backward).  Returns the number
 * of iterations, or -1 if the partitions' labels disagree at the end.
 */
int32_t orc_dobfs_dupall(int32_t n, const int32_t* off, const int32_t* col,
                         const uint8_t* owner, int32_t nparts, int32_t src,
                         uint32_t a_num, uint32_t a_den, uint32_t b_num, uint32_t b_den,
                         int32_t* depth_out, int8_t* dir) {
  const int64_t m = off[n];
  int32_t** label = (int32_t**)calloc((size_t)nparts, sizeof(int32_t*));
  int32_t** nl = (int32_t**)calloc((size_t)nparts, sizeof(int32_t*));
  int32_t* nlen = (int32_t*)calloc((size_t)nparts, sizeof(int32_t));
  for (int32_t p = 0; p < nparts; ++p) {
    label[p] = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
    nl[p] = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
    for (int32_t v = 0; v < n; ++v) label[p][v] = -1;
    label[p][src] = 0;
  }
  /* the frontier of the current level (identical on every partition) */
  int32_t* q = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
  int32_t* qn = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
  int32_t qlen = 1;
  q[0] = src;
  int64_t pcount = 1;  /* |P|: vertices with a label, frontier included */
  int cur = 0, switched = 0;
  int32_t k = 0;
  while (qlen > 0) {
    if (k > 0) {
      unsigned __int128 lhs = (unsigned __int128)(uint64_t)qlen * (uint64_t)m;
      lhs *= (uint64_t)pcount;
      unsigned __int128 rhs = (unsigned __int128)(uint64_t)(n - pcount) * (uint64_t)n;
      rhs *= (uint64_t)n;
      if (cur == 0) {
        if (!switched && lhs * a_den > rhs * a_num) {
          cur = 1;
          switched = 1;
        }
      } else if (lhs * b_den < rhs * b_num) {
        cur = 0;
      }
    }
    dir[k] = (int8_t)cur;
    /* computation on every partition, local rows only */
    for (int32_t p = 0; p < nparts; ++p) {
      int32_t* L = label[p];
      nlen[p] = 0;
      if (cur == 0) {
        for (int32_t i = 0; i < qlen; ++i) {
          int32_t u = q[i];
          if (owner[u] != p) continue; /* remote rows are empty on p */
          for (int32_t e = off[u]; e < off[u + 1]; ++e) {
            int32_t v = col[e];
            if (L[v] == -1) {
              L[v] = k + 1;
              nl[p][nlen[p]++] = v;
            }
          }
        }
      } else {
        for (int32_t v = 0; v < n; ++v) {
          if (owner[v] != p || L[v] != -1) continue;
          for (int32_t e = off[v]; e < off[v + 1]; ++e) {
            if (L[col[e]] == k) {
              L[v] = k + 1;
              nl[p][nlen[p]++] = v;
              break;
            }
          }
        }
      }
    }
    /* broadcast + combine: every partition takes every other's list */
    for (int32_t p = 0; p < nparts; ++p)
      for (int32_t r = 0; r < nparts; ++r) {
        if (r == p) continue;
        for (int32_t i = 0; i < nlen[r]; ++i) {
          int32_t v = nl[r][i];
          if (label[p][v] == -1) label[p][v] = k + 1;
        }
      }
    /* next frontier: the vertices labelled k + 1 (partition 0's view) */
    int32_t nq = 0;
    for (int32_t v = 0; v < n; ++v)
      if (label[0][v] == k + 1) qn[nq++] = v;
    int32_t* t = q; q = qn; qn = t;
    qlen = nq;
    pcount += nq;
    k++;
  }
  int32_t agree = 1;
  for (int32_t p = 1; p < nparts; ++p)
    for (int32_t v = 0; v < n; ++v)
      if (label[p][v] != label[0][v]) agree = 0;
  for (int32_t v = 0; v < n; ++v) depth_out[v] = label[0][v];
  for (int32_t p = 0; p < nparts; ++p) { free(label[p]); free(nl[p]); }
  free(label); free(nl); free(nlen); free(q); free(qn);
  return agree ? k : -1;
}

/* ----------------------------------------------------------------- O12 */

/*
 * Connected components (Table I's CC primitive): label[v] = the smallest
 * vertex id in v's component.  Vertices are taken in ascending order; an
 * unlabelled vertex is the smallest of a new component and labels every
 * vertex it reaches (FIFO queue).  Returns the number of components.
 */
int32_t orc_cc(int32_t n, const int32_t* off, const int32_t* col, int32_t* label) {
  int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  for (int32_t v = 0; v < n; ++v) label[v] = -1;
  int32_t comps = 0;
  for (int32_t s = 0; s < n; ++s) {
    if (label[s] != -1) continue;
    comps++;
    int64_t head = 0, tail = 0;
    label[s] = s;
    queue[tail++] = s;
    while (head < tail) {
      int32_t u = queue[head++];
      for (int32_t e = off[u]; e < off[u + 1]; ++e) {
        int32_t v = col[e];
        if (label[v] == -1) {
          label[v] = s;
          queue[tail++] = v;
        }
      }
    }
  }
  free(queue);
  return comps;
}

/* ----------------------------------------------------------------- O13 */

/*
 * PageRank (Alg. 3's computation, on an undirected CSR where each edge
 * carries rank both ways), in double precision.  rank_0(v) = 1 / n.  Each
 * iteration first accumulates over the edges, acc(v) = sum over neighbours
 * u of rank(u) / deg(u) (the advance step), then updates every vertex,
 * rank'(v) = (1 - d) / n + d acc(v) (the filter step); rank that reaches a
 * vertex of degree 0 is not passed on.  Convergence: stop after an
 * iteration in which every update satisfies |rank' - rank| <= tol * rank
 * (the threshold ratio; tol = 0 never stops early), or after max_iter
 * iterations.  Returns the number of iterations run.
 */
int32_t orc_pagerank(int32_t n, const int32_t* off, const int32_t* col, double d, double tol,
                     int32_t max_iter, double* rank) {
  double* acc = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  for (int32_t v = 0; v < n; ++v) rank[v] = 1.0 / (double)n;
  int32_t it = 0;
  while (it < max_iter) {
    for (int32_t v = 0; v < n; ++v) acc[v] = 0.0;
    for (int32_t u = 0; u < n; ++u) {
      int32_t deg = off[u + 1] - off[u];
      if (deg == 0) continue;
      double share = rank[u] / (double)deg;
      for (int32_t e = off[u]; e < off[u + 1]; ++e) acc[col[e]] += share;
    }
    int converged = 1;
    for (int32_t v = 0; v < n; ++v) {
      double nr = (1.0 - d) / (double)n + d * acc[v];
      double diff = nr > rank[v] ? nr - rank[v] : rank[v] - nr;
      if (diff > tol * rank[v]) converged = 0;
      rank[v] = nr;
    }
    it++;
    if (converged && tol > 0) break;
  }
  free(acc);
  return it;
}
