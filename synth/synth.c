/*
 * Seeded synthetic inputs shared by the oracle and the GPU path.
 *
 * This file holds no traversal arithmetic.  It only turns seeds into graphs
 * and into the random choices the experiments make (sources, partition
 * owners, edge weights):
 *
 *  - R-MAT edge lists with the quadrant probabilities of the paper's rmat
 *    group (Sec. VII-A: {A,B,C,D} = {0.57,0.19,0.19,0.05});
 *  - the paper's preprocessing into an undirected CSR (Sec. VII-A: converted
 *    to undirected, self-loops and duplicate edges removed), rows ascending;
 *  - 4-neighbour 2D grids (row-major ids, ascending neighbour order);
 *  - symmetric integer edge weights in [1, 64] (Sec. VII-A gives [0, 64];
 *    the workloads here use [1, 64]);
 *  - distinct random sources of nonzero degree;
 *  - random vertex-to-partition owners (the random partitioner, Sec. V-C).
 *
 * Random numbers come from one counter-based generator: the i-th output of
 * SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) seeded with `seed`,
 * i.e. mix64(seed + (i + 1) * 0x9E3779B97F4A7C15) with the Stafford Mix13
 * finaliser.  Any output can be computed independently of the others.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define SYN_GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t syn_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* i-th output of SplitMix64 seeded with `seed` (0-based). */
uint64_t syn_ctr_u64(uint64_t seed, uint64_t i) {
  return syn_mix64(seed + (i + 1ULL) * SYN_GAMMA);
}

/*
 * R-MAT edge list: edge e picks one quadrant per recursion level, most
 * significant bit first.  At level l the draw r = ctr(seed, e*64 + l) selects
 * (row bit, col bit) = (0,0) if r < t1, (0,1) if r < t2, (1,0) if r < t3,
 * else (1,1).  t1..t3 are the cumulative probabilities scaled by 2^64.
 * No noise and no label permutation, so vertex 0 is the heaviest vertex.
 */
void syn_rmat_edges(int32_t scale, int64_t num_edges, uint64_t seed,
                    uint64_t t1, uint64_t t2, uint64_t t3,
                    int32_t* eu, int32_t* ev) {
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < num_edges; ++e) {
    uint32_t u = 0, v = 0;
    for (int32_t l = 0; l < scale; ++l) {
      uint64_t r = syn_ctr_u64(seed, (uint64_t)e * 64ULL + (uint64_t)l);
      uint32_t rb, cb;
      if (r < t1) { rb = 0; cb = 0; }
      else if (r < t2) { rb = 0; cb = 1; }
      else if (r < t3) { rb = 1; cb = 0; }
      else { rb = 1; cb = 1; }
      u = (u << 1) | rb;
      v = (v << 1) | cb;
    }
    eu[e] = (int32_t)u;
    ev[e] = (int32_t)v;
  }
}

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

/*
 * Undirected simple CSR from an edge list: each edge {u,v} with u != v is
 * stored as u->v and v->u, each row sorted ascending and deduplicated.
 * Pass 1 (cols == NULL): fills row_offsets with an upper bound layout and
 * returns the number of directed slots needed (2 * non-loop edges).
 * Pass 2 (cols != NULL, capacity >= that number): scatters, sorts, dedups,
 * compacts in place and rewrites row_offsets; returns the final m.
 * `tmp_off` must hold n+1 int64 values.
 */
int64_t syn_csr_build(int32_t n, int64_t num_edges, const int32_t* eu,
                      const int32_t* ev, int64_t* tmp_off, int32_t* row_offsets,
                      int32_t* cols) {
  memset(tmp_off, 0, sizeof(int64_t) * ((size_t)n + 1));
  /* degree count (both directions) */
  for (int64_t e = 0; e < num_edges; ++e) {
    int32_t u = eu[e], v = ev[e];
    if (u == v) continue;
    tmp_off[u + 1]++;
    tmp_off[v + 1]++;
  }
  for (int32_t i = 0; i < n; ++i) tmp_off[i + 1] += tmp_off[i];
  int64_t slots = tmp_off[n];
  if (cols == NULL) return slots;
  int64_t* cursor = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  memcpy(cursor, tmp_off, sizeof(int64_t) * (size_t)n);
  for (int64_t e = 0; e < num_edges; ++e) {
    int32_t u = eu[e], v = ev[e];
    if (u == v) continue;
    cols[cursor[u]++] = v;
    cols[cursor[v]++] = u;
  }
  free(cursor);
  /* per-row sort + unique, keep unique count of each row in cursor-free way */
  int32_t* ucount = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
#pragma omp parallel for schedule(dynamic, 4096)
  for (int32_t i = 0; i < n; ++i) {
    int64_t b = tmp_off[i], e = tmp_off[i + 1];
    int32_t* row = cols + b;
    int64_t len = e - b;
    if (len > 1) qsort(row, (size_t)len, sizeof(int32_t), cmp_i32);
    int64_t k = 0;
    for (int64_t j = 0; j < len; ++j)
      if (k == 0 || row[j] != row[k - 1]) row[k++] = row[j];
    ucount[i] = (int32_t)k;
  }
  /* compact (sequential, forward: destination never passes the source) */
  int64_t w = 0;
  for (int32_t i = 0; i < n; ++i) {
    int64_t b = tmp_off[i];
    row_offsets[i] = (int32_t)w;
    if (w != b) memmove(cols + w, cols + b, sizeof(int32_t) * (size_t)ucount[i]);
    w += ucount[i];
  }
  row_offsets[n] = (int32_t)w;
  free(ucount);
  return w;
}

/* rows x cols 4-neighbour grid, id = r*cols + c, neighbours ascending. */
int64_t syn_grid_csr(int32_t rows, int32_t ncols, int32_t* row_offsets,
                     int32_t* col) {
  int64_t n = (int64_t)rows * ncols;
  /* offsets: closed form per vertex degree */
#pragma omp parallel for schedule(static)
  for (int32_t r = 0; r < rows; ++r) {
    /* number of directed entries before row r */
    int64_t before = 0;
    if (r > 0) {
      /* each full row contributes: horizontal 2*(ncols-1), vertical: up
         links for rows>0 and down links for rows<rows-1 */
      int64_t horiz = 2LL * (ncols - 1) * r;
      int64_t up = (int64_t)ncols * (r - 1);      /* rows 1..r-1 have up */
      int64_t down = (int64_t)ncols * r;          /* rows 0..r-1 have down (r <= rows-1) */
      before = horiz + up + down;
    }
    int64_t k = before;
    for (int32_t c = 0; c < ncols; ++c) {
      int64_t id = (int64_t)r * ncols + c;
      row_offsets[id] = (int32_t)k;
      if (r > 0) col[k++] = (int32_t)(id - ncols);
      if (c > 0) col[k++] = (int32_t)(id - 1);
      if (c < ncols - 1) col[k++] = (int32_t)(id + 1);
      if (r < rows - 1) col[k++] = (int32_t)(id + ncols);
    }
  }
  int64_t m = 2LL * ((int64_t)rows * (ncols - 1) + (int64_t)(rows - 1) * ncols);
  row_offsets[n] = (int32_t)m;
  return m;
}

/* w(u,v) = w(v,u) = 1 + (ctr(seed, min*n + max) mod 64), aligned with cols. */
void syn_weights(int32_t n, const int32_t* row_offsets, const int32_t* cols,
                 uint64_t seed, uint32_t* w) {
#pragma omp parallel for schedule(dynamic, 4096)
  for (int32_t u = 0; u < n; ++u) {
    for (int32_t e = row_offsets[u]; e < row_offsets[u + 1]; ++e) {
      int32_t v = cols[e];
      uint64_t lo = (uint64_t)(u < v ? u : v), hi = (uint64_t)(u < v ? v : u);
      w[e] = 1u + (uint32_t)(syn_ctr_u64(seed, lo * (uint64_t)n + hi) & 63ULL);
    }
  }
}

/* k distinct sources with degree > 0: candidate i is ctr(seed, i) mod n. */
int32_t syn_sources(int32_t n, const int32_t* row_offsets, uint64_t seed,
                    int32_t k, int32_t* out) {
  int32_t got = 0;
  uint8_t* taken = (uint8_t*)calloc((size_t)n, 1);
  for (uint64_t i = 0; got < k && i < 64ULL * (uint64_t)n + 1024; ++i) {
    int32_t v = (int32_t)(syn_ctr_u64(seed, i) % (uint64_t)n);
    if (taken[v] || row_offsets[v + 1] == row_offsets[v]) continue;
    taken[v] = 1;
    out[got++] = v;
  }
  free(taken);
  return got;
}

/* owner(v) = ctr(seed, v) mod parts: i.i.d. random partitioner. */
void syn_owner(int32_t n, uint64_t seed, int32_t parts, uint8_t* owner) {
#pragma omp parallel for schedule(static)
  for (int32_t v = 0; v < n; ++v)
    owner[v] = (uint8_t)(syn_ctr_u64(seed, (uint64_t)v) % (uint64_t)parts);
}
