/*
 * fg.h -- C ABI of the frontier graph library (libfg.so) for MI355X (gfx950).
 *
 * The library implements the single-GPU data-parallel path of frontier-
 * centric graph traversal from "Multi-GPU Graph Analytics" (Pan, Wang, Wu,
 * Yang, Owens): the advance and filter operators (Sec. II-B), breadth-first
 * search built from them (Alg. 1), direction-optimizing BFS with the
 * vertex-parallel early-exit pull step and the inexpensive direction rule
 * (Sec. VI-A, Alg. 2), advance+filter kernel fusion (Sec. VI-C), integer
 * single-source shortest paths (Table I), the per-iteration split/package
 * step of the multi-GPU framework (Sec. III-B), and a 64-lane batched BFS.
 *
 * The calls follow the problem statement of the paper's framework: load a
 * CSR graph, set the source, run the primitive, read depths / distances /
 * predecessors.
 *
 * Conventions shared by every call
 *  - All functions return fg_status: FG_OK (0) or a negative error code.
 *    They never throw.  fg_last_error() returns a thread-local message that
 *    describes the last error of the calling thread.
 *  - Argument errors are detected synchronously, before any work is
 *    enqueued; on error no output is written.
 *  - Work is enqueued asynchronously on `stream` (a hipStream_t, NULL = the
 *    null stream).  Outputs are valid after the stream has been synchronised.
 *    Device-side failures (e.g. FG_EOVERFLOW) are reported in the `status`
 *    field of the device-resident fg_run_stats of that call.
 *  - Pointers documented as "device" must be device memory of the current
 *    HIP device (e.g. torch tensor data_ptr()).  Caller owns every buffer it
 *    passes; the library never frees caller memory.
 *  - Vertex ids are int32 in [0, n); edge offsets are int32 (m < 2^31).
 *  - A workspace may not be used by two calls that overlap in time.
 */
#ifndef FG_H
#define FG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fg_status;

#define FG_OK 0
#define FG_EINVAL (-1)       /* bad argument or malformed CSR               */
#define FG_ENOMEM (-2)       /* workspace too small / allocation failed      */
#define FG_EDEVICE (-3)      /* HIP runtime error or device-side time-out    */
#define FG_EOVERFLOW (-4)    /* an output buffer's capacity was exceeded     */
#define FG_EUNSUPPORTED (-5) /* valid request the graph cannot serve         */

/* Thread-local description of the last error (never NULL). */
const char* fg_last_error(void);

/* Library version, "major.minor.patch". */
const char* fg_version(void);

/* ------------------------------------------------------------------ graph */

typedef struct fg_graph fg_graph;

#define FG_DEVICE_PTRS 1u /* the CSR arrays are device pointers              */
#define FG_BORROW 2u      /* with FG_DEVICE_PTRS: use the arrays in place;
                             the caller keeps them alive until destroy        */
#define FG_VALIDATE 4u    /* check row_offsets[0]==0, monotone offsets,
                             row_offsets[n]==m, 0<=col<n                       */
#define FG_SYMMETRIC 8u   /* the CSR is undirected (every u->v has v->u with
                             the same weight).  Required for the pull step.
                             With FG_VALIDATE the claim is checked as well,
                             which additionally requires strictly ascending
                             rows.                                           */

/*
 * Load a CSR graph (Sec. III-B: the framework's graph initialisation; the
 * paper's inputs are undirected, without self-loops or duplicate edges,
 * Sec. VII-A).  row_offsets: int32[n+1]; col_idx: int32[m]; weights:
 * uint32[m] aligned with col_idx, or NULL (required only by fg_sssp).
 * Without FG_DEVICE_PTRS the arrays are host memory and are copied.
 * Errors: FG_EINVAL (n < 1, m < 0, m >= 2^31, NULL arrays, failed
 * validation), FG_ENOMEM, FG_EDEVICE.  On success *out owns a graph that
 * is immutable and may be used from any stream of the same device.
 */
fg_status fg_graph_create_csr(int32_t n, int64_t m, const int32_t* row_offsets,
                              const int32_t* col_idx, const uint32_t* weights,
                              uint32_t flags, void* stream, fg_graph** out);

/* Release a graph (waits for the device).  NULL is accepted. */
fg_status fg_graph_destroy(fg_graph* g);

typedef struct {
  int32_t n;
  int32_t has_weights;
  int64_t m;
  int32_t symmetric;
  int32_t max_degree;
  int32_t nonzero_degree; /* vertices with at least one edge              */
  int32_t device;
  int64_t resident_bytes; /* device bytes held by the graph object          */
} fg_graph_info_t;

fg_status fg_graph_info(const fg_graph* g, fg_graph_info_t* info);

/* Device pointers of the graph's CSR arrays (read-only, owned by the graph
 * unless it was created with FG_BORROW); weights is NULL if none.  Any
 * output pointer may be NULL. */
fg_status fg_graph_csr(const fg_graph* g, const int32_t** row_offsets, const int32_t** col_idx,
                       const uint32_t** weights);

/* -------------------------------------------------------------- workspace */

#define FG_PRIM_BFS 0          /* fg_bfs, modes FG_MODE_DO / FG_MODE_PUSH      */
#define FG_PRIM_BFS_UNFUSED 1  /* fg_bfs, mode FG_MODE_PUSH_UNFUSED           */
#define FG_PRIM_SSSP 2         /* fg_sssp                                      */
#define FG_PRIM_MSBFS 3        /* fg_msbfs_* with `lanes` <= 64                */
#define FG_PRIM_MSSSP 4        /* fg_mssp_* (any `lanes` <= 64)                */
#define FG_PRIM_PR 5           /* fg_pagerank                                  */
#define FG_PRIM_CC 6           /* fg_cc                                        */

/*
 * Bytes of device workspace a call needs (just-enough sizing, Sec. VI-B:
 * frontier queues are bounded by |V_i|; the unfused advance additionally
 * needs an edge frontier bounded by |E_i|).  Returns 0 for bad arguments.
 * A workspace must be zero-filled once before its first use; every call
 * leaves it ready for the next one.  Its start must be 256-byte aligned
 * (every hipMalloc allocation is): the calls carve it into 256-byte aligned
 * pieces and return FG_EINVAL for a misaligned one.
 */
size_t fg_workspace_bytes(const fg_graph* g, int32_t primitive, int32_t lanes);

/* --------------------------------------------------------------- run stats */

#define FG_TRACE_MAX 64

/*
 * Device-resident record of one traversal, written by the library when the
 * caller passes a device pointer to it.  The per-iteration arrays hold the
 * first FG_TRACE_MAX iterations.
 */
typedef struct {
  int32_t status;           /* FG_OK or a device-side error code             */
  int32_t iterations;       /* iterations run (one per non-empty level)      */
  int64_t reached;          /* vertices with a finite depth / distance       */
  int64_t edges_inspected;  /* CSR entries read by advance / pull steps      */
  int32_t direction_switches;
  int32_t grid_blocks;      /* workgroups of the persistent launch           */
  int32_t clock_khz;        /* rate of the device wall clock below           */
  int32_t reserved;
  int64_t t_start;          /* device wall clock when the traversal started  */
  int8_t dir[FG_TRACE_MAX]; /* 0 = push (forward), 1 = pull (backward)       */
  int64_t frontier[FG_TRACE_MAX];  /* input frontier size |Q| per iteration */
  int64_t inspected[FG_TRACE_MAX]; /* CSR entries read per iteration         */
  int64_t t_end[FG_TRACE_MAX];     /* device wall clock when iteration ended */
} fg_run_stats;

/* Copy a device-resident fg_run_stats into host memory (synchronises `stream`). */
fg_status fg_stats_read(const fg_run_stats* dev_stats, fg_run_stats* host,
                        void* stream);

/* --------------------------------------------------------------------- BFS */

#define FG_MODE_DO 0            /* direction-optimizing (Sec. VI-A)            */
#define FG_MODE_PUSH 1          /* fused advance+filter only (Sec. VI-C)       */
#define FG_MODE_PUSH_UNFUSED 2  /* separate advance and filter kernels (Alg. 1) */

typedef struct {
  int32_t mode;        /* FG_MODE_*                                          */
  uint32_t do_a_num;   /* forward->backward when FV > (num/den) * BV         */
  uint32_t do_a_den;   /*   (Sec. VI-A do_a; default 1/100)                   */
  uint32_t do_b_num;   /* backward->forward when FV < (num/den) * BV         */
  uint32_t do_b_den;   /*   (Sec. VI-A do_b; default 1/10)                    */
  int32_t small_frontier; /* single-workgroup levels while |Q| <= this (0 = default) */
  int32_t small_edges;    /* ... and sum of degrees <= this (0 = default)     */
  int32_t big_degree;     /* push: vertices of at least this degree are
                             expanded by the whole grid (0 = default)         */
  int32_t blocks_per_cu;  /* persistent launch width (0 = default)            */
  int32_t team_blocks;    /* team mode width: workgroups that run medium
                             levels alone (0 = default, < 0 = off)          */
  int32_t team_edges;     /* team mode while the frontier's degree sum is at
                             most this (0 = default)                         */
  int32_t async_levels;   /* FG_MODE_PUSH, one source per call: > 1 runs the
                             traversal on a team of team_blocks workgroups
                             that synchronise every async_levels levels
                             (label-correcting keys; same depths, parents the
                             smallest-id neighbour one level closer); the
                             level-synchronous kernel takes over if a
                             member's frontier outgrows its LDS room
                             (0 = level-synchronous; at most 1024)            */
  int32_t grid_blocks;    /* workgroups of the persistent launch (0 = every CU x
                             blocks_per_cu); in fg_bfs_corun, of the list's
                             share (0 = every workgroup the team leaves)     */
} fg_bfs_opts;

/* Fill *opts with the defaults (DO mode, do_a = 1/100, do_b = 1/10). */
void fg_bfs_opts_default(fg_bfs_opts* opts);

/*
 * Breadth-first search from `src` (Alg. 1; Alg. 2 and Sec. VI-A in
 * FG_MODE_DO).  depth: device int32[n], receives the hop distance from src
 * or -1.  parent: device int32[n] or NULL; receives a BFS-tree predecessor
 * (parent[src] = src, -1 if unreached); which of several valid parents is
 * chosen may differ between runs.  ws: device workspace of at least
 * fg_workspace_bytes(g, FG_PRIM_BFS or FG_PRIM_BFS_UNFUSED, 0) bytes.
 * stats: device fg_run_stats* or NULL.  opts may be NULL (defaults).
 * Errors: FG_EINVAL (src out of range, NULL depth/ws, bad opts),
 * FG_ENOMEM (ws_bytes too small; the required size is in the message),
 * FG_EUNSUPPORTED (FG_MODE_DO on a graph without FG_SYMMETRIC), FG_EDEVICE.
 */
fg_status fg_bfs(const fg_graph* g, int32_t src, const fg_bfs_opts* opts,
                 void* ws, size_t ws_bytes, int32_t* depth, int32_t* parent,
                 fg_run_stats* stats, void* stream);

/*
 * Several BFS queries in one launch (the one-source-at-a-time workload of
 * Sec. VII: each source's traversal is exactly fg_bfs's, run after the
 * previous one has finished, without returning to the host between them).
 * srcs: device int32[nsrc]; a source outside [0, n) is skipped and its
 * record gets status FG_EINVAL.  The traversal of srcs[j] writes
 * depth + j * out_stride and parent + j * out_stride (out_stride = 0: every
 * traversal writes the same arrays, the last one's result remains;
 * otherwise out_stride >= n) and stats + j (device fg_run_stats[nsrc], or
 * NULL).  opts, ws and errors as for fg_bfs (FG_EUNSUPPORTED for the
 * unfused mode; the asynchronous push mode, async_levels > 1, is a
 * one-source mode, so the sources run level-synchronously here).  With
 * out_stride = 0 a traversal after the first writes only the vertices it
 * reaches and resets those the previous one reached alone, which keeps
 * the outputs exactly fg_bfs's; the workspace holds the visited set in
 * between, so it must not be used by another call during the launch.
 * nsrc = 0 does nothing.
 */
fg_status fg_bfs_many(const fg_graph* g, const int32_t* srcs, int32_t nsrc,
                      const fg_bfs_opts* opts, void* ws, size_t ws_bytes, int32_t* depth,
                      int32_t* parent, int64_t out_stride, fg_run_stats* stats, void* stream);

/*
 * Two BFS workloads in one launch, side by side on disjoint workgroups, for
 * callers that hold both at once (a step with a list of low-diameter
 * queries and one high-diameter query): the list `srcs` on g exactly as
 * fg_bfs_many (arguments, outputs, records and errors as there), and one
 * push query from src2 on g2 exactly as fg_bfs with opts2, which must be
 * FG_MODE_PUSH with async_levels > 1 (else FG_EINVAL).  The second query's
 * asynchronous team (opts2->team_blocks workgroups) takes the launch's
 * last workgroups and the list runs on the others (on the first
 * opts->grid_blocks of them when that is set and smaller; the rest stay
 * idle); neither waits for the other.  If the team gives up (a member's frontier outgrows its LDS room),
 * the second query runs level-synchronously after the launch, as in
 * fg_bfs.  ws2: workspace of g2 as for fg_bfs; the two workspaces must not
 * overlap (FG_EINVAL) and no other call may use either meanwhile; the two
 * queries' outputs must not overlap.  A team that leaves the list no
 * workgroup gives FG_EINVAL.  nsrc = 0 runs the second query alone.  Each
 * traversal is the one its own entry point runs (Alg. 2 and Sec. VI-A for
 * the list in FG_MODE_DO; the second query's depths as Alg. 1's); running
 * them side by side is the library's scheduling, not the paper's.
 */
fg_status fg_bfs_corun(const fg_graph* g, const int32_t* srcs, int32_t nsrc,
                       const fg_bfs_opts* opts, void* ws, size_t ws_bytes, int32_t* depth,
                       int32_t* parent, int64_t out_stride, fg_run_stats* stats,
                       const fg_graph* g2, int32_t src2, const fg_bfs_opts* opts2, void* ws2,
                       size_t ws2_bytes, int32_t* depth2, int32_t* parent2,
                       fg_run_stats* stats2, void* stream);

/*
 * fg_bfs without allocations, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same search, arguments, outputs and errors as fg_bfs
 * in modes FG_MODE_DO and FG_MODE_PUSH, but the workspace is a static
 * device array of FG_NOALLOC_SCRATCH_BYTES that the library holds on each
 * GPU it runs on until the process ends; the call itself allocates
 * nothing.  Graphs whose workspace (fg_workspace_bytes(g, FG_PRIM_BFS, 0))
 * exceeds that size get FG_ENOMEM; FG_MODE_PUSH_UNFUSED gets
 * FG_EUNSUPPORTED.  Every call on one GPU shares that GPU's array: calls
 * that overlap in time on one GPU (other streams, other threads) race and
 * give wrong results; calls ordered on one stream are safe.
 */
#define FG_NOALLOC_SCRATCH_BYTES (64u << 20)

fg_status fg_bfs_noalloc(const fg_graph* g, int32_t src, const fg_bfs_opts* opts,
                         int32_t* depth, int32_t* parent, fg_run_stats* stats, void* stream);

/* -------------------------------------------------------------------- SSSP */

typedef struct {
  int32_t small_frontier; /* single-workgroup iterations while |F| <= this (0 = default) */
  int32_t small_edges;    /* ... and sum of degrees <= this (0 = default)     */
  int32_t big_degree;     /* vertices of at least this degree are relaxed by
                             the whole grid (0 = default)                     */
  int32_t blocks_per_cu;  /* persistent launch width (0 = default)            */
  int32_t grid_blocks;    /* workgroups of the persistent launch (0 = every
                             CU x blocks_per_cu); fewer make each grid barrier
                             cheaper when frontiers are small              */
  uint32_t delta;         /* near-far threshold step: only vertices closer
                             than the threshold are relaxed; it grows by delta
                             when none is left (0 = default: 64 x mean weight
                             / mean degree; UINT32_MAX = no threshold, plain
                             frontier Bellman-Ford).  Results do not depend
                             on it.                                          */
  int32_t team_blocks;    /* workgroups that run medium frontiers from LDS
                             queues as a team (0 = 32 on graphs of mean
                             degree <= 8, no team on others; -1 = no team) */
  int32_t team_edges;     /* ... while the frontier's degree sum is at most
                             this (0 = 65536)                                */
} fg_sssp_opts;

void fg_sssp_opts_default(fg_sssp_opts* opts);

/*
 * Single-source shortest paths with the graph's uint32 weights (Table I's
 * SSSP primitive; weights are non-negative integers, Sec. VII-A).  A
 * frontier traversal whose advance relaxes every out-edge of the frontier;
 * the frontier holds the improved vertices closer than a threshold that
 * grows in steps of opts->delta (near-far ordering), and the traversal
 * converges when no distance improves.
 * dist: device uint32[n], receives the shortest-path weight from src or
 * UINT32_MAX if unreachable.  parent: device int32[n] or NULL; receives the
 * smallest-id u with an edge u->v and dist[u] + w(u,v) == dist[v]
 * (parent[src] = src, -1 if unreachable), which is unique.  ws: at least
 * fg_workspace_bytes(g, FG_PRIM_SSSP, 0) bytes.  Errors: FG_EINVAL (graph
 * without weights, src out of range, NULL dist / ws), FG_ENOMEM,
 * FG_EDEVICE; stats->status = FG_EOVERFLOW if a distance reaches 2^32 - 1.
 */
fg_status fg_sssp(const fg_graph* g, int32_t src, const fg_sssp_opts* opts, void* ws,
                  size_t ws_bytes, uint32_t* dist, int32_t* parent, fg_run_stats* stats,
                  void* stream);

/* ----------------------------------------------------------- BFS operators */

/*
 * Device-resident frontier lengths (the boundary's "length from the device
 * or the host"): the operators below that take a frontier length also take
 * `len_dev`.  When len_dev is NULL, `len` is the length.  Otherwise the
 * length is read on the device from *len_dev when the call's kernels run
 * (so a caller can chain operators without reading lengths back), and
 * `len` is an upper bound the caller guarantees; device lengths above it
 * are clamped to it.  Work is sized for `len`, so a tight bound is faster.
 */

/*
 * Advance (Sec. II-B): the edge frontier of `frontier` (device int32[len]).
 * For frontier entry i = 0..len-1 and its CSR neighbours j in order, writes
 * out_dst[k] = neighbour and out_src[k] = frontier[i] at k = sum of the
 * degrees of entries 0..i-1 plus j (a deterministic layout).  The total is
 * written to *out_len (device int64).  If it exceeds `capacity`, nothing
 * beyond capacity is written and *out_len reports the needed size; the
 * host-visible return is FG_OK (the size is only known on the device).
 * len_dev: device int32 length or NULL (see above).  ws: device workspace
 * of at least fg_workspace_bytes(g, FG_PRIM_BFS_UNFUSED, 0) bytes.
 */
fg_status fg_advance(const fg_graph* g, const int32_t* frontier, int32_t len,
                     const int32_t* len_dev, int32_t* out_dst, int32_t* out_src,
                     int64_t capacity, int64_t* out_len, void* ws, size_t ws_bytes,
                     void* stream);

/*
 * Filter (Sec. II-B, with the computation step fused): for each edge-
 * frontier entry k (device arrays dst/src of length len), if vertex dst[k]
 * is not yet set in `visited` (device uint32 bitmask of ceil(n/32) words,
 * bit v%32 of word v/32) it is atomically marked, depth[dst] = iter + 1,
 * parent[dst] = src[k] (parent may be NULL) and dst is appended to out_q
 * (device int32, capacity n).  Each vertex is appended at most once; the
 * order of out_q is unspecified.  *out_len (device int32) receives the count.
 * len_dev: device int64 edge-frontier length (e.g. fg_advance's *out_len)
 * or NULL, as described above.
 */
fg_status fg_filter(const fg_graph* g, const int32_t* dst, const int32_t* src,
                    int64_t len, const int64_t* len_dev, uint32_t* visited, int32_t iter,
                    int32_t* depth, int32_t* parent, int32_t* out_q, int32_t* out_len,
                    void* stream);

/*
 * Backward (pull) step of one iteration (Sec. VI-A): every vertex v with
 * degree > 0 whose `visited` bit is clear scans its CSR row in order and
 * stops at the first neighbour u whose bit is set in `frontier_bits`
 * (level `iter`).  Then depth[v] = iter+1, parent[v] = u (parent may be
 * NULL), v's bit is set in `visited` and in `next_bits`, and v is appended
 * to out_q.  Every word of next_bits is overwritten.  Bitmaps are device
 * uint64 arrays of ceil(n/64) words (bit v%64 of word v/64).  *out_len
 * (device int32) receives the number of new vertices and *inspected (device
 * int64, may be NULL) the number of CSR entries read.
 */
fg_status fg_pull_step(const fg_graph* g, const uint64_t* frontier_bits,
                       uint64_t* visited, uint64_t* next_bits, int32_t iter,
                       int32_t* depth, int32_t* parent, int32_t* out_q,
                       int32_t* out_len, int64_t* inspected, void* stream);

/*
 * Frontier conversions (Sec. VI-A: the newly discovered list gives a
 * direction-independent view).  queue -> bitmap ORs the bits of
 * queue[0..len) into `bits` (device uint64[ceil(n/64)], not cleared first).
 * bitmap -> queue lists the set bits in ascending order into out_q and
 * writes the count to *out_len (device int32).
 */
fg_status fg_queue_to_bitmap(const fg_graph* g, const int32_t* queue,
                             int32_t len, uint64_t* bits, void* stream);
fg_status fg_bitmap_to_queue(const fg_graph* g, const uint64_t* bits,
                             int32_t* out_q, int32_t* out_len, void* ws,
                             size_t ws_bytes, void* stream);

/* ------------------------------------------------------ batched BFS (64 lanes) */

typedef struct fg_msbfs fg_msbfs;

typedef struct {
  int32_t big_degree;    /* push: degree from which edges go to descriptors (0 = 64) */
  int32_t pull_div;      /* push -> pull when active vertices > n / pull_div (0 = 64) */
  int32_t push_div;      /* pull -> push when active vertices < n / push_div (0 = 64) */
  int32_t blocks_per_cu; /* persistent launch width (0 = default)                     */
  int32_t grid_blocks;   /* workgroups of the persistent launch (0 = every CU x
                            blocks_per_cu)                                          */
  int32_t team_blocks;   /* workgroups that run push levels of medium frontiers from
                            LDS queues as a team (> 1 = that many; 1 = 32 while
                            fewer than 4 lanes hold queries, 64 otherwise; 0 = as 1
                            on graphs of mean degree <= 8, no team on others;
                            -1 = no team)                                        */
  int32_t team_edges;    /* ... while the frontier's degree sum is at most this
                            (0 = 262144)                                            */
} fg_msbfs_opts;

void fg_msbfs_opts_default(fg_msbfs_opts* opts);

/*
 * A batch of up to 64 independent BFS queries (lanes) that share one
 * traversal with one bit per lane in each vertex word.  Each query is
 * Alg. 1's BFS (push levels, and pull levels as in Sec. VI-A's backward
 * step); the paper runs its sources one after another (Sec. VII), and
 * batching them is this library's serving mode, not the paper's.  Each
 * lane's depths equal fg_bfs's depths from its source.  Lanes are admitted at any step
 * boundary (continuous batching) and are done when their frontier empties.
 * ws: device workspace of fg_workspace_bytes(g, FG_PRIM_MSBFS, lanes) bytes,
 * owned by the caller, used exclusively by this batch until fg_msbfs_close.
 * fg_msbfs_open clears the batch state (asynchronously on `stream`).
 */
fg_status fg_msbfs_open(const fg_graph* g, int32_t lanes, void* ws, size_t ws_bytes,
                        const fg_msbfs_opts* opts, void* stream, fg_msbfs** out);
fg_status fg_msbfs_close(fg_msbfs* b);

/* Queue query `src` for lane `lane`; it starts at the next fg_msbfs_step.
 * The lane's previous result is discarded.  FG_EINVAL for a bad lane / src
 * or a lane already pending. */
fg_status fg_msbfs_admit(fg_msbfs* b, int32_t lane, int32_t src);

/* Run at most k_iters BFS levels for every live lane (fewer if all lanes
 * finish), asynchronously on `stream`. */
fg_status fg_msbfs_step(fg_msbfs* b, int32_t k_iters, void* stream);

/* Synchronise `stream`; *done_lanes = admitted lanes whose traversal has
 * finished; *iterations = levels run since fg_msbfs_open.  Either pointer
 * may be NULL.  Returns FG_EDEVICE if a step stopped early (its results
 * are then incomplete). */
fg_status fg_msbfs_poll(fg_msbfs* b, uint64_t* done_lanes, int32_t* iterations, void* stream);

/* Copy lane's depths (int32[n], -1 = unreached) to device memory `depth`
 * (asynchronous on `stream`). */
fg_status fg_msbfs_read(fg_msbfs* b, int32_t lane, int32_t* depth, void* stream);

/* Synchronise `stream`; work done since fg_msbfs_open: *edges = adjacency
 * entries read (push: whole lists of active vertices; pull: up to the early
 * exit), *verts = vertex visits (push: active vertices; pull: every vertex
 * of the graph per pull level).  Either pointer may be NULL. */
fg_status fg_msbfs_counts(fg_msbfs* b, uint64_t* edges, uint64_t* verts, void* stream);

/* Forget the query held by `lane` (it no longer reports as done). */
fg_status fg_msbfs_release(fg_msbfs* b, int32_t lane);

/* ----------------------------------------------------- batched SSSP (64 lanes) */

typedef struct fg_mssp fg_mssp;

typedef struct {
  uint32_t delta;        /* near-far threshold step of every lane (0 = the
                            fg_sssp default on graphs of mean degree <= 8,
                            twice it on others; UINT32_MAX = no threshold) */
  int32_t big_degree;    /* vertices of at least this degree are relaxed in
                            64-edge chunks by many waves (0 = 256)           */
  int32_t blocks_per_cu; /* persistent launch width (0 = default)            */
  int32_t grid_blocks;   /* workgroups of the persistent launch (0 = every CU
                            x blocks_per_cu)                                 */
  int32_t dense_lanes;   /* a vertex with at least this many frontier lanes is
                            relaxed by one wave across its lanes; fewer lanes
                            are relaxed one (edge, lane) pair per thread
                            (0 = 16)                                         */
  int32_t split_lanes;   /* lanes whose near frontier is empty wait until this
                            many can split in one scan of the far list (0 = 8) */
  int32_t split_wait;    /* ... or until they have waited this many
                            iterations (0 = 8 on graphs of mean degree <= 8,
                            1 on others); 1 = split at once                 */
  int32_t team_blocks;   /* workgroups that run near iterations of medium
                            frontiers from LDS queues as a team (0 = on
                            graphs of mean degree <= 8: 32 while fewer than
                            4 lanes hold queries, 64 otherwise; no team on
                            others; -1 = no team)                            */
  int32_t team_edges;    /* ... while the frontier's degree sum is at most
                            this (0 = 262144)                                */
} fg_mssp_opts;

void fg_mssp_opts_default(fg_mssp_opts* opts);

/*
 * A batch of up to 64 independent SSSP queries (lanes) over the graph's
 * uint32 weights (Table I's SSSP, one query per source; batching them is
 * this library's serving mode, not the paper's) sharing one traversal: each iteration relaxes, for every vertex in some lane's near
 * frontier, its edges for all of those lanes at once, and each lane orders
 * its work near-far with its own threshold (see fg_sssp).  Each lane's
 * distances equal fg_sssp's distances from its source (no parents).  Lanes
 * are admitted at any step boundary (continuous batching) and are done when
 * their near frontier and far pile are empty.  ws: device workspace of
 * fg_workspace_bytes(g, FG_PRIM_MSSSP, 64) bytes (distances for 64 lanes:
 * 256 bytes per vertex), owned by the caller, used exclusively by this batch
 * until fg_mssp_close.  fg_mssp_open clears the batch state (asynchronously
 * on `stream`).  Errors: FG_EINVAL (no weights, lanes outside [1, 64], NULL
 * arguments), FG_ENOMEM (workspace too small).
 */
fg_status fg_mssp_open(const fg_graph* g, int32_t lanes, void* ws, size_t ws_bytes,
                       const fg_mssp_opts* opts, void* stream, fg_mssp** out);
fg_status fg_mssp_close(fg_mssp* b);

/* Queue query `src` for lane `lane`; it starts at the next fg_mssp_step.
 * The lane's previous result is discarded.  FG_EINVAL for a bad lane / src
 * or a lane already pending. */
fg_status fg_mssp_admit(fg_mssp* b, int32_t lane, int32_t src);

/* Run at most k_iters iterations for every live lane (fewer if all lanes
 * finish), asynchronously on `stream`. */
fg_status fg_mssp_step(fg_mssp* b, int32_t k_iters, void* stream);

/* Synchronise `stream`; *done_lanes = admitted lanes whose query has
 * finished; *iterations = iterations run since fg_mssp_open.  Either pointer
 * may be NULL.  Returns FG_EOVERFLOW once a distance would reach 2^32 - 1
 * (the affected lane's result is then incomplete), FG_EDEVICE if a step
 * stopped early. */
fg_status fg_mssp_poll(fg_mssp* b, uint64_t* done_lanes, int32_t* iterations, void* stream);

/* Synchronise `stream`; work done since fg_mssp_open: *edges = edge visits
 * (an edge relaxed for all of a vertex's lanes counts once), *edge_lanes =
 * relaxations attempted (per lane).  Either pointer may be NULL. */
fg_status fg_mssp_counts(fg_mssp* b, uint64_t* edges, uint64_t* edge_lanes, void* stream);

/* Copy lane's distances (uint32[n], UINT32_MAX = unreachable) to device
 * memory `dist` (asynchronous on `stream`). */
fg_status fg_mssp_read(fg_mssp* b, int32_t lane, uint32_t* dist, void* stream);

/* Forget the query held by `lane` (it no longer reports as done). */
fg_status fg_mssp_release(fg_mssp* b, int32_t lane);

/* ----------------------------------------------------- partition + package */

typedef struct fg_share fg_share;

/*
 * One GPU's share of a vertex-partitioned graph (Sec. III-C duplicate-1-hop;
 * the random partitioner of Sec. V-C supplies `owner`).  Hosted vertices
 * (owner == part) get local ids 0..n_local-1 in ascending global order;
 * remote neighbours of hosted vertices become proxies n_local..n_total-1 in
 * ascending global order; a hosted row keeps its neighbours' global order,
 * renamed to local ids; proxies have no out-edges.  For each local vertex the
 * share keeps its owner, its id on the owner (conv = rank among the owner's
 * hosted vertices) and its global id.  row_offsets / col_idx / owner are host
 * arrays (int32[n+1], int32[m], uint8[n]); 1 <= nparts <= 16; n < 2^28.
 * Errors: FG_EINVAL, FG_EUNSUPPORTED (n too large), FG_ENOMEM, FG_EDEVICE.
 */
fg_status fg_share_create(int32_t n, int64_t m, const int32_t* row_offsets,
                          const int32_t* col_idx, const uint8_t* owner, int32_t nparts,
                          int32_t part, void* stream, fg_share** out);
fg_status fg_share_destroy(fg_share* s);

/*
 * Source setting on a share (the framework's reset for a new source: the
 * GPU that hosts the source seeds its frontier, the others start empty;
 * Sec. III-B): clears `visited` (device uint32[ceil(n_total/32)]), sets
 * depth (and parent, if not NULL) to -1 over the share's n_total vertices,
 * and if the share hosts global vertex `src`, marks its local id visited at
 * depth 0 (parent = src, the global id) and writes it to queue[0]; *qlen
 * (device int32) receives 1 or 0.  Everything happens on the device,
 * asynchronously on `stream`.  Errors: FG_EINVAL (NULL arguments, src
 * outside [0, n_global)).
 */
fg_status fg_share_seed(const fg_share* s, int32_t src, uint32_t* visited, int32_t* depth,
                        int32_t* parent, int32_t* queue, int32_t* qlen, void* stream);

typedef struct {
  int32_t n_global;
  int32_t n_local;
  int32_t n_total;
  int32_t nparts;
  int32_t part;
  int32_t reserved;
  int64_t m_local;
} fg_share_info_t;

fg_status fg_share_info(const fg_share* s, fg_share_info_t* info);

/* The share's local CSR as a graph (owned by the share; push traversals). */
const fg_graph* fg_share_graph(const fg_share* s);

/* Device tables of the share (owned by it): owner uint8[n_total],
 * conv int32[n_total], l2g int32[n_total].  Any output pointer may be NULL. */
fg_status fg_share_tables(const fg_share* s, const uint8_t** owner, const int32_t** conv,
                          const int32_t** l2g);

typedef struct {
  int32_t* ids;         /* device int32[nparts * capacity]; peer p at p*capacity */
  int32_t* depth;       /* same layout: depth[v] of each packaged vertex         */
  int32_t* parent;      /* same layout: global id of parent[v], or NULL          */
  int32_t* counts;      /* device int32[nparts]; counts[part] = 0                 */
  int32_t* local;       /* device int32[capacity] local sub-frontier, or NULL     */
  int32_t* local_count; /* device int32[1], or NULL                               */
  int64_t capacity;     /* entries per buffer, >= len                             */
} fg_peer_bufs;

/* Workspace bytes fg_package needs for frontiers of up to max_len entries. */
size_t fg_package_workspace_bytes(const fg_share* s, int32_t max_len);

/*
 * Split + package (Sec. III-B): walk frontier[0..len) (device, local ids) in
 * order; vertices v < n_local go to the local sub-frontier; every proxy v is
 * appended to the buffer of its owner p as (conv[v], depth[v], global id of
 * parent[v] if parent != NULL).  Buffers keep frontier order (stable), so the
 * result is deterministic.  depth / parent are device int32[n_total] (local
 * ids).  len_dev: device int32 frontier length or NULL (device-resident
 * lengths, above); the workspace is sized for `len`.  Errors: FG_EINVAL
 * (len outside [0, n_total], capacity < len, NULL buffers), FG_ENOMEM
 * (workspace), FG_EDEVICE.
 */
fg_status fg_package(const fg_share* s, const int32_t* frontier, int32_t len,
                     const int32_t* len_dev, const int32_t* depth, const int32_t* parent,
                     const fg_peer_bufs* out, void* ws, size_t ws_bytes, void* stream);

/*
 * Combine (Sec. III-B merge step; Alg. 1 combination rule): for each
 * received vertex ids[i] (device, local ids of the receiving share) that is
 * not yet set in `visited` (device uint32 bitmask, bit v%32 of word v/32),
 * atomically mark it, set depth[v] = labels[i] (and parent[v] = parents[i]
 * when both are given) and append v to out_q at position atomicAdd(out_len).
 * *out_len (device int32) is not reset, so received vertices can be appended
 * after the local sub-frontier.  A vertex received several times is taken
 * once.  len_dev: device int32 count (e.g. an entry of the sender's
 * fg_peer_bufs.counts) or NULL, as for the operators above.
 * Errors: FG_EINVAL.
 */
fg_status fg_combine(const fg_graph* g, const int32_t* ids, const int32_t* labels,
                     const int32_t* parents, int32_t len, const int32_t* len_dev,
                     uint32_t* visited, int32_t* depth, int32_t* parent, int32_t* out_q,
                     int32_t* out_len, void* stream);

/* ------------------------------- duplicate-all + broadcast DOBFS (Alg. 2) */

/*
 * One partition of a multi-GPU direction-optimizing BFS under the
 * duplicate-all vertex model with broadcast communication (Sec. III-C; the
 * BFS of Alg. 2 with the direction rule of Sec. VI-A; the newly-discovered
 * set as the direction-independent view of Sec. VI-A).  The partition
 * keeps every one of the n vertices under its global id but only the rows
 * of the vertices it hosts (owner[v] == part); one GPU would hold one
 * fg_dup, and on a single GPU several fg_dup objects emulate the
 * partitions, with device copies standing in for the transfers.
 *
 * Per iteration, on every partition: fg_dup_step (direction from the
 * global counts, identical on every partition; forward: the hosted
 * frontier vertices' rows are expanded and unlabelled neighbours take the
 * next depth; backward: every hosted unlabelled vertex scans its row in
 * order and stops at the first labelled neighbour), then fg_dup_send from
 * every partition to every other one (the broadcast: the newly-discovered
 * set as an id list after a forward step, as an n-bit bitmap after a
 * backward step), then fg_dup_combine (received vertices not yet labelled
 * take the next depth; the union is the next frontier; the iteration's
 * counters, direction state and trace advance on the device).  Nothing is
 * read back between iterations; fg_dup_poll reads the stop flag.
 *
 * The same rule as fg_bfs decides directions (do_a / do_b of `opts`, NULL =
 * 1/100 and 1/10; other fields of opts are ignored), with |E| = m, the edge
 * count of the whole graph, and |V| = n.  Depths equal fg_bfs's on the whole
 * graph.  Parents: each partition writes parent[v] for the vertices it
 * discovers itself (global ids; parent[src] = src); the partitions may
 * share one parent array, and a vertex discovered by several partitions in
 * the same forward step then keeps one of their (valid) parents.
 */
typedef struct fg_dup fg_dup;

typedef struct {
  int32_t n;              /* vertices (global)                          */
  int32_t nparts;
  int32_t part;
  int32_t hosted;         /* vertices this partition hosts              */
  int64_t m_local;        /* CSR entries of the hosted rows             */
  int64_t m_total;        /* CSR entries of the whole graph             */
  int64_t resident_bytes; /* device bytes held by the object            */
} fg_dup_info_t;

/*
 * Builds partition `part` of `nparts` (1..16) from the whole graph's host
 * CSR (row_offsets int32[n+1], col_idx int32[m]) and the host owner map
 * (uint8[n], values < nparts).  The object owns its device copy of the
 * hosted rows and its traversal state (about 4n (3 + nparts) + n/8 (3 +
 * nparts) bytes besides the rows).  Errors: FG_EINVAL (bad CSR or owner
 * map), FG_ENOMEM, FG_EDEVICE.
 */
fg_status fg_dup_create(int32_t n, int64_t m, const int32_t* row_offsets,
                        const int32_t* col_idx, const uint8_t* owner, int32_t nparts,
                        int32_t part, const fg_bfs_opts* opts, void* stream, fg_dup** out);
fg_status fg_dup_destroy(fg_dup* d);
fg_status fg_dup_info(const fg_dup* d, fg_dup_info_t* info);
/* The partition's CSR (n vertices, only hosted rows non-empty; owned). */
const fg_graph* fg_dup_graph(const fg_dup* d);

/*
 * Source setting: depth (device int32[n]) = -1 except depth[src] = 0,
 * parent (device int32[n] or NULL) = -1 except parent[src] = src, visited =
 * {src}, frontier = {src}; `stats` (device fg_run_stats or NULL) receives the
 * iteration trace (dir, frontier = |Q| of the whole graph, inspected = CSR
 * entries read by this partition).  depth / parent / stats stay bound to
 * the object until the next seed.  Errors: FG_EINVAL.
 */
fg_status fg_dup_seed(fg_dup* d, int32_t src, int32_t* depth, int32_t* parent,
                      fg_run_stats* stats, void* stream);
/* The local computation of one iteration (writes the outgoing message). */
fg_status fg_dup_step(fg_dup* d, void* stream);
/* The broadcast leg from -> to: copies from's message of this iteration into
 * to's receive slot for from's partition.  Errors: FG_EINVAL (same object,
 * or partitions of different graphs / counts). */
fg_status fg_dup_send(const fg_dup* from, fg_dup* to, void* stream);
/* Merges the received messages with the partition's own and advances the
 * iteration (device-side). */
fg_status fg_dup_combine(fg_dup* d, void* stream);
/* Synchronises `stream` and reads the stop flag and the iterations run. */
fg_status fg_dup_poll(const fg_dup* d, int32_t* done, int32_t* iterations, void* stream);

/*
 * The whole traversal from `src` over parts[0..nparts) (parts[p] must be
 * partition p of nparts, all of one graph): seeds every partition, then
 * enqueues step / send / combine rounds, reading the stop flag every
 * `poll_every` iterations (< 1: 4).  depth[p] / parent[p] / stats[p] are
 * partition p's outputs (parent and stats may be NULL, or hold NULL
 * entries).  Errors: FG_EINVAL, FG_EDEVICE.
 */
fg_status fg_dup_run(fg_dup* const* parts, int32_t nparts, int32_t src,
                     int32_t* const* depth, int32_t* const* parent,
                     fg_run_stats* const* stats, int32_t poll_every, void* stream);

/* ------------------------------------------------- connected components */

/*
 * Connected components (Table I's CC primitive, computed by hooking and
 * pointer jumping): label[v] = the smallest vertex id of v's component, so
 * the labelling is unique.  label: device int32[n], also the working
 * forest while the call runs.  components: device int64 or NULL; receives
 * the number of components.  ws: fg_workspace_bytes(g, FG_PRIM_CC, 0)
 * bytes (any contents).  Needs an undirected graph (FG_SYMMETRIC), else
 * FG_EUNSUPPORTED.  Errors: FG_EINVAL, FG_ENOMEM (workspace), FG_EDEVICE.
 */
fg_status fg_cc(const fg_graph* g, int32_t* label, int64_t* components, void* ws,
                size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- PageRank */

/*
 * PageRank by power iteration in double precision (Table I's PR primitive:
 * the rank update and the accumulation over edges of Alg. 3) on an
 * undirected graph, each edge carrying rank both ways.  rank_0 = 1/n; an
 * iteration sets rank'(v) = (1 - damping)/n + damping * sum over the
 * neighbours u of v of rank(u)/deg(u) (rank reaching a vertex of degree 0
 * is not passed on).  The run stops after an iteration in which every
 * vertex changed by at most tol times its previous rank (tol > 0), or
 * after max_iter iterations (tol = 0 runs exactly max_iter).  rank: device
 * double[n], the output.  ws: fg_workspace_bytes(g, FG_PRIM_PR, 0) bytes
 * (any contents).  stats (device, may be NULL): iterations run, and per
 * iteration frontier[i] = vertices whose change exceeded the threshold,
 * inspected[i] = m.  Nothing is read back: every one of the max_iter
 * iterations is enqueued and those after convergence return at once.
 * Sums over long rows are taken in a different order than a serial loop,
 * so ranks agree with a serial evaluation to rounding, not bit for bit.
 * Errors: FG_EINVAL (damping outside [0, 1], tol < 0, max_iter outside
 * [0, 100000]), FG_ENOMEM (workspace), FG_EUNSUPPORTED (directed graph).
 */
fg_status fg_pagerank(const fg_graph* g, double damping, double tol, int32_t max_iter,
                      void* ws, size_t ws_bytes, double* rank, fg_run_stats* stats,
                      void* stream);

#ifdef __cplusplus
}
#endif

#endif /* FG_H */
