// Breadth-first search on one GPU: fused advance+filter push iterations
// (Sec. II-B operators, Alg. 1, kernel fusion of Sec. VI-C) and the
// direction-optimizing variant with the vertex-parallel early-exit pull
// step and the inexpensive direction rule (Sec. VI-A, Alg. 2).
//
// The whole traversal runs in one cooperative (co-resident) launch: every
// iteration's direction is decided on the device from counters the
// iteration before produced, so the host is not involved between
// iterations.  Levels whose frontier is small are run by workgroup 0 alone
// (no grid barrier at all); larger levels use the whole grid and one grid
// barrier per iteration (two when high-degree vertices are present).
//
// Push load balance: a vertex of degree below `big_degree` is expanded by a
// wave-level scan-gather (each lane takes one edge per round); a vertex of
// higher degree is cut into descriptors of CH consecutive edges that every
// wave of the grid then takes in turn, so no wave walks a hub alone and no
// per-edge search is needed.
//
// Data layout in HBM (all owned by the caller's workspace, 256-B aligned):
//   visited   2 x uint64[ceil(n/64)]  current / next visited bitmap
//   queue     2 x int32[n]            input / output vertex frontier
//   desc      int4[m/CH + n + 64]     edge-chunk descriptors {vertex, first edge, end edge}
//   control   barrier, counters, hand-back state of the small-frontier mode
#include <string.h>

#include <mutex>

#include "frontier.h"

namespace {
using namespace fgk;

constexpr int PB = 1024;          // persistent workgroup size
constexpr int PWAVES = PB / FG_WAVE;
constexpr int CH = 256;           // edges per descriptor
constexpr int DIR_PUSH = 0, DIR_PULL = 1;

constexpr int QCAP = 2048;    // LDS frontier entries per workgroup in LDS-queue mode
constexpr int TEAM_MAX = 64;  // widest team (one record per lane of a wave)
// Fields of a team level word: arrivals, flagged members, vertices
// discovered, degree sum (each member's degree sum capped at TW_CAP, so 64
// members cannot carry out of the field; team_e < TW_CAP keeps every
// team-mode decision exact).
constexpr int TW_CNT = 25, TW_FLAG = 50, TW_ARR = 57;
constexpr int64_t TW_CAP = (1 << 19) - 1;
constexpr int LDS_MEAN_DEG = 64;  // LDS-queue levels need a frontier of mean degree
                                  // <= this (hubs are cut up by the whole grid)
constexpr int TPV = 4;        // LDS-queue levels: vertices of degree <= TPV are
                              // expanded by TPV lanes each, without a scan
constexpr int32_t DEF_SMALL_Q = QCAP;
// workgroup 0 alone while the frontier's degree sum fits one pass of its
// low-degree loop (PB / TPV vertices of TPV edges); larger frontiers go
// faster as a team (grid 1024²: 3.36 µs per level at 1024, 3.50 at 1536,
// 5.1 at 3072)
constexpr int64_t DEF_SMALL_E = PB;
constexpr int32_t DEF_BIG_DEG = 64;
// team width: grid 4096² / 2048² / 1024² push BFS take 35.8 / 14.6 / 6.8 ms
// with 24 members, 36.2 / 15.1 / 7.2 ms with 32 (narrower frontiers prefer
// narrower teams: 16 is best at 1024², 24-28 at 4096²)
constexpr int32_t DEF_TEAM = 24;
constexpr int64_t DEF_TEAM_E = 65536;

typedef unsigned __int128 u128;
typedef unsigned long long ull;

// Counters of one iteration parity.  Iteration k appends through slot k&1;
// every workgroup reads the slot right after the iteration's last grid
// barrier, before it can reach iteration k+2, the next user of the slot, so
// monotone counters never need resetting.
struct CtrSlot {
  Line64 q;      // vertices discovered
  Line64 desc;   // edge-chunk descriptors written
  Line64 insp;   // CSR entries read
  Line64 deg;    // sum of the degrees of the discovered vertices
};

// The control block is zero when a launch starts: a fresh workspace is
// zero-filled by the caller, and the last workgroup to leave a launch clears
// it again for the next one.
struct alignas(256) BfsCtl {
  uint32_t bar[FG_BAR_WORDS];  // grid barrier (its second line is the abort flag)
  uint32_t sm_signal;          // small-frontier hand-backs (monotone)
  uint32_t pad2[63];
  uint32_t sm_ack;             // waiters that have read a hand-back (monotone)
  uint32_t pad2b[63];
  uint32_t exit_count;         // workgroups that left the launch
  uint32_t pad3[63];
  uint32_t team_arrive;        // barrier of the team (workgroups 0..team-1)
  uint32_t pad4[63];
  // LDS-queue mode: per level parity and member, the level's totals of the
  // member (vertices discovered, their degree sum), each word tagged with
  // the level number + 1 in its upper 32 bits
  ull team_rec[2][TEAM_MAX][2];
  // LDS-queue mode: per team level mod 3, the word every member adds its
  // arrival and totals to (fields TW_*)
  Line64 team_word[3];
  Line64 team_ovf;             // entries written to the global queue by the team
  Line64 solo_ovf;             // ... by workgroup 0 alone
  Line64 aux;                  // entries written by bitmap -> queue conversion
  CtrSlot slot[2];
  // state published by workgroup 0 when a small-frontier / team episode ends
  int32_t pub_k, pub_dir, pub_prevdir, pub_switched, pub_qsel, pub_force;
  int64_t pub_qlen, pub_p, pub_insp_sum;
  int32_t pub_switches;
  int64_t pub_qdeg;
  ull pub_b[8];
  // asynchronous push mode (bfs_async and its finalising kernels; cleared
  // by async_init_kernel at the start of each such traversal):
  uint32_t as_arrive;          // team barrier arrivals
  uint32_t pad5[63];
  uint32_t as_state;           // 1: a member ran out of queue room, the
  uint32_t pad6[63];           //   level-synchronous kernel behind runs instead
  uint32_t as_exit;            // members that left
  uint32_t pad7[63];
  ull as_rec[TEAM_MAX];        // per member: its queue length (exchange)
  ull as_hist_cnt[FG_TRACE_MAX];  // vertices per depth (first depths)
  ull as_hist_deg[FG_TRACE_MAX];  // ... their degree sums
  ull as_insp;                 // CSR entries read by the team
};

struct BfsParams {
  const int32_t* __restrict__ off;
  const int32_t* __restrict__ col;
  const uint64_t* __restrict__ nz;
  const int4* __restrict__ head;  // first four neighbours per vertex
  int32_t n;
  int32_t nwords;
  int64_t m;
  int32_t src;
  int32_t mode;
  int32_t* depth;
  int32_t* parent;
  uint64_t* vis[2];
  uint64_t* reached;  // see BfsLayout::reached
  int32_t* q[2];
  int4* desc;
  BfsCtl* ctl;
  fg_run_stats* stats;
  uint32_t a_num, a_den, b_num, b_den;
  int32_t small_q;
  int64_t small_e;
  int32_t big_deg;
  int32_t clock_khz;
  int32_t team;     // workgroups of the team mode (0 = off)
  int64_t team_e;   // team mode while the frontier's degree sum <= team_e
  // several sources one after another in one launch (srcs != NULL): the
  // traversal of srcs[j] writes depth / parent + j * out_stride and
  // stats + j
  const int32_t* srcs;
  int32_t nsrc;
  int64_t out_stride;
  // asynchronous push mode: levels per super-step (bfs_async), and the flag
  // of the level-synchronous launch queued behind it, which runs only if
  // the asynchronous traversal ran out of queue room
  int32_t async_k;
  int32_t async_fallback;
  // the traversal's workgroups: [blk0, blk0 + nblk) of the launch (a launch
  // may run two traversals side by side on disjoint ranges).  The
  // level-synchronous kernel always starts at workgroup 0 (blk0 = 0: its
  // code indexes workgroups by blockIdx.x, which costs no register); only an
  // asynchronous team takes an offset.
  uint32_t blk0;
  uint32_t nblk;
};

// Workgroups of the traversal.
__device__ __forceinline__ uint32_t fgb_n(const BfsParams& P) { return P.nblk; }
// An asynchronous team member's index.
__device__ __forceinline__ uint32_t as_member(const BfsParams& P) { return blockIdx.x - P.blk0; }

// What changes from one traversal of a launch to the next: the source and
// the traversal's index, from which its outputs and record follow (kept as
// two scalars, so that the kernel arguments stay in place).
struct BfsJob {
  int32_t job;
  int32_t src;
};

__device__ __forceinline__ int32_t* J_depth(const BfsParams& P, const BfsJob& J) {
  return P.depth + (int64_t)J.job * P.out_stride;
}
__device__ __forceinline__ int32_t* J_parent(const BfsParams& P, const BfsJob& J) {
  return P.parent ? P.parent + (int64_t)J.job * P.out_stride : nullptr;
}
__device__ __forceinline__ fg_run_stats* J_stats(const BfsParams& P, const BfsJob& J) {
  return P.stats ? P.stats + J.job : nullptr;
}

// Per-iteration state, identical in every workgroup.
struct St {
  int32_t k;         // iteration (= depth of the input frontier)
  int32_t dir;       // direction of iteration k
  int32_t prevdir;   // direction of iteration k-1
  int32_t switched;  // a forward->backward switch has happened
  int32_t qsel;      // queue holding the input frontier (push)
  int32_t cur;       // visited bitmap holding levels <= k
  int32_t switches;
  int64_t qlen;      // |Q| of iteration k
  int64_t qdeg;      // sum of the degrees of Q (edges a push would read)
  int64_t p;         // |P|: vertices with a depth, Q included
  int64_t insp_sum;  // CSR entries read so far
  // last read value of slot[p].{q, desc, insp}; kept as scalars so the
  // parity select does not force the state into scratch memory
  ull b0q, b0desc, b0insp, b0deg;
  ull b1q, b1desc, b1insp, b1deg;
  ull auxbase;
};

struct Bases {
  ull q, desc, insp, deg;
};


__device__ __forceinline__ ull sel(bool odd, ull a1, ull a0) {
  // branch-free select on a wave-uniform parity
  const ull m = 0ull - (ull)odd;
  return (a1 & m) | (a0 & ~m);
}

__device__ __forceinline__ Bases get_bases(const St& S) {
  const bool odd = S.k & 1;
  return Bases{sel(odd, S.b1q, S.b0q), sel(odd, S.b1desc, S.b0desc), sel(odd, S.b1insp, S.b0insp),
               sel(odd, S.b1deg, S.b0deg)};
}

__device__ __forceinline__ void set_bases(St& S, const Bases& b) {
  const bool odd = S.k & 1;
  S.b1q = sel(odd, b.q, S.b1q);
  S.b1desc = sel(odd, b.desc, S.b1desc);
  S.b1insp = sel(odd, b.insp, S.b1insp);
  S.b1deg = sel(odd, b.deg, S.b1deg);
  S.b0q = sel(odd, S.b0q, b.q);
  S.b0desc = sel(odd, S.b0desc, b.desc);
  S.b0insp = sel(odd, S.b0insp, b.insp);
  S.b0deg = sel(odd, S.b0deg, b.deg);
}

// Direction rule of Sec. VI-A for the iteration described by S (k >= 1):
// FV = |Q| m / n, BV = |U| n / |P|, U = n - |P|; forward->backward when
// FV > do_a BV (once), backward->forward when FV < do_b BV.  Exact in
// 128-bit integers: FV > (a/b) BV  <=>  b |Q| m |P| > a |U| n n.
template <int MODE>
__device__ __forceinline__ void decide(St& S, const BfsParams& P) {
  S.prevdir = S.dir;
  if (MODE != FG_MODE_DO || S.k == 0) {
    S.dir = DIR_PUSH;
    return;
  }
  const u128 lhs = (u128)(ull)S.qlen * (ull)P.m * (ull)S.p;
  const u128 rhs = (u128)(ull)((int64_t)P.n - S.p) * (ull)P.n * (ull)P.n;
  if (S.dir == DIR_PUSH) {
    if (!S.switched && lhs * P.a_den > rhs * P.a_num) {
      S.dir = DIR_PULL;
      S.switched = 1;
      S.switches++;
    }
  } else if (lhs * P.b_den < rhs * P.b_num) {
    S.dir = DIR_PUSH;
    S.switches++;
  }
}

__device__ __forceinline__ void trace_iter(const St& S, const BfsParams& P, const BfsJob& J) {
  if (blockIdx.x == 0 && threadIdx.x == 0 && J_stats(P, J) && S.k < FG_TRACE_MAX) {
    J_stats(P, J)->dir[S.k] = (int8_t)S.dir;
    J_stats(P, J)->frontier[S.k] = S.qlen;
  }
}

__device__ __forceinline__ void trace_insp(int32_t k, int64_t insp, const BfsParams& P,
                                           const BfsJob& J) {
  if (blockIdx.x == 0 && threadIdx.x == 0 && J_stats(P, J) && k < FG_TRACE_MAX) {
    J_stats(P, J)->inspected[k] = insp;
    J_stats(P, J)->t_end[k] = (int64_t)wall_clock64();
  }
}

// Filter step for up to four edges per lane, all in flight together: plain
// visited pre-check of the four targets, then the test-and-sets of the
// candidates, then depth / parent of the winners.  v[r] must be a vertex id
// even where ok[r] is false.
__device__ __forceinline__ void visit4(const BfsParams& P, const BfsJob& J, uint32_t* vis32, int32_t d,
                                       const int32_t (&v)[4], const int32_t (&pu)[4],
                                       const bool (&ok)[4], bool (&won)[4]) {
  const int lane = fg_lane();
  uint32_t w[4], old[4], excl[4];
  uint64_t tails[4];
  bool cand[4], lead[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) w[r] = vis32[v[r] >> 5];
  // Lanes of one round that test bits of the same visited word in a run of
  // adjacent lanes (a sorted adjacency list's consecutive entries) combine
  // them: the run's last lane sets all of the run's bits with one atomic,
  // and each lane reads its own bit's previous value from that atomic's
  // result.  A hub's list of consecutive small ids would otherwise send up
  // to 64 atomics to one word from one instruction.
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    cand[r] = ok[r] && !((w[r] >> (v[r] & 31)) & 1u);
    const int32_t key = cand[r] ? (v[r] >> 5) : ~lane;  // non-candidates: runs of their own
    const uint32_t bm = cand[r] ? 1u << (v[r] & 31) : 0u;
    const int32_t kp = __shfl_up(key, 1, FG_WAVE);
    const int32_t kn = __shfl_down(key, 1, FG_WAVE);
    const bool head = lane == 0 || kp != key;
    const bool tl = lane == FG_WAVE - 1 || kn != key;
    const uint64_t H = __ballot(head);
    tails[r] = __ballot(tl);
    const uint64_t upto = lane == FG_WAVE - 1 ? ~0ull : ((2ull << lane) - 1ull);
    const int32_t start = 63 - __builtin_clzll(H & upto);
    // segmented inclusive OR over the lanes of the run up to this one
    uint32_t x = bm;
#pragma unroll
    for (int dd = 1; dd < FG_WAVE; dd <<= 1) {
      const uint32_t y = __shfl_up(x, dd, FG_WAVE);
      if (lane - dd >= start) x |= y;
    }
    // the bits of the run's earlier lanes (a target listed twice in a run
    // is won by its first lane only)
    const uint32_t xp = __shfl_up(x, 1, FG_WAVE);
    excl[r] = lane > start ? xp : 0u;
    lead[r] = tl && cand[r];
  }
  // old is only set and read where lead[r]: no merge with a default value,
  // so the compiler need not wait inside each branch
#pragma unroll
  for (int r = 0; r < 4; ++r)
    if (lead[r]) old[r] = atomicOr(vis32 + (v[r] >> 5), excl[r] | (1u << (v[r] & 31)));
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int tail = lane + __builtin_ctzll(tails[r] >> lane);
    const uint32_t o = __shfl(lead[r] ? old[r] : 0u, tail, FG_WAVE);
    // bits set before the run's atomic, or claimed by an earlier lane of it
    won[r] = cand[r] && !(((o | excl[r]) >> (v[r] & 31)) & 1u);
    if (won[r]) {
      J_depth(P, J)[v[r]] = d;
      if (J_parent(P, J)) J_parent(P, J)[v[r]] = pu[r];
    }
  }
}

constexpr int STAGE = 512;   // per-wave LDS staging of discovered vertices
constexpr int DSTAGE = 64;   // per-wave LDS room of 16-byte entries (pull: set-aside list)

struct Lds {
  // LDS-queue mode: frontier share of this workgroup as (vertex, first edge,
  // end edge), double buffered
  int32_t lq_v[2][QCAP];
  int32_t lq_b[2][QCAP];
  int32_t lq_e[2][QCAP];
  int32_t lq_cnt[3];   // per level mod 3: entries appended
  int32_t lq_deg[3];   // ... their degree sum
  int32_t lq_big[3];   // ... an input vertex of degree > TPV was seen
  // Full-grid phases and LDS-queue episodes never overlap in a workgroup
  // (each ends behind a block barrier), so their staging shares LDS.
  union {
    struct {
      int32_t stage[PWAVES][STAGE];
      int4 dstage[PWAVES][DSTAGE];
      // per-wave scan-gather staging (push, full grid)
      int32_t w_sc[PWAVES][FG_WAVE];
      int32_t w_u[PWAVES][FG_WAVE];
      int32_t w_b[PWAVES][FG_WAVE];
      int32_t w_e[PWAVES][FG_WAVE];
      // per-wave pull batch: unvisited vertices of nonzero degree per
      // bitmap word, and the vertices found per word
      uint64_t pw_act[PWAVES][FG_WAVE];
      uint64_t pw_nb[PWAVES][FG_WAVE];
    };
    // LDS-queue mode: the head-table entry (first four neighbours) of each
    // queued vertex, loaded beside its offsets when it is discovered, so a
    // level of low-degree vertices starts from LDS instead of a dependent
    // load of the column array
    int4 lq_h[2][QCAP];
  };
  // block-level staging (small-frontier mode)
  int32_t b_sc[PB];
  int32_t b_u[PB];
  int32_t b_b[PB];
  int64_t red[PWAVES + 1];
  int32_t red32[PWAVES + 1];
  int32_t newcnt;
  int32_t flag;
  int32_t ackbad;  // workgroup 0: a hand-off acknowledgement wait failed
  int64_t bcast[20];
  int32_t tsum[6];
};

// The final flush of every wave's staged entries with one global atomic
// per workgroup: the waves' counts meet in LDS, thread 0 reserves the
// workgroup's total behind `*total`, and each wave stores its entries at
// its prefix.  (One atomic per wave put some 4096 same-address atomics on
// the counter at the end of every push level.)  Every thread of the
// workgroup must take part.
template <class T, int CAP>
__device__ __forceinline__ void block_flush(WaveStage<T, CAP>& st, ull* total, ull base, T* out,
                                            Lds& L) {
  const int lane = fg_lane();
  const int wid = threadIdx.x / FG_WAVE;
  __syncthreads();
  if (lane == 0) L.red32[wid] = st.cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t sum = 0;
    for (int w = 0; w < PWAVES; ++w) {
      const int32_t c = L.red32[w];
      L.red32[w] = sum;
      sum += c;
    }
    L.bcast[0] = sum ? (int64_t)atomicAdd(total, (ull)sum) : 0;
  }
  __syncthreads();
  const ull pos = (ull)L.bcast[0] + (ull)L.red32[wid] - base;
  // written through: read by other workgroups after the next barrier
  for (int i = lane; i < st.cnt; i += FG_WAVE) fg_st_shared(&out[pos + i], st.buf[i]);
  st.cnt = 0;
  __syncthreads();
}

// ---- push, full grid, phase A: each wave takes 64-entry chunks of the
// frontier (static stride).  Vertices below big_deg are expanded by a
// wave-level scan-gather; the others become CH-edge descriptors.
__device__ void push_phase_a(const BfsParams& P, const BfsJob& J, const St& S, Lds& L,
                             uint32_t nblocks) {
  const int lane = fg_lane();
  const int wid = threadIdx.x / FG_WAVE;
  const int32_t* Qin = P.q[S.qsel];
  int32_t* Qout = P.q[S.qsel ^ 1];
  uint32_t* vis32 = (uint32_t*)P.vis[S.cur];
  const int32_t d_new = S.k + 1;
  int32_t* sc = L.w_sc[wid];
  int32_t* su = L.w_u[wid];
  int32_t* sb = L.w_b[wid];
  CtrSlot& C = P.ctl->slot[S.k & 1];
  const Bases B = get_bases(S);
  WaveStage<int32_t, STAGE> st{L.stage[wid], 0};
  int32_t* se = L.w_e[wid];
  // work items are dealt wave-major over the workgroups (item i to
  // workgroup i mod G): a level with few items spreads them over as many
  // CUs instead of filling the first workgroups' waves
  const int64_t gw = (int64_t)wid * nblocks + blockIdx.x;
  const int64_t W = (int64_t)nblocks * PWAVES;
  int64_t insp = 0;
  for (int64_t base = gw * FG_WAVE; base < S.qlen; base += W * FG_WAVE) {
    const int64_t i = base + lane;
    int32_t u = 0, b = 0, deg = 0;
    if (i < S.qlen) {
      u = Qin[i];
      b = P.off[u];
      deg = P.off[u + 1] - b;
    }
    insp += deg;
    const bool big = deg >= P.big_deg;
    // descriptors of the high-degree lanes, written cooperatively
    const int32_t nd = big ? (deg + CH - 1) / CH : 0;
    const int32_t ndi = fg_wave_incl_scan(nd);
    const int32_t ND = __shfl(ndi, FG_WAVE - 1, FG_WAVE);
    if (ND > 0) {
      wave_lds_fence();
      sc[lane] = ndi - nd;
      su[lane] = u;
      sb[lane] = b;
      se[lane] = b + deg;
      wave_lds_fence();
      // one reservation for all of the wave's descriptors, then 64 written
      // per step (a wave holding an R-MAT source's hubs writes thousands)
      ull pos = 0;
      if (lane == 0) pos = atomicAdd(&C.desc.v, (ull)ND);
      pos = __shfl(pos, 0, FG_WAVE) - B.desc;
      for (int32_t t0 = 0; t0 < ND; t0 += FG_WAVE) {
        const int32_t t = t0 + lane;
        if (t < ND) {
          const int32_t j = upper_idx(sc, FG_WAVE, t);
          const int32_t first = sb[j] + (t - sc[j]) * CH;
          // written through: read by other workgroups after the barrier
          fg_st_shared(&P.desc[pos + t],
                       make_int4(su[j], first, first + CH < se[j] ? first + CH : se[j], 0));
        }
      }
    }
    // scan-gather of the low-degree lanes
    const int32_t d = big ? 0 : deg;
    const int32_t inc = fg_wave_incl_scan(d);
    const int32_t T = __shfl(inc, FG_WAVE - 1, FG_WAVE);
    if (T == 0) continue;
    wave_lds_fence();
    sc[lane] = inc - d;
    su[lane] = u;
    sb[lane] = b;
    wave_lds_fence();
    // four rounds of 64 edges per step, their loads and atomics overlapped
    for (int32_t t0 = 0; t0 < T; t0 += 4 * FG_WAVE) {
      int32_t v[4], pu[4];
      bool ok[4], won[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int32_t t = t0 + r * FG_WAVE + lane;
        ok[r] = t < T;
        const int32_t j = upper_idx(sc, FG_WAVE, ok[r] ? t : T - 1);
        pu[r] = su[j];
        v[r] = P.col[sb[j] + ((ok[r] ? t : T - 1) - sc[j])];
      }
      visit4(P, J, vis32, d_new, v, pu, ok, won);
#pragma unroll
      for (int r = 0; r < 4; ++r) st.push(won[r], v[r], &C.q.v, B.q, Qout);
    }
  }
  block_flush(st, &C.q.v, B.q, Qout, L);
  // per workgroup and level the sum is at most m < 2^31
  const int32_t tot = fg_block_sum<PB>((int32_t)insp, L.red32);
  if (threadIdx.x == 0 && tot) atomicAdd(&C.insp.v, (ull)tot);
}

// ---- push, full grid, phase B: waves take descriptors in turn; the CH
// edges of a descriptor are contiguous, so each round is one coalesced read
// of 64 column indices and no search is needed.
__device__ void push_phase_b(const BfsParams& P, const BfsJob& J, const St& S, int64_t ndesc, Lds& L,
                             uint32_t nblocks) {
  const int lane = fg_lane();
  const int wid = threadIdx.x / FG_WAVE;
  // work items are dealt wave-major over the workgroups (item i to
  // workgroup i mod G): a level with few items spreads them over as many
  // CUs instead of filling the first workgroups' waves
  const int64_t gw = (int64_t)wid * nblocks + blockIdx.x;
  const int64_t W = (int64_t)nblocks * PWAVES;
  int32_t* Qout = P.q[S.qsel ^ 1];
  uint32_t* vis32 = (uint32_t*)P.vis[S.cur];
  const int32_t d_new = S.k + 1;
  CtrSlot& C = P.ctl->slot[S.k & 1];
  const Bases B = get_bases(S);
  WaveStage<int32_t, STAGE> st{L.stage[wid], 0};
  // the next descriptor is loaded while the current one is processed
  int4 nd = gw < ndesc ? P.desc[gw] : make_int4(0, 0, 0, 0);
  for (int64_t i = gw; i < ndesc; i += W) {
    const int4 dsc = nd;
    if (i + W < ndesc) nd = P.desc[i + W];
    const int32_t u = dsc.x;
    const int32_t e1 = dsc.z;
    // the CH / 64 = 4 rounds of a descriptor with their loads and atomics
    // overlapped (indices past the chunk clamped to its last edge)
    static_assert(CH == 4 * FG_WAVE, "one visit4 per descriptor");
    int32_t v[4], pu[4];
    bool ok[4], won[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int32_t e = dsc.y + r * FG_WAVE + lane;
      ok[r] = e < e1;
      v[r] = P.col[ok[r] ? e : e1 - 1];
      pu[r] = u;
    }
    visit4(P, J, vis32, d_new, v, pu, ok, won);
#pragma unroll
    for (int r = 0; r < 4; ++r) st.push(won[r], v[r], &C.q.v, B.q, Qout);
  }
  block_flush(st, &C.q.v, B.q, Qout, L);
}

// ---- push, full grid, frontier of at most 64 vertices (the hubs an R-MAT
// source reaches first): every wave lists the frontier's CH-edge chunks
// itself (one lane per vertex, a wave scan of the chunk counts) and takes
// chunks gw, gw + W, ...; no descriptors in memory, one grid barrier.
__device__ void push_tiny(const BfsParams& P, const BfsJob& J, const St& S, Lds& L) {
  const int lane = fg_lane();
  const int wid = threadIdx.x / FG_WAVE;
  const int32_t* Qin = P.q[S.qsel];
  int32_t* Qout = P.q[S.qsel ^ 1];
  uint32_t* vis32 = (uint32_t*)P.vis[S.cur];
  const int32_t d_new = S.k + 1;
  int32_t* sc = L.w_sc[wid];
  int32_t* su = L.w_u[wid];
  int32_t* sb = L.w_b[wid];
  int32_t* se = L.w_e[wid];
  CtrSlot& C = P.ctl->slot[S.k & 1];
  const Bases B = get_bases(S);
  WaveStage<int32_t, STAGE> st{L.stage[wid], 0};
  int32_t u = 0, b = 0, deg = 0;
  if (lane < S.qlen) {
    u = Qin[lane];
    b = P.off[u];
    deg = P.off[u + 1] - b;
  }
  const int32_t nch = (deg + CH - 1) / CH;
  const int32_t incl = fg_wave_incl_scan(nch);
  const int32_t NC = __builtin_amdgcn_readlane(incl, FG_WAVE - 1);
  wave_lds_fence();
  sc[lane] = incl - nch;
  su[lane] = u;
  sb[lane] = b;
  se[lane] = b + deg;
  wave_lds_fence();
  // work items are dealt wave-major over the workgroups (item i to
  // workgroup i mod G): a level with few items spreads them over as many
  // CUs instead of filling the first workgroups' waves
  const int64_t gw = (int64_t)wid * fgb_n(P) + blockIdx.x;
  const int64_t W = (int64_t)fgb_n(P) * PWAVES;
  static_assert(CH == 4 * FG_WAVE, "one visit4 per chunk");
  for (int64_t c = gw; c < NC; c += W) {
    // the last vertex whose first chunk is at or before c (vertices without
    // chunks share their successor's start and are never picked)
    const int32_t j = upper_idx(sc, FG_WAVE, (int32_t)c);
    const int32_t e0 = sb[j] + ((int32_t)c - sc[j]) * CH;
    const int32_t e1 = e0 + CH < se[j] ? e0 + CH : se[j];
    int32_t v[4], pu[4];
    bool ok[4], won[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int32_t e = e0 + r * FG_WAVE + lane;
      ok[r] = e < e1;
      v[r] = P.col[ok[r] ? e : e1 - 1];
      pu[r] = su[j];
    }
    visit4(P, J, vis32, d_new, v, pu, ok, won);
#pragma unroll
    for (int r = 0; r < 4; ++r) st.push(won[r], v[r], &C.q.v, B.q, Qout);
  }
  block_flush(st, &C.q.v, B.q, Qout, L);
  // the frontier's degree sum, once
  const int32_t tot = fg_wave_sum(deg);
  if (blockIdx.x == 0 && threadIdx.x == 0 && tot) atomicAdd(&C.insp.v, (ull)tot);
}

// Position of the r-th set bit (r = 0 first) of x; x has more than r bits set.
__device__ __forceinline__ int nth_bit(uint64_t x, int r) {
  int pos = 0;
#pragma unroll
  for (int h = 32; h > 0; h >>= 1) {
    const int c = __popcll(x & ((1ull << h) - 1));
    if (r >= c) {
      r -= c;
      x >>= h;
      pos += h;
    }
  }
  return pos;
}

// Early-exit probe of up to four consecutive CSR entries [i0, min(i0+4, e))
// (needs i0 < e): all column loads, then all visited-word loads, in flight
// together.  The loads are unconditional (indices clamped to the last
// entry) so that no per-entry branch makes the compiler wait between them.
// Returns the offset of the first entry whose vertex is visited, or -1.
__device__ __forceinline__ int32_t probe4(const BfsParams& P, const uint64_t* Vin, int32_t i0,
                                          int32_t e, int32_t& pu) {
  int32_t u[4];
  uint64_t wv[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) u[j] = P.col[i0 + j < e ? i0 + j : e - 1];
#pragma unroll
  for (int j = 0; j < 4; ++j) wv[j] = Vin[u[j] >> 6];
  int32_t hit = -1;
#pragma unroll
  for (int j = 3; j >= 0; --j) {
    if (i0 + j < e && ((wv[j] >> (u[j] & 63)) & 1ull)) {
      hit = j;
      pu = u[j];
    }
  }
  return hit;
}

// ---- pull (backward) iteration, vertex-parallel with early exit
// (Sec. VI-A): an unvisited vertex scans its neighbours in CSR order and
// stops at the first one in the frontier.  For an unvisited v, a visited
// neighbour has depth exactly k, so the visited bitmap is the frontier
// test.  Each wave takes bitmap words with a static stride, 64 at a time:
// it loads the 64 words at once, lists their unvisited vertices of nonzero
// degree, and runs them two per lane and round, probing each vertex's first
// four entries from the head table.  Vertices with more entries and no hit
// among the first four are set aside in an LDS list and resumed together
// once the batch's rounds are done: lists of up to 16 entries four at a
// time, lane by lane, longer ones by the whole wave, 64 entries per step.
// (Resumed inside the rounds, the few such lanes held their whole wave for
// up to three more probe steps per round.)  Writes the next visited bitmap
// Vout = Vin | found (whole words, no atomics).
constexpr int PULL_DEFER = STAGE;  // set-aside vertices per wave

// The found vertex v (bit `bit` of batch word jw): depth, parent, next bit.
__device__ __forceinline__ void pull_found(const BfsParams& P, const BfsJob& J, uint64_t* nbw, int32_t v,
                                           int32_t pu, int32_t d_new, int32_t jw, int32_t bit) {
  J_depth(P, J)[v] = d_new;
  if (J_parent(P, J)) J_parent(P, J)[v] = pu;
  atomicOr((unsigned long long*)&nbw[jw], 1ull << bit);
}

// Resumes the set-aside vertices dv[0..cnt) (entries from the fifth on);
// dj holds jw << 6 | bit.  Every lane of the wave must take part.
__device__ void pull_resume(const BfsParams& P, const BfsJob& J, const uint64_t* Vin, uint64_t* nbw,
                            const int32_t* dv, const uint16_t* dj, int32_t cnt, int32_t d_new,
                            int32_t& insp, int32_t& ndeg, int32_t& nnew) {
  const int lane = fg_lane();
  for (int32_t a0 = 0; a0 < cnt; a0 += FG_WAVE) {
    const int32_t a = a0 + lane;
    const bool mine = a < cnt;
    int32_t v = 0, b = 0, e = 0, pu = -1, ins = 0;
    if (mine) {
      v = dv[a];
      b = P.off[v];
      e = P.off[v + 1];
    }
    bool found = false;
    // lists of up to 16 entries: four at a time, lane by lane
    bool shortl = mine && e - b <= 16;
    for (int32_t i0 = 4; i0 < 16 && __ballot(shortl); i0 += 4) {
      if (shortl) {
        if (b + i0 < e) {
          const int32_t h = probe4(P, Vin, b + i0, e, pu);
          if (h >= 0) {
            found = true;
            shortl = false;
            ins += h + 1;
          } else {
            ins += min(4, e - b - i0);
          }
        } else {
          shortl = false;
        }
      }
    }
    // longer lists: the whole wave scans one at a time
    uint64_t pend = __ballot(mine && e - b > 16);
    while (pend) {
      const int l = __builtin_ctzll(pend);
      pend &= pend - 1;
      const int32_t lb = __builtin_amdgcn_readlane(b, l) + 4;
      const int32_t le = __builtin_amdgcn_readlane(e, l);
      int32_t cnt2 = 0, hu = -1;
      for (int32_t i0 = lb; i0 < le; i0 += FG_WAVE) {
        const int32_t i = i0 + lane;
        int32_t u = 0;
        bool hb = false;
        if (i < le) {
          u = P.col[i];
          hb = (Vin[u >> 6] >> (u & 63)) & 1ull;
        }
        const uint64_t m = __ballot(hb);
        if (m) {
          const int f = __builtin_ctzll(m);
          cnt2 += f + 1;
          hu = __builtin_amdgcn_readlane(u, f);
          break;
        }
        cnt2 += min(FG_WAVE, le - i0);
      }
      if (lane == l) {
        ins += cnt2;
        if (hu >= 0) {
          found = true;
          pu = hu;
        }
      }
    }
    insp += ins;
    if (found) {
      const int32_t jb = dj[a];
      pull_found(P, J, nbw, v, pu, d_new, jb >> 6, jb & 63);
      ndeg += e - b;
      nnew++;
    }
  }
}

__device__ void pull_phase(const BfsParams& P, const BfsJob& J, const St& S, Lds& L) {
  const int lane = fg_lane();
  const int wid = threadIdx.x / FG_WAVE;
  const int64_t gw = (int64_t)blockIdx.x * PWAVES + wid;
  const int64_t W = (int64_t)fgb_n(P) * PWAVES;
  const uint64_t* Vin = P.vis[S.cur];
  uint64_t* Vout = P.vis[S.cur ^ 1];
  const int32_t d_new = S.k + 1;
  int32_t* sc = L.w_sc[wid];
  uint64_t* actw = L.pw_act[wid];
  uint64_t* nbw = L.pw_nb[wid];
  // the set-aside list lives in this wave's push staging (unused here)
  int32_t* dv = L.stage[wid];
  uint16_t* dj = (uint16_t*)L.dstage[wid];
  static_assert(sizeof(L.dstage[0]) >= PULL_DEFER * sizeof(uint16_t), "set-aside list fits");
  int32_t insp = 0, ndeg = 0, nnew = 0;
  for (int64_t t0 = 0; gw + t0 * W < P.nwords; t0 += FG_WAVE) {
    const int64_t wj = gw + (t0 + lane) * W;  // this lane's word of the batch
    uint64_t vis = 0, act = 0;
    if (wj < P.nwords) {
      vis = Vin[wj];
      act = P.nz[wj] & ~vis;
    }
    const int32_t c = __popcll(act);
    const int32_t incl = fg_wave_incl_scan(c);
    const int32_t tot = __builtin_amdgcn_readlane(incl, FG_WAVE - 1);
    sc[lane] = incl - c;
    actw[lane] = act;
    nbw[lane] = 0;
    wave_lds_fence();
    int32_t ndef = 0;
    // two candidates per lane and round: the offsets and head entries of
    // both, then the eight visited words of their first four neighbours,
    // are in flight together (lanes past the list take candidate 0 again,
    // a valid vertex, and discard the result)
    for (int32_t a0 = 0; a0 < tot; a0 += 2 * FG_WAVE) {
      if (ndef > PULL_DEFER - 2 * FG_WAVE) {
        // room for a whole round: resume what is set aside now
        pull_resume(P, J, Vin, nbw, dv, dj, ndef, d_new, insp, ndeg, nnew);
        wave_lds_fence();
        ndef = 0;
      }
      int32_t v[2], b[2], e[2], jw[2], bit[2];
      int4 hd[2];
      bool mine[2];
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2) {
        const int32_t a = a0 + s2 * FG_WAVE + lane;
        mine[s2] = a < tot;
        const int32_t ac = mine[s2] ? a : 0;
        jw[s2] = upper_idx(sc, FG_WAVE, ac);
        bit[s2] = nth_bit(actw[jw[s2]], ac - sc[jw[s2]]);
        v[s2] = (int32_t)((gw + (t0 + jw[s2]) * W) * 64 + bit[s2]);
      }
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2) {
        b[s2] = P.off[v[s2]];
        e[s2] = P.off[v[s2] + 1];
        hd[s2] = P.head[v[s2]];
      }
      uint64_t wv[2][4];
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2) {
        // a candidate has nonzero degree: its head entries are vertices
        wv[s2][0] = Vin[hd[s2].x >> 6];
        wv[s2][1] = Vin[hd[s2].y >> 6];
        wv[s2][2] = Vin[hd[s2].z >> 6];
        wv[s2][3] = Vin[hd[s2].w >> 6];
      }
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2) {
        const int32_t u[4] = {hd[s2].x, hd[s2].y, hd[s2].z, hd[s2].w};
        const int32_t dg = e[s2] - b[s2];
        int32_t h = -1, pu = -1;
#pragma unroll
        for (int j = 3; j >= 0; --j) {
          if (j < dg && ((wv[s2][j] >> (u[j] & 63)) & 1ull)) {
            h = j;
            pu = u[j];
          }
        }
        const bool found = mine[s2] && h >= 0;
        const bool defer = mine[s2] && h < 0 && dg > 4;
        insp += !mine[s2] ? 0 : (h >= 0 ? h + 1 : min(4, dg));
        if (found) {
          pull_found(P, J, nbw, v[s2], pu, d_new, jw[s2], bit[s2]);
          ndeg += dg;
          nnew++;
        }
        const uint64_t dm = __ballot(defer);
        if (defer) {
          const int32_t pos = ndef + fg_mbcnt(dm);
          dv[pos] = v[s2];
          dj[pos] = (uint16_t)((jw[s2] << 6) | bit[s2]);
        }
        ndef += __popcll(dm);
      }
    }
    wave_lds_fence();
    if (ndef > 0) pull_resume(P, J, Vin, nbw, dv, dj, ndef, d_new, insp, ndeg, nnew);
    wave_lds_fence();
    if (wj < P.nwords) fg_st_shared(&Vout[wj], vis | nbw[lane]);
  }
  const int32_t tot = fg_block_sum<PB>(insp, L.red32);
  const int32_t tdeg = fg_block_sum<PB>(ndeg, L.red32);
  const int32_t tn = fg_block_sum<PB>(nnew, L.red32);
  CtrSlot& C = P.ctl->slot[S.k & 1];
  if (threadIdx.x == 0) {
    if (tot) atomicAdd(&C.insp.v, (ull)tot);
    if (tdeg) atomicAdd(&C.deg.v, (ull)tdeg);
    if (tn) atomicAdd(&C.q.v, (ull)tn);
  }
}

// ---- backward -> forward switch: the new frontier is the set difference
// of the current and the previous visited bitmap, listed into Q[qsel].
__device__ void bitmap_diff_to_queue(const BfsParams& P, const St& S, Lds& L) {
  // each workgroup lists a contiguous range of bitmap words (a multiple of
  // 64 words, 64 per wave and step) and reserves its queue slots with one
  // atomic per step
  const int lane = fg_lane();
  const int wid = threadIdx.x / FG_WAVE;
  const uint64_t* Vnew = P.vis[S.cur];
  const uint64_t* Vold = P.vis[S.cur ^ 1];
  int32_t* Q = P.q[S.qsel];
  const int64_t per = ((P.nwords + fgb_n(P) - 1) / fgb_n(P) + FG_WAVE - 1) / FG_WAVE * FG_WAVE;
  const int64_t wb = (int64_t)blockIdx.x * per;
  const int64_t we = wb + per < P.nwords ? wb + per : P.nwords;
  for (int64_t c0 = wb; c0 < we; c0 += PWAVES * FG_WAVE) {
    const int64_t w = c0 + wid * FG_WAVE + lane;
    const uint64_t diff0 = w < we ? Vnew[w] & ~Vold[w] : 0ull;
    const int32_t c = __popcll(diff0);
    const int32_t inc = fg_wave_incl_scan(c);
    if (lane == FG_WAVE - 1) L.red32[wid] = inc;
    __syncthreads();
    int32_t before = 0, btot = 0;
#pragma unroll
    for (int i = 0; i < PWAVES; ++i) {
      const int32_t x = L.red32[i];
      before += i < wid ? x : 0;
      btot += x;
    }
    if (threadIdx.x == 0)
      L.bcast[0] = btot ? (int64_t)(atomicAdd(&P.ctl->aux.v, (ull)btot) - S.auxbase) : 0;
    __syncthreads();
    int64_t pos = L.bcast[0] + before + inc - c;
    uint64_t diff = diff0;
    while (diff) {
      const int bit = __builtin_ctzll(diff);
      diff &= diff - 1;
      fg_st_shared(&Q[pos++], (int32_t)(w * 64 + bit));
    }
    __syncthreads();
  }
}

// ---- LDS-queue mode: a team of T workgroups (T = 1 for the smallest
// frontiers) runs push levels back to back.  Each member keeps its share of
// the frontier in LDS as (vertex, first edge, end edge, head entry) and
// appends each vertex it discovers, with the offsets and head entry loaded
// once its visited test-and-set is won, to its next LDS queue: no global
// queue, no global output counter and no offset reloads.  A vertex of
// degree <= TPV is expanded by TPV adjacent lanes, one edge each, the
// neighbour taken from its head entry (no scan, no search, no column
// load); larger vertices go through a block scan-gather.  Per level the
// dependent memory chain is visited atomic -> winner's offsets and head
// entry, then one workgroup barrier, plus the exchange of the members'
// totals when T > 1.  A member whose LDS queue is full appends the
// overflow to the global queue, which ends the episode.  On exit the
// members write their LDS queues to the global queue (written through, so
// the team barrier needs no L2 write-back), and the other modes continue
// from Q[qsel] as usual.
struct TeamSync {
  uint32_t* arrive;
  uint32_t* abort_flag;
  uint32_t T;
  uint32_t count;

  // Without the L2 write-back, as fg_grid_sync::sync_acquire: for data the
  // members write with fg_st_shared or atomics.
  __device__ bool sync_acquire(int* s_flag) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
      count++;
      __hip_atomic_fetch_add(arrive, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      *s_flag = !fg_wait_geq(arrive, count * T, abort_flag, 1);
    }
    __syncthreads();
    return *s_flag == 0;
  }
};

// Bases of the global-queue counters, held by the members (identical in
// all of them).
struct TeamBases {
  ull ovf, solo_ovf;
  uint32_t levels;  // team level exchanges so far
};

// Level totals of a team, fast path: every member adds one word to the
// level's team word (arrival, flag, count, capped degree sum) and thread 0
// polls that word until all T members are in: one atomic and one polled
// address per level.  All are agent-scope atomics, so no cache write-back
// or invalidation is needed: within an episode the members share nothing
// but the visited bitmap, which is only touched by atomics.  The words
// rotate over three slots; workgroup 0 clears the slot of the next level
// (its last readers are done: they have all arrived at this level) and
// makes its own arrival wait for the clear, which every later arrival at
// that slot follows.  A member flags itself when its count exceeds `lim`.
// L.tsum: [0] discovered, [1] degree sum, [2] flagged members.
// Workgroup 0 clears the word of team level `level + 1` (issued early in
// the level; team_fast waits for it before arriving).
__device__ __forceinline__ ull team_clear_next(const BfsParams& P, uint32_t level) {
  if (blockIdx.x == 0 && threadIdx.x == 0)
    return __hip_atomic_exchange(&P.ctl->team_word[(level + 1) % 3].v, 0ull, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
  return 0;
}

__device__ bool team_fast(const BfsParams& P, Lds& L, uint32_t T, uint32_t level, int32_t bcnt,
                          int32_t bdeg, int32_t lim, ull cleared) {
  if (threadIdx.x == 0) {
    ull* w = &P.ctl->team_word[level % 3].v;
    const ull g = bdeg < TW_CAP ? (ull)bdeg : (ull)TW_CAP;
    const ull add = (1ull << TW_ARR) | ((ull)(bcnt > lim) << TW_FLAG) | ((ull)bcnt << TW_CNT) | g;
    // the exchange's old value is consumed before the arrival is issued
    asm volatile("" ::"v"(cleared) : "memory");
    __hip_atomic_fetch_add(w, add, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t* abort_flag = P.ctl->bar + FG_BAR_STRIDE;
    uint32_t spins = 0;
    int bad = 0;
    ull x;
    for (;;) {
      x = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if ((x >> TW_ARR) >= T) break;
      if ((++spins & 31u) == 0 &&
          __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        bad = 1;
        break;
      }
      if (spins > FG_SPIN_LIMIT) {
        __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        bad = 1;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    L.tsum[0] = (int32_t)((x >> TW_CNT) & ((1ull << (TW_FLAG - TW_CNT)) - 1));
    L.tsum[1] = (int32_t)(x & ((1ull << TW_CNT) - 1));
    L.tsum[2] = (int32_t)((x >> TW_FLAG) & ((1ull << (TW_ARR - TW_FLAG)) - 1));
    L.flag = bad;
  }
  __syncthreads();
  return L.flag == 0;
}

// Slow path, taken when the episode ends or a member flagged itself: wave 0
// reads every member's record (vertices discovered, exact degree sum; each
// word tagged with the level, re-read until current, since a record and
// the arrival are not ordered).  L.tsum: [2] members that overflowed their
// LDS queue, [3] overflow entries in all, [4] entries kept in LDS by the
// members before this one, [5] largest member count.
__device__ bool team_records(const BfsParams& P, Lds& L, uint32_t T, uint32_t seq, int odd) {
  const int tid = threadIdx.x;
  if (tid < FG_WAVE) {
    uint32_t* abort_flag = P.ctl->bar + FG_BAR_STRIDE;
    int32_t c = 0, bad = 0;
    if ((uint32_t)tid < T) {
      const ull* r = P.ctl->team_rec[odd][tid];
      uint32_t spins = 0;
      for (;;) {
        const ull a = __hip_atomic_load(r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((uint32_t)(a >> 32) == seq) {
          c = (int32_t)(uint32_t)a;
          break;
        }
        if (++spins > FG_SPIN_LIMIT) {
          __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          bad = 1;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    const int32_t keep = c < QCAP ? c : QCAP;
    const int32_t keep_incl = fg_wave_incl_scan(keep);
    const int32_t before = __builtin_amdgcn_readlane(keep_incl - keep, blockIdx.x);
    const int32_t tof = fg_wave_sum(c > QCAP ? 1 : 0);
    const int32_t tov = fg_wave_sum(c - keep);
    int32_t mx = c;
#pragma unroll
    for (int d = FG_WAVE / 2; d > 0; d >>= 1) {
      const int32_t y = __shfl_xor(mx, d, FG_WAVE);
      mx = y > mx ? y : mx;
    }
    bad = fg_wave_sum(bad);
    if (tid == 0) {
      L.tsum[2] = tof;
      L.tsum[3] = tov;
      L.tsum[4] = before;
      L.tsum[5] = mx;
      L.flag = bad;
    }
  }
  __syncthreads();
  return L.flag == 0;
}

// The head entry of a vertex just discovered from `u`, with u's slots set
// to -1: u is visited, so testing it again next level is wasted work.
__device__ __forceinline__ int4 blank_parent(int4 h, int32_t u) {
  h.x = h.x == u ? -1 : h.x;
  h.y = h.y == u ? -1 : h.y;
  h.z = h.z == u ? -1 : h.z;
  h.w = h.w == u ? -1 : h.w;
  return h;
}

// Reserves `w` consecutive slots per lane behind `*counter` (LDS) for the
// whole wave with one atomic; returns this lane's first slot.  Every lane of
// the wave must take part.
__device__ __forceinline__ int32_t wave_reserve(int32_t w, int32_t* counter) {
  const int32_t incl = fg_wave_incl_scan(w);
  const int32_t tot = __builtin_amdgcn_readlane(incl, FG_WAVE - 1);
  int32_t base = 0;
  if (tot) {
    if (fg_lane() == 0) base = atomicAdd(counter, tot);
    base = __builtin_amdgcn_readfirstlane(base);
  }
  return base + incl - w;
}

// Stores this lane's discovered vertex (if `won`) at slot `pos` of the next
// LDS queue; slots past QCAP go to the global queue, one atomic per wave.
// Every lane of the wave must take part.
__device__ __forceinline__ void wave_put(Lds& L, int nxt, bool won, int32_t pos, int32_t v,
                                         int32_t vb, int32_t ve, int4 vh, int32_t* Qo, ull* ovf,
                                         ull ovf_base) {
  const bool over = won && pos >= QCAP;
  if (won && !over) {
    L.lq_v[nxt][pos] = v;
    L.lq_b[nxt][pos] = vb;
    L.lq_e[nxt][pos] = ve;
    L.lq_h[nxt][pos] = vh;
  }
  const uint64_t om = __ballot(over);
  if (om) {
    ull base = 0;
    if (fg_lane() == 0) base = atomicAdd(ovf, (ull)__popcll(om));
    base = fg_uni(base);
    if (over) fg_st_shared(&Qo[base - ovf_base + fg_mbcnt(om)], v);
  }
}

template <int MODE>
__device__ bool lds_mode(const BfsParams& P, const BfsJob& J, St& S, Lds& L, uint32_t T, TeamSync& ts,
                         TeamBases& tb) {
  const int tid = threadIdx.x;
  const int lane = fg_lane();
  const bool solo = T == 1;
  ull* ovf = solo ? &P.ctl->solo_ovf.v : &P.ctl->team_ovf.v;
  ull ovf_base = solo ? tb.solo_ovf : tb.ovf;
  // LDS counters rotate over three slots: the level's input, its output,
  // and the one cleared for the next level (its last reader finished a
  // barrier ago, its next writer starts a barrier later)
  int cur = 0, ci = 0, ni = 1, ri = 2;
  bool load = true;
  for (;;) {
    const int32_t* Qg = P.q[S.qsel];
    int32_t* Qo = P.q[S.qsel ^ 1];
    if (load) {
      // my even slice of the global frontier -> LDS queue `cur`
      load = false;
      const int64_t lo = S.qlen * blockIdx.x / T, hi = S.qlen * (blockIdx.x + 1) / T;
      const int32_t cnt = (int32_t)(hi - lo);
      int32_t sd = 0;
      for (int32_t i = tid; i < cnt; i += PB) {
        const int32_t u = Qg[lo + i];
        const int32_t b = P.off[u], e = P.off[u + 1];
        const int4 h = P.head[u];
        L.lq_v[cur][i] = u;
        L.lq_b[cur][i] = b;
        L.lq_e[cur][i] = e;
        L.lq_h[cur][i] = h;
        sd += e - b;
      }
      if (tid == 0) {
        L.lq_cnt[ci] = cnt;
        L.lq_cnt[ni] = 0;
        L.lq_deg[ni] = 0;
        L.lq_big[ni] = 0;
      }
      if (S.qdeg < 0) {
        // a full-grid push does not add up the degrees of what it finds:
        // take the frontier's degree sum now and hand the level back if it
        // does not suit this mode
        int64_t qd = fg_block_sum<PB>(sd, L.red32);
        if (!solo) {
          if (!team_fast(P, L, T, tb.levels, cnt, (int32_t)qd, QCAP, team_clear_next(P, tb.levels)))
            return false;
          tb.levels++;
          qd = fg_uni(L.tsum[1]);
        }
        S.qdeg = qd;
        if (qd > LDS_MEAN_DEG * S.qlen || qd > (solo ? P.small_e : P.team_e)) return true;
      }
      __syncthreads();
    }
    const int nxt = cur ^ 1;
    const int32_t cnt = L.lq_cnt[ci];
    // issued now, so that it is done by the time this level's exchange
    // needs it
    const ull cleared = solo ? 0ull : team_clear_next(P, tb.levels);
    if (tid == 0) {
      L.lq_cnt[ri] = 0;
      L.lq_deg[ri] = 0;
      L.lq_big[ri] = 0;
    }
    uint32_t* vis32 = (uint32_t*)P.vis[S.cur];
    const int32_t d_new = S.k + 1;
    bool big = false;
    // vertices of degree <= TPV: TPV consecutive lanes per vertex, one edge
    // each, the neighbour taken from the vertex's head entry in LDS
    for (int32_t c0 = 0; c0 < cnt; c0 += PB / TPV) {
      const int32_t i = c0 + tid / TPV;
      const int32_t j = tid % TPV;
      int32_t u = 0, b = 0, d = 0;
      if (i < cnt) {
        u = L.lq_v[cur][i];
        b = L.lq_b[cur][i];
        d = L.lq_e[cur][i] - b;
      }
      big |= d > TPV;
      bool won = false;
      int32_t v = 0, vb = 0, ve = 0;
      int4 vh = make_int4(0, 0, 0, 0);
      if (d <= TPV && j < d) {
        v = ((const int32_t*)&L.lq_h[cur][i])[j];
        // -1: the slot of the vertex's discoverer (visited), skipped
        if (v >= 0) {
          // what the next level needs (offsets, head entry) is loaded
          // beside the test-and-set, so its latency hides behind the
          // atomic's instead of following it; losers drop it
          vb = P.off[v];
          ve = P.off[v + 1];
          vh = P.head[v];
          const uint32_t bit = 1u << (v & 31);
          won = !(atomicOr(&vis32[v >> 5], bit) & bit);
        }
      }
      if (won) {
        vh = blank_parent(vh, u);
        J_depth(P, J)[v] = d_new;
        if (J_parent(P, J)) J_parent(P, J)[v] = u;
      }
      const int32_t pos = wave_reserve(won ? 1 : 0, &L.lq_cnt[ni]);
      const int32_t wdeg = fg_wave_sum(won ? ve - vb : 0);
      if (lane == 0 && wdeg) atomicAdd(&L.lq_deg[ni], wdeg);
      wave_put(L, nxt, won, pos, v, vb, ve, vh, Qo, ovf, ovf_base);
    }
    if (big) L.lq_big[ni] = 1;
    __syncthreads();
    if (L.lq_big[ni]) {
      // vertices of degree > TPV: block scan-gather over their edges
      for (int32_t c0 = 0; c0 < cnt; c0 += PB) {
        const int32_t i = c0 + tid;
        int32_t u = 0, b = 0, d = 0;
        if (i < cnt) {
          u = L.lq_v[cur][i];
          b = L.lq_b[cur][i];
          d = L.lq_e[cur][i] - b;
        }
        if (d <= TPV) d = 0;
        int32_t Tn = 0;
        const int32_t ex = fg_block_excl_scan<PB>(d, L.red32, &Tn);
        L.b_sc[tid] = ex;
        L.b_u[tid] = u;
        L.b_b[tid] = b;
        __syncthreads();
        const int32_t nc = cnt - c0 < PB ? cnt - c0 : PB;
        for (int32_t t0 = 0; t0 < Tn; t0 += PB) {
          const int32_t t = t0 + tid;
          bool won = false;
          int32_t v = 0, vb = 0, ve = 0, pu = 0;
          int4 vh = make_int4(0, 0, 0, 0);
          if (t < Tn) {
            const int32_t j = upper_idx(L.b_sc, nc, t);
            pu = L.b_u[j];
            v = P.col[L.b_b[j] + (t - L.b_sc[j])];
            const uint32_t bit = 1u << (v & 31);
            won = !(atomicOr(&vis32[v >> 5], bit) & bit);
          }
          if (won) {
            vb = P.off[v];
            ve = P.off[v + 1];
            vh = blank_parent(P.head[v], pu);
            J_depth(P, J)[v] = d_new;
            if (J_parent(P, J)) J_parent(P, J)[v] = pu;
          }
          const int32_t pos = wave_reserve(won ? 1 : 0, &L.lq_cnt[ni]);
          const int32_t wdeg = fg_wave_sum(won ? ve - vb : 0);
          if (lane == 0 && wdeg) atomicAdd(&L.lq_deg[ni], wdeg);
          wave_put(L, nxt, won, pos, v, vb, ve, vh, Qo, ovf, ovf_base);
        }
        __syncthreads();
      }
    }
    const int32_t bcnt = L.lq_cnt[ni];
    const int32_t bdeg = L.lq_deg[ni];
    int64_t nq, nqdeg, nflag;
    if (solo) {
      nq = bcnt;
      nqdeg = bdeg;
      nflag = bcnt > QCAP;
    } else {
      if (tid == 0) {
        // the record behind the word, read only on the slow path
        ull* r = P.ctl->team_rec[S.k & 1][blockIdx.x];
        const ull tag = (ull)((uint32_t)S.k + 1u) << 32;
        __hip_atomic_store(r, tag | (uint32_t)bcnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      const int64_t lim = (5 * S.qlen / T + 64) / 4;
      if (!team_fast(P, L, T, tb.levels, bcnt, bdeg, (int32_t)(lim < QCAP ? lim : QCAP), cleared))
        return false;
      tb.levels++;
      nq = fg_uni(L.tsum[0]);
      nqdeg = fg_uni(L.tsum[1]);
      nflag = fg_uni(L.tsum[2]);
    }
    // a push level reads every CSR entry of its frontier: the degree sum
    trace_insp(S.k, S.qdeg, P, J);
    S.insp_sum += S.qdeg;
    S.k++;
    S.qlen = nq;
    S.qdeg = nqdeg;
    S.p += nq;
    decide<MODE>(S, P);
    trace_iter(S, P, J);
    bool stay = nq > 0 && S.dir == DIR_PUSH && nqdeg <= LDS_MEAN_DEG * nq &&
                (solo ? (nq <= P.small_q && nqdeg <= P.small_e)
                      : (nqdeg <= P.team_e && !(nq <= P.small_q && nqdeg <= P.small_e)));
    int64_t nover = bcnt > QCAP ? bcnt - QCAP : 0, before = 0;
    bool rebalance = false;
    if (solo) {
      stay = stay && nflag == 0;
    } else if (!stay || nflag) {
      if (!team_records(P, L, T, (uint32_t)S.k, (S.k - 1) & 1)) return false;
      nover = fg_uni(L.tsum[3]);
      before = fg_uni(L.tsum[4]);
      stay = stay && fg_uni(L.tsum[2]) == 0;
      // the frontier grows at its ends: even out the members' shares when
      // the largest is more than 1.25 times the mean (+16)
      rebalance = stay && 4 * fg_uni(L.tsum[5]) * (int64_t)T > 5 * nq + 64 * (int64_t)T;
    }
    if (!stay || rebalance) {
      // global queue: the overflow entries, then every member's LDS queue
      // in member order
      const int32_t nloc = bcnt < QCAP ? bcnt : QCAP;
      int32_t* dst = Qo + nover + before;
      for (int32_t i = tid; i < nloc; i += PB) fg_st_shared(&dst[i], L.lq_v[nxt][i]);
      ovf_base += (ull)nover;
      if (solo) {
        tb.solo_ovf = ovf_base;
        __syncthreads();
      } else {
        tb.ovf = ovf_base;
        if (!ts.sync_acquire(&L.flag)) return false;
      }
      S.qsel ^= 1;
      if (!stay) return true;
      load = true;
    }
    cur = nxt;
    const int t3 = ci;
    ci = ni;
    ni = ri;
    ri = t3;
  }
}

// MODE is FG_MODE_DO or FG_MODE_PUSH (one kernel per mode).
template <int MODE, bool MULTI>
__device__ __forceinline__ void bfs_persistent_run(const BfsParams& P, Lds& L) {
  fg_grid_sync gs{P.ctl->bar, fgb_n(P), 0u};
  bool ok = true;
  // one traversal, or (MULTI, a build of its own: the loop around the
  // traversal raises the register pressure) P.nsrc traversals in turn
  const int32_t njobs = MULTI ? P.nsrc : 1;
  // queued behind an asynchronous traversal: run only if that one gave up
  if (P.async_fallback &&
      __hip_atomic_load(&P.ctl->as_state, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
    return;
  // shared outputs (fg_bfs_many, out_stride 0): once one traversal of this
  // launch has completed, the outputs hold -1 exactly outside its visited
  // set (kept in P.reached), so the next traversal writes only what it
  // reaches and afterwards resets the vertices the previous one reached and
  // it did not, instead of filling 8n bytes first
  bool have_prev = false;
  for (int32_t job = 0; job < njobs && ok; ++job) {
  BfsJob J{job, P.src};
  if (MULTI) {
    if (job > 0) {
      // every workgroup has left the previous traversal: the workgroups
      // clear the control block for the next one, a share each, all but the
      // grid barrier (in use; its counters are monotone); the init barrier
      // below publishes the clear
      if (!gs.sync(&L.flag)) {
        ok = false;
        break;
      }
      {
        uint32_t* w = (uint32_t*)P.ctl;
        for (int i = FG_BAR_WORDS + (int)(blockIdx.x * PB + threadIdx.x); i < (int)(sizeof(BfsCtl) / 4);
             i += (int)(fgb_n(P) * PB))
          w[i] = 0u;
      }
    }
    J.src = P.srcs[job];
    if (J.src < 0 || J.src >= P.n) {
      // every workgroup reads the same entry and skips the traversal
      if (blockIdx.x == 0 && threadIdx.x == 0 && J_stats(P, J)) {
        fg_run_stats* st = J_stats(P, J);
        st->status = FG_EINVAL;
        st->iterations = 0;
        st->reached = 0;
        st->edges_inspected = 0;
      }
      continue;
    }
  }
  St S = {};
  S.dir = DIR_PUSH;
  S.prevdir = DIR_PUSH;
  S.qlen = 1;
  S.p = 1;
  uint32_t sm_seen = 0;
  uint32_t ack_need = 0;  // workgroup 0: acknowledgements of the hand-backs so far
  TeamSync ts{&P.ctl->team_arrive, P.ctl->bar + FG_BAR_STRIDE, (uint32_t)P.team, 0u};
  TeamBases tb = {};
  const bool shared_out = MULTI && P.out_stride == 0;
  const bool incremental = shared_out && have_prev;
  // a1: depth = parent = -1 except at the source, visited = {src}, Q = {src}
  {
    const int64_t tid = (int64_t)blockIdx.x * PB + threadIdx.x;
    const int64_t nth = (int64_t)fgb_n(P) * PB;
    const int32_t src = J.src;
    if (blockIdx.x == 0 && J_stats(P, J)) {
      uint32_t* sw = (uint32_t*)J_stats(P, J);
      for (int i = threadIdx.x; i < (int)(sizeof(fg_run_stats) / 4); i += PB) sw[i] = 0u;
    }
    const bool vec = !incremental && ((((uintptr_t)J_depth(P, J)) | ((uintptr_t)(J_parent(P, J) ? J_parent(P, J) : J_depth(P, J)))) & 15) == 0;
    if (vec) {
      const int64_t n4 = P.n / 4;
      int4* d4 = (int4*)J_depth(P, J);
      int4* p4 = (int4*)J_parent(P, J);
      for (int64_t i = tid; i < n4; i += nth) {
        const bool hit = (src >> 2) == i;
        const int r = src & 3;
        const int4 d = make_int4(hit && r == 0 ? 0 : -1, hit && r == 1 ? 0 : -1,
                                 hit && r == 2 ? 0 : -1, hit && r == 3 ? 0 : -1);
        const int4 pp = make_int4(hit && r == 0 ? src : -1, hit && r == 1 ? src : -1,
                                  hit && r == 2 ? src : -1, hit && r == 3 ? src : -1);
        d4[i] = d;
        if (J_parent(P, J)) p4[i] = pp;
      }
      for (int64_t i = n4 * 4 + tid; i < P.n; i += nth) {
        J_depth(P, J)[i] = i == src ? 0 : -1;
        if (J_parent(P, J)) J_parent(P, J)[i] = i == src ? src : -1;
      }
    } else if (!incremental) {
      for (int64_t i = tid; i < P.n; i += nth) {
        J_depth(P, J)[i] = i == src ? 0 : -1;
        if (J_parent(P, J)) J_parent(P, J)[i] = i == src ? src : -1;
      }
    } else if (tid == 0) {
      J_depth(P, J)[src] = 0;
      if (J_parent(P, J)) J_parent(P, J)[src] = src;
    }
    uint64_t* v0 = P.vis[0];
    for (int64_t w = tid; w < P.nwords; w += nth)
      v0[w] = (w == (src >> 6)) ? (1ull << (src & 63)) : 0ull;
    if (tid == 0) P.q[0][0] = src;
    if (!gs.sync(&L.flag)) ok = false;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && J_stats(P, J)) {
    J_stats(P, J)->t_start = (int64_t)wall_clock64();
    J_stats(P, J)->clock_khz = P.clock_khz;
  }
  S.qdeg = fg_uni((int32_t)(P.off[J.src + 1] - P.off[J.src]));
  trace_iter(S, P, J);
  while (ok && S.qlen > 0) {
    // backward -> forward: list the last pull's discoveries first
    if (MODE == FG_MODE_DO && S.dir == DIR_PUSH && S.prevdir == DIR_PULL) {
      bitmap_diff_to_queue(P, S, L);
      if (!(ok = gs.sync_acquire(&L.flag))) break;
      S.auxbase = fg_atomic_load_u64(&P.ctl->aux.v);
      S.prevdir = DIR_PUSH;
    }
    // qdeg < 0: not known after a full-grid push; the LDS modes take it
    // on entry and hand the level back when it does not fit
    const bool qdu = S.qdeg < 0;
    const bool lds_ok = S.dir == DIR_PUSH && (qdu || S.qdeg <= LDS_MEAN_DEG * S.qlen);
    const bool small_ep = lds_ok && S.qlen <= P.small_q && (qdu || S.qdeg <= P.small_e);
    const bool team_ep = !small_ep && lds_ok && P.team > 1 && (qdu || S.qdeg <= P.team_e) &&
                         S.qlen <= (int64_t)QCAP * P.team / 2;
    if (small_ep || team_ep) {
      sm_seen++;
      const bool member = small_ep ? blockIdx.x == 0 : blockIdx.x < (uint32_t)P.team;
      if (member) {
        if (!lds_mode<MODE>(P, J, S, L, small_ep ? 1u : (uint32_t)P.team, ts, tb)) ok = false;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
          BfsCtl* c = P.ctl;
          // every waiter of the previous hand-back has read it (on a
          // timeout the abort flag is set and every wait ends)
          L.ackbad = !fg_wait_geq(&c->sm_ack, ack_need, c->bar + FG_BAR_STRIDE, 1);
          // a failed wait has set the abort flag: publish nothing (a slow
          // waiter may still be reading the previous hand-off); the waiters
          // see the flag and leave
          if (!L.ackbad) {
            c->pub_k = S.k;
            c->pub_dir = S.dir;
            c->pub_prevdir = S.prevdir;
            c->pub_switched = S.switched;
            c->pub_qsel = S.qsel;
            c->pub_qlen = S.qlen;
            c->pub_qdeg = S.qdeg;
            c->pub_p = S.p;
            c->pub_insp_sum = S.insp_sum;
            c->pub_switches = S.switches;
            c->pub_b[0] = S.b0q;
            c->pub_b[1] = S.b0desc;
            c->pub_b[2] = S.b0insp;
            c->pub_b[3] = S.b0deg;
            c->pub_b[4] = S.b1q;
            c->pub_b[5] = S.b1desc;
            c->pub_b[6] = S.b1insp;
            c->pub_b[7] = S.b1deg;
            __hip_atomic_fetch_add(&c->sm_signal, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            ack_need += fgb_n(P) - (small_ep ? 1u : (uint32_t)P.team);
          }
        }
        __syncthreads();
        if (!ok || (blockIdx.x == 0 && L.ackbad)) {
          ok = false;
          break;
        }
      } else {
        if (threadIdx.x == 0) {
          const int bad = !fg_wait_geq(&P.ctl->sm_signal, sm_seen, P.ctl->bar + FG_BAR_STRIDE, 4096);
          L.flag = bad;
          if (!bad) {
            const BfsCtl* c = P.ctl;
            L.bcast[0] = c->pub_k;
            L.bcast[1] = c->pub_dir;
            L.bcast[2] = c->pub_prevdir;
            L.bcast[3] = c->pub_switched;
            L.bcast[4] = c->pub_qsel;
            L.bcast[5] = c->pub_qdeg;
            L.bcast[6] = c->pub_qlen;
            L.bcast[7] = c->pub_p;
            L.bcast[8] = c->pub_insp_sum;
            L.bcast[9] = c->pub_switches;
            for (int i = 0; i < 8; ++i) L.bcast[10 + i] = (int64_t)c->pub_b[i];
            fg_handoff_ack(&P.ctl->sm_ack);
          }
        }
        __syncthreads();
        if (L.flag) {
          ok = false;
          break;
        }
        S.k = fg_uni((int32_t)L.bcast[0]);
        S.dir = fg_uni((int32_t)L.bcast[1]);
        S.prevdir = fg_uni((int32_t)L.bcast[2]);
        S.switched = fg_uni((int32_t)L.bcast[3]);
        S.qsel = fg_uni((int32_t)L.bcast[4]);
        S.qdeg = fg_uni(L.bcast[5]);
        S.qlen = fg_uni(L.bcast[6]);
        S.p = fg_uni(L.bcast[7]);
        S.insp_sum = fg_uni(L.bcast[8]);
        S.switches = fg_uni((int32_t)L.bcast[9]);
        S.b0q = fg_uni((ull)L.bcast[10]);
        S.b0desc = fg_uni((ull)L.bcast[11]);
        S.b0insp = fg_uni((ull)L.bcast[12]);
        S.b0deg = fg_uni((ull)L.bcast[13]);
        S.b1q = fg_uni((ull)L.bcast[14]);
        S.b1desc = fg_uni((ull)L.bcast[15]);
        S.b1insp = fg_uni((ull)L.bcast[16]);
        S.b1deg = fg_uni((ull)L.bcast[17]);
        __syncthreads();
      }
      continue;
    }
    CtrSlot& C = P.ctl->slot[S.k & 1];
    Bases B = get_bases(S);
    if ((MODE != FG_MODE_DO || S.dir == DIR_PUSH) && S.qlen <= FG_WAVE) {
      push_tiny(P, J, S, L);
      if (!(ok = gs.sync_acquire(&L.flag))) break;
      S.qsel ^= 1;
    } else if (MODE != FG_MODE_DO || S.dir == DIR_PUSH) {
      push_phase_a(P, J, S, L, fgb_n(P));
      if (!(ok = gs.sync_acquire(&L.flag))) break;
      const ull dt = fg_atomic_load_u64(&C.desc.v);
      const int64_t ndesc = (int64_t)(dt - B.desc);
      if (ndesc > 0) {
        push_phase_b(P, J, S, ndesc, L, fgb_n(P));
        if (!(ok = gs.sync_acquire(&L.flag))) break;
      }
      B.desc = dt;
      S.qsel ^= 1;
    } else {
      pull_phase(P, J, S, L);
      if (!(ok = gs.sync_acquire(&L.flag))) break;
      S.cur ^= 1;
    }
    const ull qt = fg_atomic_load_u64(&C.q.v);
    const ull it = fg_atomic_load_u64(&C.insp.v);
    const ull gt = fg_atomic_load_u64(&C.deg.v);
    const int64_t nq = (int64_t)(qt - B.q);
    const int64_t insp = (int64_t)(it - B.insp);
    B.q = qt;
    B.insp = it;
    // only a pull adds up the degrees of what it finds
    S.qdeg = S.dir == DIR_PULL ? (int64_t)(gt - B.deg) : -1;
    B.deg = gt;
    set_bases(S, B);
    trace_insp(S.k, insp, P, J);
    S.insp_sum += insp;
    S.k++;
    S.qlen = nq;
    S.p += nq;
    decide<MODE>(S, P);
    trace_iter(S, P, J);
  }
  if (shared_out && ok) {
    // every test-and-set of the traversal has completed (the last level's
    // grid barrier or team word); one agent-scope acquire per workgroup
    // drops stale bitmap lines from this CU's and XCD's caches before the
    // final bitmap is read with plain loads
    __syncthreads();
    if (threadIdx.x == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    __syncthreads();
    const uint64_t* fin = P.vis[S.cur];
    const int64_t tid = (int64_t)blockIdx.x * PB + threadIdx.x;
    const int64_t nth = (int64_t)fgb_n(P) * PB;
    for (int64_t w = tid; w < P.nwords; w += nth) {
      const uint64_t now = fin[w];
      if (incremental) {
        // reached by the previous traversal, not by this one: back to -1
        uint64_t stale = P.reached[w] & ~now;
        while (stale) {
          const int64_t v = w * 64 + __builtin_ctzll(stale);
          stale &= stale - 1;
          J_depth(P, J)[v] = -1;
          if (J_parent(P, J)) J_parent(P, J)[v] = -1;
        }
      }
      // read by this same thread after the next traversal
      P.reached[w] = now;
    }
    have_prev = true;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && J_stats(P, J)) {
    fg_run_stats* st = J_stats(P, J);
    // a wait that failed in any workgroup has set the abort flag
    const uint32_t aborted = __hip_atomic_load(P.ctl->bar + FG_BAR_STRIDE, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
    st->status = (ok && !aborted) ? FG_OK : FG_EDEVICE;
    st->iterations = S.k;
    st->reached = S.p;
    st->edges_inspected = S.insp_sum;
    st->direction_switches = S.switches;
    st->grid_blocks = (int32_t)fgb_n(P);
  }
  }  // jobs
  // the last workgroup out clears the control block for the next launch
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t done = __hip_atomic_fetch_add(&P.ctl->exit_count, 1u, __ATOMIC_ACQ_REL,
                                                 __HIP_MEMORY_SCOPE_AGENT);
    L.flag = done == fgb_n(P) - 1;
  }
  __syncthreads();
  if (L.flag) {
    uint32_t* w = (uint32_t*)P.ctl;
    for (int i = threadIdx.x; i < (int)(sizeof(BfsCtl) / 4); i += PB) w[i] = 0u;
  }
}

template <int MODE, bool MULTI>
__global__ __launch_bounds__(PB) void bfs_persistent(BfsParams P) {
  __shared__ Lds L;
  bfs_persistent_run<MODE, MULTI>(P, L);
}

// ---- asynchronous push mode (high-diameter graphs) ----------------------
//
// A team of T workgroups (the whole launch) runs K push levels between two
// synchronisations instead of one: each member expands its own LDS queue
// level after level and keeps what it discovers, without waiting for the
// others.  Members run at different speeds, so a vertex may first be
// reached over a longer path than its shortest; the visited test-and-set is
// therefore replaced by a 64-bit atomicMin on a key (depth << 32 | parent)
// per vertex, and a vertex joins the discoverer's next queue whenever its
// depth decreases (label correcting: the queues empty only when every key
// holds its shortest depth).  A decrease is won by exactly one relaxation,
// so each improvement queues the vertex once; equal depths from a smaller
// parent only lower the key.  At the end every key holds the BFS depth and
// the smallest-id neighbour one level closer to the source (a valid
// parent).  After K levels the members exchange queue lengths, stop when
// all are empty, and otherwise even out their queues through global memory.
// On grids and road-like graphs the members' regions advance as one front,
// so corrections are rare and K - 1 of every K level barriers disappear.
// If a member's queue overflows its LDS room, the traversal stops and the
// level-synchronous kernel launched behind it runs instead.

constexpr int AQ = QCAP;  // LDS queue entries per member

struct AsLds {
  int32_t qv[2][AQ];
  int32_t qb[2][AQ];
  int32_t qe[2][AQ];
  int4 qh[2][AQ];
  int32_t cnt[2];
  // by level parity: an append of the level did not fit; a vertex of degree
  // > TPV is in the level's queue
  int32_t ovf[2];
  int32_t big[2];
  int32_t flag;
  int32_t tot;
  int32_t pre;
  int32_t stop;
  int32_t b_sc[PB];
  int32_t b_u[PB];
  int32_t b_b[PB];
  int32_t red32[PWAVES + 1];
  int64_t red64[PWAVES + 1];
};

// Relaxation of v from u at depth d1 (= depth(u) + 1): true if it lowered
// v's depth (then the caller queues v).
__device__ __forceinline__ bool as_relax(ull* key, int32_t v, int32_t u, int32_t d1) {
  const ull kn = ((ull)(uint32_t)d1 << 32) | (uint32_t)u;
  const ull old = atomicMin(&key[v], kn);
  return (uint32_t)(old >> 32) > (uint32_t)d1;
}

// Queues the winners of a relaxation round in the next LDS queue (room
// permitting; an overflow, flagged in L.ovf[par], stops the traversal).
// Every lane must take part.
__device__ __forceinline__ void as_put(AsLds& L, int nxt, int par, bool won, int32_t v,
                                      int32_t vb, int32_t ve, int4 vh) {
  const int32_t pos = wave_reserve(won ? 1 : 0, &L.cnt[nxt]);
  if (won) {
    if (pos < AQ) {
      L.qv[nxt][pos] = v;
      L.qb[nxt][pos] = vb;
      L.qe[nxt][pos] = ve;
      L.qh[nxt][pos] = vh;
    } else {
      L.ovf[par] = 1;
    }
  }
}

__device__ __forceinline__ void bfs_async_run(const BfsParams& P, AsLds& L) {
  const int tid = threadIdx.x;
  const int lane = fg_lane();
  const uint32_t T = fgb_n(P);
  BfsCtl* C = P.ctl;
  uint32_t* abort_flag = C->bar + FG_BAR_STRIDE;
  TeamSync ts{&C->as_arrive, abort_flag, T, 0u};
  ull* key = (ull*)P.desc;  // the key array lives in the descriptor region
  int32_t* G = P.q[0];      // exchange buffer
  const int32_t K = P.async_k;
  int64_t insp = 0;
  if (tid == 0) {
    L.cnt[0] = as_member(P) == 0 ? 1 : 0;
    L.cnt[1] = 0;
    L.ovf[0] = L.ovf[1] = 0;
    L.big[0] = L.big[1] = 0;
    L.stop = 0;
    if (as_member(P) == 0) {
      L.qv[0][0] = P.src;
      L.qb[0][0] = P.off[P.src];
      L.qe[0][0] = P.off[P.src + 1];
      L.qh[0][0] = P.head[P.src];
    }
  }
  __syncthreads();
  int cur = 0;
  int32_t base = 0;  // depth of the entries of queue `cur` at a super-step start
  bool overflow = false;
  bool ok = true;
  // every super-step advances the queued depths by K, and no shortest
  // depth exceeds n - 1: past this many the team gives up (the
  // level-synchronous kernel behind it then answers)
  const uint32_t max_steps = (uint32_t)(P.n / K) + 2;
  for (uint32_t step = 0; ok; ++step) {
    if (step > max_steps) {
      if (as_member(P) == 0 && tid == 0)
        __hip_atomic_store(&C->as_state, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
    for (int32_t t = 0; t < K; ++t) {
      const int nxt = cur ^ 1;
      const int32_t cnt = L.cnt[cur] < AQ ? L.cnt[cur] : AQ;
      const int32_t d1 = base + t + 1;
      // the next queue's counter and this level's flags were cleared in the
      // previous level, after every thread had read what they held (see
      // below): no barriers at the start of a level
      const int par = (base + t) & 1;
      // vertices of degree <= TPV: TPV lanes each, neighbours from the head
      // entry in LDS (the discoverer's slot blanked)
      bool big = false;
      for (int32_t c0 = 0; c0 < cnt; c0 += PB / TPV) {
        const int32_t i = c0 + tid / TPV;
        const int32_t j = tid % TPV;
        int32_t u = 0, b = 0, d = 0;
        if (i < cnt) {
          u = L.qv[cur][i];
          b = L.qb[cur][i];
          d = L.qe[cur][i] - b;
        }
        big |= d > TPV;
        bool won = false;
        int32_t v = 0, vb = 0, ve = 0;
        int4 vh = make_int4(0, 0, 0, 0);
        if (d <= TPV && j < d) {
          v = ((const int32_t*)&L.qh[cur][i])[j];
          if (v >= 0) {
            vb = P.off[v];
            ve = P.off[v + 1];
            vh = P.head[v];
            won = as_relax(key, v, u, d1);
            insp++;
          }
        }
        if (won) vh = blank_parent(vh, u);
        as_put(L, nxt, par, won, v, vb, ve, vh);
      }
      if (big) L.big[par] = 1;
      __syncthreads();
      if (tid == 0) {
        // every thread has read this level's input count (at the start) and
        // the flags of the previous level (behind the last barrier)
        L.cnt[cur] = 0;
        L.ovf[par ^ 1] = 0;
        L.big[par ^ 1] = 0;
      }
      if (L.big[par]) {
        // vertices of degree > TPV: block scan-gather over their rows
        for (int32_t c0 = 0; c0 < cnt; c0 += PB) {
          const int32_t i = c0 + tid;
          int32_t u = 0, b = 0, d = 0;
          if (i < cnt) {
            u = L.qv[cur][i];
            b = L.qb[cur][i];
            d = L.qe[cur][i] - b;
          }
          if (d <= TPV) d = 0;
          int32_t Tn = 0;
          const int32_t ex = fg_block_excl_scan<PB>(d, L.red32, &Tn);
          L.b_sc[tid] = ex;
          L.b_u[tid] = u;
          L.b_b[tid] = b;
          __syncthreads();
          const int32_t nc = cnt - c0 < PB ? cnt - c0 : PB;
          for (int32_t t0 = 0; t0 < Tn; t0 += PB) {
            const int32_t tt = t0 + tid;
            bool won = false;
            int32_t v = 0, vb = 0, ve = 0, pu = 0;
            int4 vh = make_int4(0, 0, 0, 0);
            if (tt < Tn) {
              const int32_t jj = upper_idx(L.b_sc, nc, tt);
              pu = L.b_u[jj];
              v = P.col[L.b_b[jj] + (tt - L.b_sc[jj])];
              vb = P.off[v];
              ve = P.off[v + 1];
              vh = P.head[v];
              won = as_relax(key, v, pu, d1);
              insp++;
            }
            if (won) vh = blank_parent(vh, pu);
            as_put(L, nxt, par, won, v, vb, ve, vh);
          }
          __syncthreads();
        }
      }
      __syncthreads();
      cur = nxt;
      // every append of this level is behind that barrier, and the next
      // level flags the other slot: every thread sees the same value
      if (L.ovf[par]) {
        overflow = true;
        break;
      }
    }
    base += K;
    // exchange: queue lengths (and an overflow) to the team
    if (tid == 0) {
      const int32_t c = L.cnt[cur] < AQ ? L.cnt[cur] : AQ;
      fg_st_shared(&C->as_rec[as_member(P)], ((ull)(overflow ? 1 : 0) << 63) | (ull)(uint32_t)c);
    }
    if (!ts.sync_acquire(&L.flag)) {
      ok = false;
      break;
    }
    if (tid < FG_WAVE) {
      ull r = 0;
      if ((uint32_t)tid < T)
        r = __hip_atomic_load(&C->as_rec[tid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const int32_t c = (int32_t)(uint32_t)r;
      const int32_t o = (int32_t)(r >> 63);
      const int32_t incl = fg_wave_incl_scan(c);
      const int32_t tot = __builtin_amdgcn_readlane(incl, FG_WAVE - 1);
      const int32_t pre = __builtin_amdgcn_readlane(incl - c, as_member(P));
      const int32_t anyo = fg_wave_sum(o);
      if (tid == 0) {
        L.tot = tot;
        L.pre = pre;
        // stop: done (nothing queued), or out of room (an LDS queue, or the
        // exchange buffer)
        L.stop = anyo ? 2 : (tot == 0 ? 1 : ((int64_t)tot > (int64_t)P.n ? 2 : 0));
      }
    }
    __syncthreads();
    if (L.stop) {
      if (L.stop == 2 && as_member(P) == 0 && tid == 0)
        __hip_atomic_store(&C->as_state, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
    // even shares: every member writes its queue to the exchange buffer at
    // its prefix, then loads an equal slice (offsets and head entries
    // reloaded)
    const int32_t mine = L.cnt[cur] < AQ ? L.cnt[cur] : AQ;
    for (int32_t i = tid; i < mine; i += PB) fg_st_shared(&G[L.pre + i], L.qv[cur][i]);
    if (!ts.sync_acquire(&L.flag)) {
      ok = false;
      break;
    }
    const int64_t tot = L.tot;
    const int32_t lo = (int32_t)(tot * as_member(P) / T), hi = (int32_t)(tot * (as_member(P) + 1) / T);
    for (int32_t i = tid; i < hi - lo; i += PB) {
      const int32_t v = G[lo + i];
      L.qv[cur][i] = v;
      L.qb[cur][i] = P.off[v];
      L.qe[cur][i] = P.off[v + 1];
      L.qh[cur][i] = P.head[v];
    }
    __syncthreads();
    if (tid == 0) L.cnt[cur] = hi - lo;
    __syncthreads();
  }
  // totals; the last member out clears the team's barrier and records
  insp = fg_block_sum<PB>(insp, L.red64);
  if (tid == 0) {
    if (insp) atomicAdd(&C->as_insp, (ull)insp);
    if (!ok) __hip_atomic_store(&C->as_state, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t done = __hip_atomic_fetch_add(&C->as_exit, 1u, __ATOMIC_ACQ_REL,
                                                 __HIP_MEMORY_SCOPE_AGENT);
    if (done == T - 1) {
      C->as_arrive = 0;
      C->as_exit = 0;
      for (uint32_t i = 0; i < T; ++i) C->as_rec[i] = 0;
    }
  }
}

__global__ __launch_bounds__(PB) void bfs_async(BfsParams P) {
  __shared__ AsLds L;
  bfs_async_run(P, L);
}

// Two traversals side by side in one launch (fg_bfs_corun): workgroups
// [0, A.nblk) run A's list of sources as bfs_persistent does, workgroups
// [B.blk0, B.blk0 + B.nblk) run B's asynchronous push traversal as bfs_async
// does, any in between leave at once.  Neither range waits for the other;
// each synchronises only its own workgroups.
union CorunLds {
  Lds a;
  AsLds b;
};

template <int MODE>
__global__ __launch_bounds__(PB) void bfs_corun(BfsParams A, BfsParams B) {
  __shared__ CorunLds L;
  if (blockIdx.x < A.nblk)
    bfs_persistent_run<MODE, true>(A, L.a);
  else if (blockIdx.x >= B.blk0)
    bfs_async_run(B, L.b);
}

// Start of an asynchronous traversal: every key "unreached" but the
// source's (depth 0, parent itself); the asynchronous fields of the control
// block cleared; the record cleared.
__global__ void async_init_kernel(BfsParams P) {
  ull* key = (ull*)P.desc;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = tid; v < P.n; v += nth)
    key[v] = v == P.src ? (ull)(uint32_t)P.src : ~0ull;
  if (blockIdx.x == 0) {
    BfsCtl* C = P.ctl;
    for (int i = threadIdx.x; i < FG_TRACE_MAX; i += blockDim.x) {
      C->as_hist_cnt[i] = 0;
      C->as_hist_deg[i] = 0;
    }
    for (int i = threadIdx.x; i < TEAM_MAX; i += blockDim.x) C->as_rec[i] = 0;
    if (threadIdx.x == 0) {
      C->as_arrive = 0;
      C->as_state = 0;
      C->as_exit = 0;
      C->as_insp = 0;
    }
    if (P.stats) {
      uint32_t* sw = (uint32_t*)P.stats;
      for (int i = threadIdx.x; i < (int)(sizeof(fg_run_stats) / 4); i += blockDim.x) sw[i] = 0u;
    }
  }
  if (tid == 0 && P.stats) {
    P.stats->t_start = (int64_t)wall_clock64();
    P.stats->clock_khz = P.clock_khz;
  }
}

// Outputs from the keys: depth = key >> 32, parent = low word (-1 / -1 if
// unreached), plus the level sizes and their degree sums for the record.
// Per-workgroup totals of the finalize pass (vertices reached, largest
// depth), two words per workgroup in the half of the descriptor region the
// keys leave free (it holds 16 bytes per vertex, the keys 8), summed by the
// record kernel: no atomics on one address from every wave.
__device__ __forceinline__ ull* fin_partials(const BfsParams& P) { return (ull*)P.desc + P.n; }

__global__ __launch_bounds__(256) void async_finalize_kernel(BfsParams P) {
  __shared__ ull s_cnt[FG_TRACE_MAX], s_deg[FG_TRACE_MAX];
  __shared__ ull s_red[256 / FG_WAVE];
  __shared__ uint32_t s_max[256 / FG_WAVE];
  BfsCtl* C = P.ctl;
  if (__hip_atomic_load(&C->as_state, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  for (int i = threadIdx.x; i < FG_TRACE_MAX; i += blockDim.x) {
    s_cnt[i] = 0;
    s_deg[i] = 0;
  }
  __syncthreads();
  const ull* key = (const ull*)P.desc;
  ull reached = 0;
  uint32_t maxd = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // four vertices per round, their keys loaded before any store
  for (int64_t v0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v0 < P.n; v0 += 4 * stride) {
    ull k[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t v = v0 + r * stride;
      k[r] = v < P.n ? key[v] : ~0ull;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t v = v0 + r * stride;
      if (v >= P.n) continue;
      if (k[r] == ~0ull) {
        P.depth[v] = -1;
        if (P.parent) P.parent[v] = -1;
      } else {
        const uint32_t d = (uint32_t)(k[r] >> 32);
        P.depth[v] = (int32_t)d;
        if (P.parent) P.parent[v] = (int32_t)(uint32_t)k[r];
        reached++;
        maxd = d > maxd ? d : maxd;
        if (d < FG_TRACE_MAX) {
          atomicAdd(&s_cnt[d], 1ull);
          atomicAdd(&s_deg[d], (ull)(P.off[v + 1] - P.off[v]));
        }
      }
    }
  }
  reached = fg_block_sum<256>(reached, s_red);
  for (int d = FG_WAVE / 2; d > 0; d >>= 1) {
    const uint32_t o = __shfl_xor(maxd, d, FG_WAVE);
    maxd = o > maxd ? o : maxd;
  }
  if (fg_lane() == 0) s_max[threadIdx.x / FG_WAVE] = maxd;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < 256 / FG_WAVE; ++i) maxd = s_max[i] > maxd ? s_max[i] : maxd;
    fin_partials(P)[2 * blockIdx.x] = reached;
    fin_partials(P)[2 * blockIdx.x + 1] = maxd;
  }
  for (int i = threadIdx.x; i < FG_TRACE_MAX; i += blockDim.x) {
    if (s_cnt[i]) atomicAdd(&C->as_hist_cnt[i], s_cnt[i]);
    if (s_deg[i]) atomicAdd(&C->as_hist_deg[i], s_deg[i]);
  }
}

// The record of an asynchronous traversal: levels = largest depth + 1, the
// per-level trace from the level sizes (the entries a level-synchronous
// push reads: the frontier's degree sum), the entries the team read.  One
// wave; `parts` = workgroups of the finalize pass.
__global__ void async_stats_kernel(BfsParams P, int32_t team, int32_t parts) {
  BfsCtl* C = P.ctl;
  if (blockIdx.x != 0 || !P.stats) return;
  if (__hip_atomic_load(&C->as_state, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  ull reached = 0;
  uint32_t maxd = 0;
  for (int i = threadIdx.x; i < parts; i += FG_WAVE) {
    reached += fin_partials(P)[2 * i];
    const uint32_t d = (uint32_t)fin_partials(P)[2 * i + 1];
    maxd = d > maxd ? d : maxd;
  }
  reached = fg_wave_sum(reached);
  for (int d = FG_WAVE / 2; d > 0; d >>= 1) {
    const uint32_t o = __shfl_xor(maxd, d, FG_WAVE);
    maxd = o > maxd ? o : maxd;
  }
  if (threadIdx.x != 0) return;
  fg_run_stats* st = P.stats;
  const int32_t L = (int32_t)maxd + 1;
  const int64_t now = (int64_t)wall_clock64();
  for (int32_t k = 0; k < L && k < FG_TRACE_MAX; ++k) {
    st->dir[k] = 0;
    st->frontier[k] = (int64_t)C->as_hist_cnt[k];
    st->inspected[k] = (int64_t)C->as_hist_deg[k];
    st->t_end[k] = now;
  }
  st->status = FG_OK;
  st->iterations = L;
  st->reached = (int64_t)reached;
  st->edges_inspected = (int64_t)C->as_insp;
  st->direction_switches = 0;
  st->grid_blocks = team;
}

// a1: depth = -1 / parent = -1 except at the source, visited = {src},
// queue 0 = {src}, control block and stats cleared.
__global__ void bfs_init_kernel(int32_t n, int32_t nwords, int32_t src, int32_t* depth,
                                int32_t* parent, uint64_t* vis0, int32_t* q0, uint32_t* ctl,
                                int32_t ctl_words, uint32_t* stats, int32_t stats_words) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  const bool vec = ((((uintptr_t)depth) | ((uintptr_t)(parent ? parent : depth))) & 15) == 0;
  if (vec) {
    const int64_t n4 = n / 4;
    int4* d4 = (int4*)depth;
    int4* p4 = (int4*)parent;
    const int4 neg = make_int4(-1, -1, -1, -1);
    for (int64_t i = tid; i < n4; i += nth) {
      d4[i] = neg;
      if (parent) p4[i] = neg;
    }
    for (int64_t i = n4 * 4 + tid; i < n; i += nth) {
      depth[i] = -1;
      if (parent) parent[i] = -1;
    }
  } else {
    for (int64_t i = tid; i < n; i += nth) {
      depth[i] = -1;
      if (parent) parent[i] = -1;
    }
  }
  for (int64_t w = tid; w < nwords; w += nth) vis0[w] = 0ull;
  if (blockIdx.x == 0) {
    for (int i = threadIdx.x; i < ctl_words; i += blockDim.x) ctl[i] = 0u;
    if (stats)
      for (int i = threadIdx.x; i < stats_words; i += blockDim.x) stats[i] = 0u;
  }
}

// Source entries, after the bulk fill (stream order).
__global__ void bfs_seed_kernel(int32_t src, int32_t* depth, int32_t* parent, uint64_t* vis0,
                                int32_t* q0) {
  if (threadIdx.x == 0) {
    depth[src] = 0;
    if (parent) parent[src] = src;
    vis0[src >> 6] = 1ull << (src & 63);
    q0[0] = src;
  }
}

struct BfsLayout {
  BfsCtl* ctl;
  uint64_t* vis[2];
  int32_t* q[2];
  int4* desc;
  uint64_t* reached;  // fg_bfs_many, shared outputs: the last traversal's visited set
  size_t bytes;
};

BfsLayout bfs_layout(const fg_graph* g, void* ws) {
  fg_carver c(ws);
  BfsLayout L;
  L.ctl = c.take<BfsCtl>(1);
  L.vis[0] = c.take<uint64_t>(g->nwords);
  L.vis[1] = c.take<uint64_t>(g->nwords);
  L.q[0] = c.take<int32_t>(g->n);
  L.q[1] = c.take<int32_t>(g->n);
  L.desc = c.take<int4>((size_t)(g->m / CH) + (size_t)g->n + 64);
  L.reached = c.take<uint64_t>(g->nwords);
  L.bytes = c.used;
  return L;
}

int g_occupancy[2][64];

template <int MODE>
int persistent_blocks_per_cu(int device) {
  if (device < 0 || device >= 64) return 1;
  int& occ = g_occupancy[MODE == FG_MODE_DO ? 0 : 1][device];
  if (occ == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, bfs_persistent<MODE, false>, PB, 0) !=
            hipSuccess ||
        nb < 1)
      nb = 1;
    occ = nb;
  }
  return occ;
}

}  // namespace

size_t fg_bfs_workspace_bytes(const fg_graph* g) { return bfs_layout(g, nullptr).bytes; }

// a1 for every BFS variant: bulk fill, then the source entries.
void fg_bfs_launch_init(const fg_graph* g, int32_t src, int32_t* depth, int32_t* parent,
                        uint64_t* vis0, int32_t* q0, fg_run_stats* stats, hipStream_t s,
                        void* ctl, int32_t ctl_bytes) {
  int init_blocks = (int)((g->n + 4095) / 4096);
  if (init_blocks > 2048) init_blocks = 2048;
  if (init_blocks < 1) init_blocks = 1;
  bfs_init_kernel<<<init_blocks, 256, 0, s>>>(g->n, g->nwords, src, depth, parent, vis0, q0,
                                              (uint32_t*)ctl, ctl_bytes / 4, (uint32_t*)stats,
                                              (int32_t)(sizeof(fg_run_stats) / 4));
  bfs_seed_kernel<<<1, 64, 0, s>>>(src, depth, parent, vis0, q0);
}

// Argument checks shared by fg_bfs and fg_bfs_noalloc; fills *o.
static fg_status bfs_check(const char* fn, const fg_graph* g, int32_t src, const fg_bfs_opts* opts,
                           int32_t* depth, fg_bfs_opts* o) {
  if (!g) return fg_set_error(FG_EINVAL, "%s: graph is NULL", fn);
  if (src < 0 || src >= g->n)
    return fg_set_error(FG_EINVAL, "%s: src=%d outside [0, %d)", fn, src, g->n);
  if (!depth) return fg_set_error(FG_EINVAL, "%s: depth is NULL", fn);
  if (opts) *o = *opts; else fg_bfs_opts_default(o);
  if (o->mode != FG_MODE_DO && o->mode != FG_MODE_PUSH && o->mode != FG_MODE_PUSH_UNFUSED)
    return fg_set_error(FG_EINVAL, "%s: unknown mode %d", fn, o->mode);
  if (o->mode == FG_MODE_DO) {
    if (!g->symmetric)
      return fg_set_error(FG_EUNSUPPORTED,
                          "%s: the pull step needs an undirected graph (FG_SYMMETRIC)", fn);
    if (o->do_a_den == 0 || o->do_b_den == 0)
      return fg_set_error(FG_EINVAL, "%s: zero denominator in do_a / do_b", fn);
  }
  return FG_OK;
}

// Width of the persistent launch: workgroups per CU as occupancy allows (at
// most 2 by default; blocks_per_cu lowers it) times the CUs, at most
// grid_blocks when that is set.
static int persistent_grid(const fg_bfs_opts& o, const fg_device_props& pr, int occ) {
  int bpc = occ;
  if (o.blocks_per_cu > 0 && o.blocks_per_cu < bpc) bpc = o.blocks_per_cu;
  if (o.blocks_per_cu == 0 && bpc > 2) bpc = 2;
  const int grid = pr.cus * bpc;
  return o.grid_blocks > 0 && o.grid_blocks < grid ? o.grid_blocks : grid;
}

// Kernel parameters of one traversal (src) or of a list (srcs, nsrc) over
// the workspace `lay` (whose control block is zero), run by workgroups
// [0, nblk) of their launch.
static BfsParams bfs_params(const fg_graph* g, int32_t src, const fg_bfs_opts& o,
                            const BfsLayout& lay, int32_t* depth, int32_t* parent,
                            fg_run_stats* stats, const fg_device_props& pr, int nblk,
                            const int32_t* srcs, int32_t nsrc, int64_t out_stride) {
  BfsParams P;
  memset(&P, 0, sizeof(P));
  P.off = g->off;
  P.col = g->col;
  P.nz = g->nzmask;
  P.head = g->head;
  P.n = g->n;
  P.nwords = g->nwords;
  P.m = g->m;
  P.src = src;
  P.mode = o.mode;
  P.depth = depth;
  P.parent = parent;
  P.vis[0] = lay.vis[0];
  P.vis[1] = lay.vis[1];
  P.reached = lay.reached;
  P.q[0] = lay.q[0];
  P.q[1] = lay.q[1];
  P.desc = lay.desc;
  P.ctl = lay.ctl;
  P.stats = stats;
  P.a_num = o.do_a_num;
  P.a_den = o.do_a_den;
  P.b_num = o.do_b_num;
  P.b_den = o.do_b_den;
  P.small_q = o.small_frontier > 0 ? o.small_frontier : DEF_SMALL_Q;
  if (P.small_q > QCAP) P.small_q = QCAP;
  P.small_e = o.small_edges > 0 ? o.small_edges : DEF_SMALL_E;
  P.big_deg = o.big_degree > 0 ? o.big_degree : DEF_BIG_DEG;
  P.clock_khz = pr.clock_khz;
  P.team = o.team_blocks > 0 ? o.team_blocks : (o.team_blocks < 0 ? 0 : DEF_TEAM);
  if (P.team > nblk) P.team = nblk;
  if (P.team > TEAM_MAX) P.team = TEAM_MAX;
  P.team_e = o.team_edges > 0 ? o.team_edges : DEF_TEAM_E;
  // team decisions are exact below the word's degree cap
  if (P.team_e > TW_CAP - 1) P.team_e = TW_CAP - 1;
  if (P.small_e > TW_CAP - 1) P.small_e = TW_CAP - 1;
  P.srcs = srcs;
  P.nsrc = nsrc;
  P.out_stride = out_stride;
  P.async_k = o.async_levels > 1024 ? 1024 : o.async_levels;
  P.blk0 = 0;
  P.nblk = (uint32_t)nblk;
  return P;
}

// Workgroups of an asynchronous team.
static int async_team(const fg_bfs_opts& o, const fg_device_props& pr) {
  int T = o.team_blocks > 0 ? o.team_blocks : DEF_TEAM;
  if (T > pr.cus) T = pr.cus;
  if (T > TEAM_MAX) T = TEAM_MAX;
  if (T < 1) T = 1;
  return T;
}

// Workgroups of the per-vertex kernels around an asynchronous traversal.
static int async_fill_blocks(const fg_graph* g) {
  int fb = (int)((g->n + 4095) / 4096);
  if (fb > 2048) fb = 2048;
  if (fb < 1) fb = 1;
  return fb;
}

// The level-synchronous launch queued behind an asynchronous traversal: it
// runs only if the team gave up.
static fg_status async_fallback_launch(BfsParams P, int grid, hipStream_t s) {
  P.async_fallback = 1;
  P.blk0 = 0;
  P.nblk = (uint32_t)grid;
  if (P.team > grid) P.team = grid;
  void* args[] = {&P};
  FG_HIP_TRY(hipLaunchCooperativeKernel((const void*)bfs_persistent<FG_MODE_PUSH, false>,
                                        dim3(grid), dim3(PB), args, 0, s));
  return FG_OK;
}

// One persistent launch of the fused BFS kernel over the workspace `lay`
// (whose control block is zero).
static fg_status bfs_launch(const fg_graph* g, int32_t src, const fg_bfs_opts& o,
                            const BfsLayout& lay, int32_t* depth, int32_t* parent,
                            fg_run_stats* stats, hipStream_t s, const int32_t* srcs = nullptr,
                            int32_t nsrc = 0, int64_t out_stride = 0) {
  int dev = 0;
  FG_HIP_TRY(hipGetDevice(&dev));
  fg_device_props pr = fg_props(dev);
  if (!pr.coop) return fg_set_error(FG_EUNSUPPORTED, "fg_bfs: device lacks cooperative launch");
  const int grid = persistent_grid(o, pr, o.mode == FG_MODE_DO
                                              ? persistent_blocks_per_cu<FG_MODE_DO>(dev)
                                              : persistent_blocks_per_cu<FG_MODE_PUSH>(dev));
  BfsParams P = bfs_params(g, src, o, lay, depth, parent, stats, pr, grid, srcs, nsrc, out_stride);

  if (o.mode == FG_MODE_PUSH && o.async_levels > 1 && !srcs) {
    // asynchronous push: keys, the team's launch, outputs and record, and
    // the level-synchronous launch that runs only if the team gave up
    const int T = async_team(o, pr);
    const int fb = async_fill_blocks(g);
    BfsParams PA = P;
    PA.nblk = (uint32_t)T;
    async_init_kernel<<<fb, 256, 0, s>>>(PA);
    void* aargs[] = {&PA};
    FG_HIP_TRY(hipLaunchCooperativeKernel((const void*)bfs_async, dim3(T), dim3(PB), aargs, 0, s));
    async_finalize_kernel<<<fb, 256, 0, s>>>(PA);
    async_stats_kernel<<<1, FG_WAVE, 0, s>>>(PA, T, fb);
    return async_fallback_launch(P, grid, s);
  }

  void* args[] = {&P};
  const void* fn;
  if (srcs)
    fn = o.mode == FG_MODE_DO ? (const void*)bfs_persistent<FG_MODE_DO, true>
                              : (const void*)bfs_persistent<FG_MODE_PUSH, true>;
  else
    fn = o.mode == FG_MODE_DO ? (const void*)bfs_persistent<FG_MODE_DO, false>
                              : (const void*)bfs_persistent<FG_MODE_PUSH, false>;
  FG_HIP_TRY(hipLaunchCooperativeKernel(fn, dim3(grid), dim3(PB), args, 0, s));
  return FG_OK;
}

extern "C" fg_status fg_bfs(const fg_graph* g, int32_t src, const fg_bfs_opts* opts, void* ws,
                            size_t ws_bytes, int32_t* depth, int32_t* parent,
                            fg_run_stats* stats, void* stream) {
  fg_bfs_opts o;
  fg_status rc = bfs_check("fg_bfs", g, src, opts, depth, &o);
  if (rc != FG_OK) return rc;
  if (!ws) return fg_set_error(FG_EINVAL, "fg_bfs: workspace is NULL");
  if (o.mode == FG_MODE_PUSH_UNFUSED)
    return fg_bfs_unfused(g, src, ws, ws_bytes, depth, parent, stats, (hipStream_t)stream);
  BfsLayout lay = bfs_layout(g, ws);
  FG_CHECK_WS_ALIGN(ws, "fg_bfs");
  if (ws_bytes < lay.bytes)
    return fg_set_error(FG_ENOMEM, "fg_bfs: workspace of %zu bytes < required %zu", ws_bytes,
                        lay.bytes);
  return bfs_launch(g, src, o, lay, depth, parent, stats, (hipStream_t)stream);
}

extern "C" fg_status fg_bfs_many(const fg_graph* g, const int32_t* srcs, int32_t nsrc,
                                 const fg_bfs_opts* opts, void* ws, size_t ws_bytes,
                                 int32_t* depth, int32_t* parent, int64_t out_stride,
                                 fg_run_stats* stats, void* stream) {
  if (!g) return fg_set_error(FG_EINVAL, "fg_bfs_many: graph is NULL");
  if (nsrc < 0) return fg_set_error(FG_EINVAL, "fg_bfs_many: nsrc=%d < 0", nsrc);
  if (nsrc == 0) return FG_OK;
  if (!srcs) return fg_set_error(FG_EINVAL, "fg_bfs_many: srcs is NULL");
  if (out_stride != 0 && out_stride < g->n)
    return fg_set_error(FG_EINVAL, "fg_bfs_many: out_stride=%lld is neither 0 nor >= n=%d",
                        (long long)out_stride, g->n);
  fg_bfs_opts o;
  // the sources are device data, checked on the device: src 0 stands in here
  fg_status rc = bfs_check("fg_bfs_many", g, 0, opts, depth, &o);
  if (rc != FG_OK) return rc;
  if (!ws) return fg_set_error(FG_EINVAL, "fg_bfs_many: workspace is NULL");
  if (o.mode == FG_MODE_PUSH_UNFUSED)
    return fg_set_error(FG_EUNSUPPORTED, "fg_bfs_many: the unfused mode runs one source per call");
  BfsLayout lay = bfs_layout(g, ws);
  FG_CHECK_WS_ALIGN(ws, "fg_bfs_many");
  if (ws_bytes < lay.bytes)
    return fg_set_error(FG_ENOMEM, "fg_bfs_many: workspace of %zu bytes < required %zu", ws_bytes,
                        lay.bytes);
  return bfs_launch(g, 0, o, lay, depth, parent, stats, (hipStream_t)stream, srcs, nsrc,
                    out_stride);
}

static bool ranges_overlap(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  return x < y + nb && y < x + na;
}

static int g_corun_occupancy[2][64];

template <int MODE>
int corun_blocks_per_cu(int device) {
  if (device < 0 || device >= 64) return 1;
  int& occ = g_corun_occupancy[MODE == FG_MODE_DO ? 0 : 1][device];
  if (occ == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, bfs_corun<MODE>, PB, 0) != hipSuccess ||
        nb < 1)
      nb = 1;
    occ = nb;
  }
  return occ;
}

extern "C" fg_status fg_bfs_corun(const fg_graph* g, const int32_t* srcs, int32_t nsrc,
                                  const fg_bfs_opts* opts, void* ws, size_t ws_bytes,
                                  int32_t* depth, int32_t* parent, int64_t out_stride,
                                  fg_run_stats* stats, const fg_graph* g2, int32_t src2,
                                  const fg_bfs_opts* opts2, void* ws2, size_t ws2_bytes,
                                  int32_t* depth2, int32_t* parent2, fg_run_stats* stats2,
                                  void* stream) {
  const hipStream_t s = (hipStream_t)stream;
  // the asynchronous query
  fg_bfs_opts o2;
  fg_status rc = bfs_check("fg_bfs_corun", g2, src2, opts2, depth2, &o2);
  if (rc != FG_OK) return rc;
  if (o2.mode != FG_MODE_PUSH || o2.async_levels <= 1)
    return fg_set_error(FG_EINVAL,
                        "fg_bfs_corun: the second query needs FG_MODE_PUSH with async_levels > 1");
  if (!ws2) return fg_set_error(FG_EINVAL, "fg_bfs_corun: second workspace is NULL");
  FG_CHECK_WS_ALIGN(ws2, "fg_bfs_corun");
  const BfsLayout lay2 = bfs_layout(g2, ws2);
  if (ws2_bytes < lay2.bytes)
    return fg_set_error(FG_ENOMEM, "fg_bfs_corun: second workspace of %zu bytes < required %zu",
                        ws2_bytes, lay2.bytes);
  // the list
  if (!g) return fg_set_error(FG_EINVAL, "fg_bfs_corun: graph is NULL");
  if (nsrc < 0) return fg_set_error(FG_EINVAL, "fg_bfs_corun: nsrc=%d < 0", nsrc);
  if (nsrc > 0 && !srcs) return fg_set_error(FG_EINVAL, "fg_bfs_corun: srcs is NULL");
  if (out_stride != 0 && out_stride < g->n)
    return fg_set_error(FG_EINVAL, "fg_bfs_corun: out_stride=%lld is neither 0 nor >= n=%d",
                        (long long)out_stride, g->n);
  fg_bfs_opts o;
  rc = bfs_check("fg_bfs_corun", g, 0, opts, depth, &o);
  if (rc != FG_OK) return rc;
  if (o.mode == FG_MODE_PUSH_UNFUSED)
    return fg_set_error(FG_EUNSUPPORTED, "fg_bfs_corun: the unfused mode runs one source per call");
  if (!ws) return fg_set_error(FG_EINVAL, "fg_bfs_corun: workspace is NULL");
  FG_CHECK_WS_ALIGN(ws, "fg_bfs_corun");
  const BfsLayout lay = bfs_layout(g, ws);
  if (ws_bytes < lay.bytes)
    return fg_set_error(FG_ENOMEM, "fg_bfs_corun: workspace of %zu bytes < required %zu", ws_bytes,
                        lay.bytes);
  if (ranges_overlap(ws, lay.bytes, ws2, lay2.bytes))
    return fg_set_error(FG_EINVAL, "fg_bfs_corun: the two workspaces overlap");
  if (nsrc == 0) return bfs_launch(g2, src2, o2, lay2, depth2, parent2, stats2, s);

  int dev = 0;
  FG_HIP_TRY(hipGetDevice(&dev));
  fg_device_props pr = fg_props(dev);
  if (!pr.coop)
    return fg_set_error(FG_EUNSUPPORTED, "fg_bfs_corun: device lacks cooperative launch");
  fg_bfs_opts ow = o;
  ow.grid_blocks = 0;
  const int grid = persistent_grid(ow, pr, o.mode == FG_MODE_DO ? corun_blocks_per_cu<FG_MODE_DO>(dev)
                                                                : corun_blocks_per_cu<FG_MODE_PUSH>(dev));
  const int T = async_team(o2, pr);
  if (grid - T < 1)
    return fg_set_error(FG_EINVAL,
                        "fg_bfs_corun: a team of %d workgroups leaves none of %d for the list", T,
                        grid);
  // the list on workgroups [0, nA), the team on the last T; workgroups in
  // between (a list narrowed by grid_blocks, so that it loads the memory
  // system less while the latency-bound team runs) leave at once
  const int nA = o.grid_blocks > 0 && o.grid_blocks < grid - T ? o.grid_blocks : grid - T;
  BfsParams PA = bfs_params(g, 0, o, lay, depth, parent, stats, pr, nA, srcs, nsrc, out_stride);
  BfsParams PB2 = bfs_params(g2, src2, o2, lay2, depth2, parent2, stats2, pr, T, nullptr, 0, 0);
  PB2.blk0 = (uint32_t)(grid - T);
  const int fb = async_fill_blocks(g2);
  async_init_kernel<<<fb, 256, 0, s>>>(PB2);
  void* args[] = {&PA, &PB2};
  const void* fn = o.mode == FG_MODE_DO ? (const void*)bfs_corun<FG_MODE_DO>
                                        : (const void*)bfs_corun<FG_MODE_PUSH>;
  FG_HIP_TRY(hipLaunchCooperativeKernel(fn, dim3(grid), dim3(PB), args, 0, s));
  async_finalize_kernel<<<fb, 256, 0, s>>>(PB2);
  async_stats_kernel<<<1, FG_WAVE, 0, s>>>(PB2, T, fb);
  // if the team gave up, the second query runs level-synchronously
  const int grid2 = persistent_grid(o2, pr, persistent_blocks_per_cu<FG_MODE_PUSH>(dev));
  BfsParams PF = bfs_params(g2, src2, o2, lay2, depth2, parent2, stats2, pr, grid2, nullptr, 0, 0);
  return async_fallback_launch(PF, grid2, s);
}

// ------------------------------------------------ BFS without allocations
//
// The workspace of fg_bfs_noalloc lives in this file-scope device array,
// one copy per GPU, held until the process ends.  Host code never passes
// the array's name to a kernel (on the host it is only a stand-in for the
// symbol): the device address of each GPU's copy is looked up once per
// device with hipGetSymbolAddress and used from then on.
static __device__ __align__(256) unsigned char scratch[FG_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEV = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEV];

// Zeroes `words` 32-bit words (a fill kernel rather than a memset node, so
// the call can also be recorded into a graph).
__global__ void zero_words_kernel(uint32_t* p, int32_t words) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < words; i += gridDim.x * blockDim.x)
    p[i] = 0u;
}
}  // namespace

static fg_status scratch_ptr(int dev, void** out) {
  if (dev < 0 || dev >= MAX_DEV)
    return fg_set_error(FG_EUNSUPPORTED, "fg_bfs_noalloc: device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fg_set_error(FG_EDEVICE, "fg_bfs_noalloc: hipGetSymbolAddress failed: %s",
                          hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return FG_OK;
}

extern "C" fg_status fg_bfs_noalloc(const fg_graph* g, int32_t src, const fg_bfs_opts* opts,
                                    int32_t* depth, int32_t* parent, fg_run_stats* stats,
                                    void* stream) {
  fg_bfs_opts o;
  fg_status rc = bfs_check("fg_bfs_noalloc", g, src, opts, depth, &o);
  if (rc != FG_OK) return rc;
  if (o.mode == FG_MODE_PUSH_UNFUSED)
    return fg_set_error(FG_EUNSUPPORTED,
                        "fg_bfs_noalloc: FG_MODE_PUSH_UNFUSED needs a caller workspace (fg_bfs)");
  const size_t need = bfs_layout(g, nullptr).bytes;
  if (need > (size_t)FG_NOALLOC_SCRATCH_BYTES)
    return fg_set_error(FG_ENOMEM,
                        "fg_bfs_noalloc: the graph needs %zu bytes of workspace, more than the "
                        "%zu-byte static scratch; use fg_bfs with a caller workspace",
                        need, (size_t)FG_NOALLOC_SCRATCH_BYTES);
  int dev = 0;
  FG_HIP_TRY(hipGetDevice(&dev));
  void* ws = nullptr;
  rc = scratch_ptr(dev, &ws);
  if (rc != FG_OK) return rc;
  BfsLayout lay = bfs_layout(g, ws);
  hipStream_t s = (hipStream_t)stream;
  // the scratch keeps whatever the previous call on this GPU left: the
  // control block must start at zero (the rest is written before it is read)
  const int32_t ctl_words = (int32_t)(sizeof(BfsCtl) / 4);
  zero_words_kernel<<<(ctl_words + 255) / 256, 256, 0, s>>>((uint32_t*)lay.ctl, ctl_words);
  FG_HIP_TRY(hipGetLastError());
  return bfs_launch(g, src, o, lay, depth, parent, stats, s);
}
