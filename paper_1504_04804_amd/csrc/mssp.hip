// Batched single-source shortest paths: up to 64 independent SSSP queries
// (lanes) share one traversal, so the per-iteration cost of the persistent
// loop (grid barrier, queue bookkeeping) is paid once for all of them.  Each
// lane's distances equal fg_sssp's distances from its source.  Lanes are
// admitted at any step boundary (continuous batching) and finish when their
// work runs out.
//
// Distances are lane-minor, dist[v * 64 + lane], so one wave takes one
// vertex for all of its lanes and every distance access of a wave is one
// 256-byte line.  Per vertex, three 64-bit words hold one bit per lane:
// F[0] / F[1] (the vertex is in the lane's current / next near frontier)
// and Ff (the vertex is in the lane's far pile).
//
// Every lane follows the near-far ordering of the single-source kernel with
// its own threshold T[lane]: a relaxation that strictly improves (v, lane)
// to a distance below T[lane] sets the lane's bit in next[v] (a vertex whose
// next word was 0 joins the next active list); one that improves it to
// T[lane] or more sets the bit in Ff[v] (a vertex whose far word was 0 joins
// the far list).  A lane whose near frontier is empty at the start of an
// iteration splits instead of relaxing: T grows to the lane's next
// threshold, and a scan of the far list moves its entries now below T into
// the next frontier, drops the stale ones (below the old T: relaxed as near
// since) and keeps the rest.  The scan reads the whole far list whatever
// the number of lanes splitting, so idle lanes wait (a few iterations at
// most) until several of them can split in one scan.  A split that finds nothing ends the lane; one
// that only keeps entries sets the next threshold from their smallest
// distance.  Splits of some lanes run in the same iteration as the
// relaxations of the others, so an iteration ends with one grid barrier (two
// when vertices of high degree were cut into edge chunks).
//
// Data layout in HBM (caller workspace, 256-B aligned):
//   state    iteration, list selectors and lengths, live lanes, per-lane
//            thresholds (persists across steps)
//   dist     uint32[n][64]
//   F[0], F[1], Ff   uint64[n]
//   q        2 x int32[n]        active vertices (near frontier)
//   far      2 x int32[n]        far list (a vertex is listed once)
//   desc     int4[m/CHS + n + 64]  {vertex, first edge, lanes lo, lanes hi}
//   control  barrier and per-iteration counters of one launch (cleared on
//            exit)
#include <string.h>

#include "frontier.h"

namespace {
using namespace fgk;

constexpr int PB = 1024;
constexpr int PWAVES = PB / FG_WAVE;
constexpr int MAXL = 64;
constexpr int CHS = 64;  // edges per descriptor
constexpr int STAGE = 256;
constexpr int FSTAGE = 128;
constexpr uint32_t DIST_INF = 0xFFFFFFFFu;
// Team mode (see mp_team): LDS queue entries per member, widest team,
// packed team word fields, frontier shape it takes, default widths.
constexpr int QCAP = 2048;
constexpr int TEAM_MAX = 64;
constexpr int TW_CNT = 25, TW_FLAG = 50, TW_ARR = 57;
constexpr int64_t TW_CAP = (1 << 19) - 1;
constexpr int LDS_MEAN_DEG = 64;
constexpr int32_t DEF_TEAM = 32;
constexpr int32_t DEF_TEAM_WIDE = 64;
constexpr int64_t DEF_TEAM_E = 1 << 18;
constexpr int64_t TEAM_AUTO_DEG = 8;

struct MpState {
  int32_t it;      // iterations since open
  int32_t qsel;    // list holding the current active vertices
  int32_t fsel;    // F array of the current near frontier
  int32_t psel;    // far list in use
  int64_t qlen;    // current active vertices
  int64_t plen;    // entries of the far list
  ull live;        // lanes holding an unfinished query
  ull used;        // lanes admitted at least once
  ull nearl;       // lanes with a non-empty current near frontier
  ull edges;       // edge visits (one per edge and wave, all lanes at once)
  ull edge_lanes;  // edge relaxations attempted (per lane)
  uint32_t overflow;
  int32_t swait;   // iterations idle lanes have waited for a split
  uint32_t T[MAXL];
  uint32_t Tnext[MAXL];
};

// Counts of iteration k of a launch live in slot k % 3, which iteration k - 1
// cleared: a slot is read after its iteration's barriers and written again
// two iterations later, after at least one more grid barrier.
struct alignas(256) MpCtl {
  uint32_t bar[FG_BAR_WORDS];
  uint32_t exit_count;
  uint32_t pad0[63];
  Line64 qcnt[3];    // next active list appends
  Line64 dcnt[3];    // descriptors
  Line64 fcnt[3];    // far list appends
  Line64 nearw[3];   // lanes given a next near frontier entry
  Line64 stayw[3];   // lanes whose split kept far entries
  uint32_t minst[3][MAXL];  // per lane: smallest distance a split kept
  Line64 farpos;     // far list positions (monotone within a launch)
  Line64 edges;
  Line64 edge_lanes;
  int64_t pub_qlen, pub_plen;
  ull pub_live;
  uint32_t pub_ovf;
  // team mode: hand-back signal, team barrier, per-member records, level
  // words, lanes given next-frontier entries per level, overflow counter
  uint32_t sm_signal;
  uint32_t pad1[63];
  uint32_t sm_ack;  // waiters that have read a hand-back (monotone)
  uint32_t pad1b[63];
  uint32_t team_arrive;
  uint32_t pad2[63];
  ull team_rec[2][TEAM_MAX][2];
  Line64 team_word[3];
  Line64 tnear[3];
  Line64 team_ovf;
  int32_t tp_it, tp_qsel, tp_fsel, tp_levels, tp_force, tp_swait;
  int64_t tp_qlen, tp_plen;
  ull tp_live, tp_nearl;
};

struct MpParams {
  const int32_t* __restrict__ off;
  const int32_t* __restrict__ col;
  const uint32_t* __restrict__ w;
  int32_t n;
  uint32_t* dist;  // [n][64]
  ull* F[2];
  ull* Ff;
  int32_t* q[2];
  int32_t* far[2];
  int4* desc;
  MpState* state;
  MpCtl* ctl;
  int32_t k_iters;
  int32_t npend;
  int32_t pend_lane[MAXL];
  int32_t pend_src[MAXL];
  uint32_t delta;
  int32_t big_deg;
  int32_t dense;        // lanes from which a vertex is relaxed lane-parallel
  int32_t split_lanes;  // idle lanes that trigger a split of the far list
  int32_t split_wait;   // ... or iterations the idle lanes have waited
  int32_t team;         // workgroups of a team (<= 1: no team mode)
  int64_t team_e;       // largest frontier degree sum a team takes
};

struct Lds {
  int32_t stage[PWAVES][STAGE];
  int32_t fstage[PWAVES][FSTAGE];
  int32_t w_sc[PWAVES][FG_WAVE];
  int32_t w_u[PWAVES][FG_WAVE];
  int32_t w_b[PWAVES][FG_WAVE];
  int32_t w_d[PWAVES][FG_WAVE];
  ull w_m[PWAVES][FG_WAVE];
  ull redu[PWAVES];
  int64_t red64[PWAVES];
  uint32_t T[MAXL];
  uint32_t Tnext[MAXL];
  uint32_t minl[MAXL];
  int32_t flag;
  int32_t ackbad;  // workgroup 0: a hand-off acknowledgement wait failed
  // team mode: this member's share of the frontier (vertex, first edge, end
  // edge) for the current and the next level, counters over three slots,
  // block scan-gather arrays, exchange results
  int32_t lq_v[2][QCAP];
  int32_t lq_b[2][QCAP];
  int32_t lq_e[2][QCAP];
  int32_t lq_cnt[3];
  int32_t lq_deg[3];
  int32_t tsum[6];
  int32_t b_sc[PB];
  int32_t b_u[PB];
  int32_t b_b[PB];
  int32_t b_d[PB];
  ull b_m[PB];
  ull tnear;
  int64_t tfar;
  int32_t red32[PWAVES + 1];
};

__device__ __forceinline__ uint32_t sat_add(uint32_t a, uint32_t b) {
  const ull s = (ull)a + (ull)b;
  return s >= (ull)DIST_INF ? DIST_INF : (uint32_t)s;
}

__device__ __forceinline__ ull block_or(ull x, ull* scratch) {
  x = fg_wave_or64(x);
  const int wid = threadIdx.x / FG_WAVE;
  __syncthreads();
  if (fg_lane() == 0) scratch[wid] = x;
  __syncthreads();
  ull s = 0;
#pragma unroll
  for (int i = 0; i < PWAVES; ++i) s |= scratch[i];
  return s;
}

// Far-list appends: positions from the monotone counter, the number
// appended added to the iteration's count slot.
struct PileStage {
  int32_t* buf;
  int32_t cnt;

  __device__ __forceinline__ void flush(ull* pos_ctr, ull* count, ull base, int32_t* out) {
    if (cnt == 0) return;
    wave_lds_fence();
    ull pos = 0;
    if (fg_lane() == 0) {
      pos = atomicAdd(pos_ctr, (ull)cnt);
      atomicAdd(count, (ull)cnt);
    }
    pos = __shfl(pos, 0, FG_WAVE) - base;
    // written through: read by other workgroups after the next barrier
    for (int i = fg_lane(); i < cnt; i += FG_WAVE) fg_st_shared(&out[pos + i], buf[i]);
    wave_lds_fence();
    cnt = 0;
  }

  __device__ __forceinline__ void push(bool keep, int32_t x, ull* pos_ctr, ull* count, ull base,
                                       int32_t* out) {
    const uint64_t mask = __ballot(keep);
    if (!mask) return;
    const int32_t c = __popcll(mask);
    if (cnt + c > FSTAGE) flush(pos_ctr, count, base, out);
    if (keep) buf[cnt + fg_mbcnt(mask)] = x;
    cnt += c;
  }
};

// Where one iteration's outputs go.
struct Out {
  ull* Fn;
  int32_t* Qn;       // next active list (positions from qcnt)
  ull* qcnt;
  int32_t* pile;     // far list receiving appends
  ull* fpos;
  ull* fcnt;
  ull fbase;
};

// Relax the edges [e0, e1) of u for the lanes in m (one wave, lane = query
// lane).  Lanes of m get dist[u][lane] + w; four edges per step keep four
// distance loads in flight.
__device__ void relax_edges(const MpParams& P, const Lds& L, int32_t u, int32_t e0, int32_t e1,
                            ull m, const Out& O, WaveStage<int32_t, STAGE>& st, PileStage& fst,
                            ull& nearb, bool& ovf) {
  const int lane = fg_lane();
  const bool act = (m >> lane) & 1ull;
  const uint32_t du = P.dist[(int64_t)u * MAXL + lane];
  const uint32_t Tl = L.T[lane];
  for (int32_t j = e0; j < e1; j += 4) {
    int32_t v[4];
    uint32_t wt[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int32_t jj = j + r < e1 ? j + r : e1 - 1;
      v[r] = P.col[jj];
      wt[r] = P.w[jj];
    }
    uint32_t cur[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) cur[r] = P.dist[(int64_t)v[r] * MAXL + lane];
    int code[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      code[r] = 0;
      const ull nd = (ull)du + (ull)wt[r];
      if (act && j + r < e1) {
        if (nd >= (ull)DIST_INF) {
          ovf = true;  // a distance would not fit the uint32 output
        } else if ((uint32_t)nd < cur[r]) {
          const uint32_t old = atomicMin(&P.dist[(int64_t)v[r] * MAXL + lane], (uint32_t)nd);
          if ((uint32_t)nd < old) code[r] = (uint32_t)nd < Tl ? 1 : 2;
        }
      }
    }
    ull mn[4], mf[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      mn[r] = __ballot(code[r] == 1);
      mf[r] = __ballot(code[r] == 2);
    }
    nearb |= mn[0] | mn[1] | mn[2] | mn[3];
    // lane r publishes edge r's lanes
    const ull myn = lane == 0 ? mn[0] : lane == 1 ? mn[1] : lane == 2 ? mn[2] : lane == 3 ? mn[3] : 0ull;
    const ull myf = lane == 0 ? mf[0] : lane == 1 ? mf[1] : lane == 2 ? mf[2] : lane == 3 ? mf[3] : 0ull;
    const int32_t myv = lane == 0 ? v[0] : lane == 1 ? v[1] : lane == 2 ? v[2] : v[3];
    bool firstn = false, firstf = false;
    if (myn) firstn = atomicOr(&O.Fn[myv], myn) == 0ull;
    if (myf) firstf = atomicOr(&P.Ff[myv], myf) == 0ull;
    st.push(firstn, myv, O.qcnt, 0ull, O.Qn);
    fst.push(firstf, myv, O.fpos, O.fcnt, O.fbase, O.pile);
  }
}

// Relax edge e of u for lane l alone (one thread).
__device__ __forceinline__ void relax_one(const MpParams& P, const Lds& L, int32_t u, int l,
                                          int32_t e, const Out& O, bool& firstn, bool& firstf,
                                          int32_t& vout, ull& nearb, bool& ovf) {
  const int32_t v = P.col[e];
  vout = v;
  const ull nd = (ull)P.dist[(int64_t)u * MAXL + l] + (ull)P.w[e];
  if (nd >= (ull)DIST_INF) {
    ovf = true;
    return;
  }
  uint32_t* dp = &P.dist[(int64_t)v * MAXL + l];
  if ((uint32_t)nd >= *dp) return;
  const uint32_t old = atomicMin(dp, (uint32_t)nd);
  if ((uint32_t)nd >= old) return;
  const ull bit = 1ull << l;
  if ((uint32_t)nd < L.T[l]) {
    firstn = atomicOr(&O.Fn[v], bit) == 0ull;
    nearb |= bit;
  } else {
    firstf = atomicOr(&P.Ff[v], bit) == 0ull;
  }
}

// Index of the k-th set bit of m (k < popcount(m)).
__device__ __forceinline__ int kth_bit(ull m, int k) {
  for (int i = 0; i < k; ++i) m &= m - 1;
  return __builtin_ctzll(m);
}


// ---------------------------------------------------------------- team mode
//
// Near iterations of medium frontiers (at most QCAP * T / 2 vertices, mean
// degree <= LDS_MEAN_DEG, degree sum <= team_e) run as a team of T
// workgroups from LDS queues, as in the single-source kernels: each member
// keeps its share of the active vertices as (vertex, first edge, end edge)
// in LDS, takes a vertex's lanes with an agent-scope exchange of its
// current word, spreads the (edge, lane) pairs over its threads by a block
// scan, and appends a vertex whose next word was 0 (offsets loaded
// alongside) to its next LDS queue; far entries go to the far list as
// elsewhere.  A lane's own distance is read with an agent-scope atomic load
// (another member may just have lowered it).  Per level the members OR the
// lanes they gave next-frontier entries into the level's near word, then
// add one packed word to the level's team word and poll it (the near word
// is complete once every member has arrived: each OR returned before its
// member arrived).  Lanes whose near frontier empties wait as in the full
// grid; when their split is due, or the frontier leaves the mode's range,
// the members write their LDS queues to the global queue and the next
// iteration runs on the full grid.
struct TeamSync {
  uint32_t* arrive;
  uint32_t* abort_flag;
  uint32_t T;
  uint32_t count;

  __device__ bool sync(int* s_flag) {
    __syncthreads();
    if (threadIdx.x == 0) {
      count++;
      __hip_atomic_fetch_add(arrive, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      *s_flag = !fg_wait_geq(arrive, count * T, abort_flag, 1);
    }
    __syncthreads();
    return *s_flag == 0;
  }
};

struct TeamBases {
  ull ovf;          // team_ovf value at which the current global queue starts
  uint32_t levels;  // team word exchanges so far
};

// Workgroup 0 clears the team and near words of exchange `level + 1`.
__device__ __forceinline__ ull team_clear_next(const MpParams& P, uint32_t level) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const ull a = __hip_atomic_exchange(&P.ctl->team_word[(level + 1) % 3].v, 0ull,
                                        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const ull b = __hip_atomic_exchange(&P.ctl->tnear[(level + 1) % 3].v, 0ull, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
    return a | b;
  }
  return 0;
}

__device__ bool team_fast(const MpParams& P, Lds& L, uint32_t T, uint32_t level, int32_t bcnt,
                          int32_t bdeg, int32_t lim, ull cleared) {
  if (threadIdx.x == 0) {
    ull* w = &P.ctl->team_word[level % 3].v;
    const ull g = bdeg < TW_CAP ? (ull)bdeg : (ull)TW_CAP;
    const ull add = (1ull << TW_ARR) | ((ull)(bcnt > lim) << TW_FLAG) | ((ull)bcnt << TW_CNT) | g;
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
    L.tnear = __hip_atomic_load(&P.ctl->tnear[level % 3].v, __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_AGENT);
    L.tfar = (int64_t)__hip_atomic_load(&P.ctl->farpos.v, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
    L.flag = bad;
  }
  __syncthreads();
  return L.flag == 0;
}

__device__ bool team_records(const MpParams& P, Lds& L, uint32_t T, uint32_t seq, int odd) {
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

__device__ __forceinline__ void wave_put(Lds& L, int nxt, bool won, int32_t pos, int32_t v,
                                         int32_t vb, int32_t ve, int32_t* Qo, ull* ovf,
                                         ull ovf_base) {
  const bool over = won && pos >= QCAP;
  if (won && !over) {
    L.lq_v[nxt][pos] = v;
    L.lq_b[nxt][pos] = vb;
    L.lq_e[nxt][pos] = ve;
  }
  const uint64_t om = __ballot(over);
  if (om) {
    ull base = 0;
    if (fg_lane() == 0) base = atomicAdd(ovf, (ull)__popcll(om));
    base = fg_uni(base);
    if (over) Qo[base - ovf_base + fg_mbcnt(om)] = v;
  }
}

// Far-list append of a wave's new far vertices (one atomic per wave).
__device__ __forceinline__ void far_put(const MpParams& P, bool put, int32_t v, int32_t* pile,
                                        ull fbase) {
  const uint64_t m = __ballot(put);
  if (m) {
    ull base = 0;
    if (fg_lane() == 0) base = atomicAdd(&P.ctl->farpos.v, (ull)__popcll(m));
    base = fg_uni(base);
    if (put) pile[base - fbase + fg_mbcnt(m)] = v;
  }
}

// Batch state the team reads and advances (identical in every member).
struct MpRun {
  int32_t it, qsel, fsel, psel, swait;
  int64_t qlen, plen;
  ull fbase, live, nearl;
};

// Near iterations as a team of T members (blockIdx.x < T), at most `budget`.
// Returns false on a device error; *levels = iterations run; *handback = 1
// when the frontier met on entry does not suit the mode.
__device__ bool mp_team(const MpParams& P, MpRun& R, Lds& L, uint32_t T, TeamSync& ts,
                        TeamBases& tb, int32_t budget, int32_t kbase, int32_t* levels,
                        int* handback, bool& ovf, ull& edges, ull& edge_lanes) {
  const int tid = threadIdx.x;
  const int lane = fg_lane();
  MpCtl* C = P.ctl;
  ull* ovfc = &C->team_ovf.v;
  ull ovf_base = tb.ovf;
  int cur = 0, ci = 0, ni = 1, ri = 2;
  *levels = 0;
  *handback = 0;
  {
    const int32_t* Qg = P.q[R.qsel];
    const int64_t lo = R.qlen * blockIdx.x / T, hi = R.qlen * (blockIdx.x + 1) / T;
    const int32_t cnt = (int32_t)(hi - lo);
    int32_t sd = 0;
    for (int32_t i = tid; i < cnt; i += PB) {
      const int32_t u = Qg[lo + i];
      const int32_t b = P.off[u], e = P.off[u + 1];
      L.lq_v[cur][i] = u;
      L.lq_b[cur][i] = b;
      L.lq_e[cur][i] = e;
      sd += e - b;
    }
    if (tid == 0) {
      L.lq_cnt[ci] = cnt;
      L.lq_cnt[ni] = 0;
      L.lq_deg[ni] = 0;
    }
    const int32_t bsd = fg_block_sum<PB>(sd, L.red32);
    if (!team_fast(P, L, T, tb.levels, cnt, bsd, QCAP, team_clear_next(P, tb.levels)))
      return false;
    tb.levels++;
    const int64_t qd = fg_uni(L.tsum[1]);
    if (qd > LDS_MEAN_DEG * R.qlen || qd > P.team_e) {
      *handback = 1;
      return true;
    }
    __syncthreads();
  }
  for (;;) {
    int32_t* Qo = P.q[R.qsel ^ 1];
    const int nxt = cur ^ 1;
    const int32_t cnt = L.lq_cnt[ci];
    const ull cleared = team_clear_next(P, tb.levels);
    if (tid == 0) {
      L.lq_cnt[ri] = 0;
      L.lq_deg[ri] = 0;
    }
    ull* Fc = P.F[R.fsel];
    ull* Fn = P.F[R.fsel ^ 1];
    int32_t* pile = P.far[R.psel];
    ull nearb = 0;
    for (int32_t c0 = 0; c0 < cnt; c0 += PB) {
      const int32_t i = c0 + tid;
      int32_t u = 0, b = 0, d = 0;
      ull m = 0;
      if (i < cnt) {
        u = L.lq_v[cur][i];
        b = L.lq_b[cur][i];
        d = L.lq_e[cur][i] - b;
        m = __hip_atomic_exchange(&Fc[u], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      const int32_t pc = __popcll(m);
      edges += m ? (ull)d : 0ull;
      edge_lanes += (ull)d * (ull)pc;
      const int32_t items = d * pc;
      int32_t Tn = 0;
      const int32_t ex = fg_block_excl_scan<PB>(items, L.red32, &Tn);
      L.b_sc[tid] = ex;
      L.b_u[tid] = u;
      L.b_b[tid] = b;
      L.b_d[tid] = d;
      L.b_m[tid] = m;
      __syncthreads();
      const int32_t nc = cnt - c0 < PB ? cnt - c0 : PB;
      for (int32_t t0 = 0; t0 < Tn; t0 += PB) {
        const int32_t t = t0 + tid;
        bool won = false, fput = false;
        int32_t v = 0, vb = 0, ve = 0;
        if (t < Tn) {
          const int32_t jj = upper_idx(L.b_sc, nc, t);
          const int32_t r = t - L.b_sc[jj];
          const int32_t dj = L.b_d[jj];
          const int32_t li = r / dj;
          const int l = kth_bit(L.b_m[jj], li);
          const int32_t e = L.b_b[jj] + (r - li * dj);
          const int32_t uj = L.b_u[jj];
          v = P.col[e];
          const uint32_t wt = P.w[e];
          vb = P.off[v];
          ve = P.off[v + 1];
          const ull nd = (ull)__hip_atomic_load(&P.dist[(int64_t)uj * MAXL + l], __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT) + (ull)wt;
          if (nd >= (ull)DIST_INF) {
            ovf = true;
          } else {
            const uint32_t old = atomicMin(&P.dist[(int64_t)v * MAXL + l], (uint32_t)nd);
            if ((uint32_t)nd < old) {
              const ull bit = 1ull << l;
              if ((uint32_t)nd < L.T[l]) {
                won = atomicOr(&Fn[v], bit) == 0ull;
                nearb |= bit;
              } else {
                fput = atomicOr(&P.Ff[v], bit) == 0ull;
              }
            }
          }
        }
        const int32_t pos = wave_reserve(won ? 1 : 0, &L.lq_cnt[ni]);
        const int32_t wdeg = fg_wave_sum(won ? ve - vb : 0);
        if (lane == 0 && wdeg) atomicAdd(&L.lq_deg[ni], wdeg);
        wave_put(L, nxt, won, pos, v, vb, ve, Qo, ovfc, ovf_base);
        far_put(P, fput, v, pile, R.fbase);
      }
      __syncthreads();
    }
    const ull bn = block_or(nearb, L.redu);
    const int32_t bcnt = L.lq_cnt[ni];
    const int32_t bdeg = L.lq_deg[ni];
    ull orv = 0;
    if (tid == 0) {
      if (bn)
        orv = __hip_atomic_fetch_or(&C->tnear[tb.levels % 3].v, bn, __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT);
      ull* rr = C->team_rec[R.it & 1][blockIdx.x];
      const ull tag = (ull)((uint32_t)R.it + 1u) << 32;
      __hip_atomic_store(rr, tag | (uint32_t)bcnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const int64_t lim = (5 * R.qlen / T + 64) / 4;
    // the near OR returns before the arrival is issued
    asm volatile("" ::"v"(orv) : "memory");
    if (!team_fast(P, L, T, tb.levels, bcnt, bdeg, (int32_t)(lim < QCAP ? lim : QCAP), cleared))
      return false;
    tb.levels++;
    const int64_t nq = fg_uni(L.tsum[0]);
    const int64_t nqdeg = fg_uni(L.tsum[1]);
    const int64_t nflag = fg_uni(L.tsum[2]);
    const ull nw = L.tnear;
    const int64_t far_now = L.tfar;
    R.it++;
    R.qlen = nq;
    R.fsel ^= 1;
    R.nearl = nw;
    R.plen = (int64_t)((ull)far_now - R.fbase);
    (*levels)++;
    // lanes whose near frontier emptied: finished when nothing is far; a
    // due split ends the episode, otherwise they wait as on the full grid
    ull idle = R.live & ~R.nearl;
    if (idle && R.plen == 0) {
      R.live &= ~idle;
      idle = 0;
    }
    const bool split_due = idle && (__popcll(idle) >= P.split_lanes || (R.live & R.nearl) == 0 ||
                                    R.swait + 1 >= P.split_wait);
    if (idle && !split_due) R.swait++;
    bool stay = nq > 0 && R.live != 0 && !split_due && nqdeg <= LDS_MEAN_DEG * nq &&
                nqdeg <= P.team_e && nq <= (int64_t)QCAP * T / 2 && *levels < budget;
    int64_t nover = bcnt > QCAP ? bcnt - QCAP : 0, before = 0;
    bool rebalance = false;
    if (!stay || nflag) {
      if (!team_records(P, L, T, (uint32_t)R.it, (R.it - 1) & 1)) return false;
      nover = fg_uni(L.tsum[3]);
      before = fg_uni(L.tsum[4]);
      stay = stay && fg_uni(L.tsum[2]) == 0;
      rebalance = stay && 4 * fg_uni(L.tsum[5]) * (int64_t)T > 5 * nq + 64 * (int64_t)T;
    }
    if (!stay || rebalance) {
      const int32_t nloc = bcnt < QCAP ? bcnt : QCAP;
      int32_t* dst = Qo + nover + before;
      for (int32_t i = tid; i < nloc; i += PB) dst[i] = L.lq_v[nxt][i];
      ovf_base += (ull)nover;
      tb.ovf = ovf_base;
      if (!stay && blockIdx.x == 0) {
        // the count slot of the next full-grid iteration starts cleared
        const int s = (kbase + *levels) % 3;
        if (tid == 0) {
          __hip_atomic_store(&C->qcnt[s].v, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(&C->dcnt[s].v, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(&C->fcnt[s].v, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(&C->nearw[s].v, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(&C->stayw[s].v, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (tid < MAXL)
          __hip_atomic_store(&C->minst[s][tid], DIST_INF, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
      }
      if (!ts.sync(&L.flag)) return false;
      R.qsel ^= 1;
      if (!stay) return true;
      // reload an even share from the global queue
      const int32_t* Qg = P.q[R.qsel];
      const int64_t lo = R.qlen * blockIdx.x / T, hi = R.qlen * (blockIdx.x + 1) / T;
      const int32_t c2 = (int32_t)(hi - lo);
      for (int32_t i = tid; i < c2; i += PB) {
        const int32_t u = Qg[lo + i];
        L.lq_v[nxt][i] = u;
        L.lq_b[nxt][i] = P.off[u];
        L.lq_e[nxt][i] = P.off[u + 1];
      }
      __syncthreads();
      if (tid == 0) L.lq_cnt[ni] = c2;
      __syncthreads();
    }
    cur = nxt;
    const int t3 = ci;
    ci = ni;
    ni = ri;
    ri = t3;
  }
}

// TEAM = false compiles the kernel without the team episodes: their code
// raises the register pressure of the whole kernel (spills on every path),
// which costs more than the team saves on graphs of high mean degree.
template <bool TEAM>
__global__ __launch_bounds__(PB) void mssp_persistent(MpParams P) {
  __shared__ Lds L;
  fg_grid_sync gs{P.ctl->bar, gridDim.x, 0u};
  const int64_t tid = (int64_t)blockIdx.x * PB + threadIdx.x;
  const int64_t nth = (int64_t)gridDim.x * PB;
  const int lane = fg_lane();
  const int wid = threadIdx.x / FG_WAVE;
  const int64_t gw = (int64_t)blockIdx.x * PWAVES + wid;
  const int64_t W = (int64_t)gridDim.x * PWAVES;
  MpCtl* C = P.ctl;
  // every workgroup reads the state before anyone writes it
  int32_t it = P.state->it, qsel = P.state->qsel, fsel = P.state->fsel, psel = P.state->psel;
  int32_t swait = P.state->swait;
  int64_t qlen = P.state->qlen, plen = P.state->plen;
  ull live = P.state->live, used = P.state->used, nearl = P.state->nearl;
  if (threadIdx.x < MAXL) {
    L.T[threadIdx.x] = P.state->T[threadIdx.x];
    L.Tnext[threadIdx.x] = P.state->Tnext[threadIdx.x];
  }
  // farpos restarts at 0 in every launch: the far list's next append goes to
  // index plen
  ull fbase = 0ull - (ull)plen;
  bool ovf = false;
  if (blockIdx.x == 0 && threadIdx.x < MAXL) C->minst[0][threadIdx.x] = DIST_INF;
  bool ok = gs.sync(&L.flag);

  // ---- admissions: clear the pending lanes' distances (and their bits if
  // the lane held an earlier query), seed the sources
  if (ok && P.npend > 0) {
    ull mask = 0;
    for (int i = 0; i < P.npend; ++i) mask |= 1ull << P.pend_lane[i];
    const ull reused = mask & used;
    for (int64_t v = tid; v < P.n; v += nth) {
      uint32_t* row = P.dist + v * MAXL;
      for (int i = 0; i < P.npend; ++i) row[P.pend_lane[i]] = DIST_INF;
    }
    if (reused) {
      // clear the lanes' bits and rebuild the far list without them
      int32_t* nl = P.far[psel ^ 1];
      WaveStage<int32_t, STAGE> st{L.stage[wid], 0};
      for (int64_t v0 = gw * FG_WAVE; v0 < P.n; v0 += W * FG_WAVE) {
        const int64_t v = v0 + lane;
        bool keep = false;
        if (v < P.n) {
          P.F[0][v] &= ~reused;
          P.F[1][v] &= ~reused;
          const ull f = P.Ff[v];
          const ull g = f & ~reused;
          if (f != g) P.Ff[v] = g;
          keep = g != 0ull;
        }
        st.push(keep, (int32_t)v, &C->farpos.v, 0ull, nl);
      }
      st.flush(&C->farpos.v, 0ull, nl);
    }
    ok = gs.sync(&L.flag);
    if (reused) {
      plen = (int64_t)fg_atomic_load_u64(&C->farpos.v);
      fbase = 0ull;
      psel ^= 1;
    }
    if (ok && tid == 0) {
      int64_t ql = qlen;
      for (int i = 0; i < P.npend; ++i) {
        const int32_t l = P.pend_lane[i], s = P.pend_src[i];
        P.dist[(int64_t)s * MAXL + l] = 0u;
        if (P.F[fsel][s] == 0ull) P.q[qsel][ql++] = s;
        P.F[fsel][s] |= 1ull << l;
      }
      C->pub_qlen = ql;
    }
    if (threadIdx.x < MAXL && ((mask >> threadIdx.x) & 1ull)) {
      L.T[threadIdx.x] = P.delta;
      L.Tnext[threadIdx.x] = sat_add(P.delta, P.delta);
    }
    ok = ok && gs.sync(&L.flag);
    qlen = C->pub_qlen;
    live |= mask;
    used |= mask;
    nearl |= mask;
  }

  ull edges = 0, edge_lanes = 0;
  TeamSync ts{&C->team_arrive, C->bar + FG_BAR_STRIDE, (uint32_t)(P.team > 1 ? P.team : 1), 0u};
  TeamBases tb = {};
  uint32_t sm_seen = 0;
  uint32_t ack_need = 0;  // workgroup 0: acknowledgements of the hand-backs so far
  int force_full = 0;
  for (int32_t k = 0; ok && k < P.k_iters && live != 0ull; ++k) {
    // ---- near iterations of medium frontiers as a team (the others sleep)
    {
      const ull idle0 = live & ~nearl;
      const bool split_now = idle0 && plen > 0 &&
                             (__popcll(idle0) >= P.split_lanes || (live & nearl) == 0 ||
                              swait + 1 >= P.split_wait);
      if (TEAM && !force_full && !split_now && P.team > 1 && qlen > 0 &&
          qlen <= (int64_t)QCAP * P.team / 2) {
        sm_seen++;
        int32_t nl = 0;
        if (blockIdx.x < (uint32_t)P.team) {
          MpRun R{it, qsel, fsel, psel, swait, qlen, plen, fbase, live, nearl};
          int hb = 0;
          if (!mp_team(P, R, L, (uint32_t)P.team, ts, tb, P.k_iters - k, k, &nl, &hb, ovf, edges,
                       edge_lanes))
            ok = false;
          it = R.it;
          qsel = R.qsel;
          fsel = R.fsel;
          swait = R.swait;
          qlen = R.qlen;
          plen = R.plen;
          live = R.live;
          nearl = R.nearl;
          if (blockIdx.x == 0 && threadIdx.x == 0) {
            // every waiter of the previous hand-back has read it (on a
            // timeout the abort flag is set and every wait ends)
            L.ackbad = !fg_wait_geq(&C->sm_ack, ack_need, C->bar + FG_BAR_STRIDE, 1);
            // a failed wait has set the abort flag: publish nothing (a slow
            // waiter may still be reading the previous hand-off); the waiters
            // see the flag and leave
            if (!L.ackbad) {
              C->tp_it = it;
              C->tp_qsel = qsel;
              C->tp_fsel = fsel;
              C->tp_levels = nl;
              C->tp_force = hb;
              C->tp_swait = swait;
              C->tp_qlen = qlen;
              C->tp_plen = plen;
              C->tp_live = live;
              C->tp_nearl = nearl;
              __hip_atomic_fetch_add(&C->sm_signal, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
              ack_need += gridDim.x - (uint32_t)P.team;
            }
          }
          force_full = hb;
          __syncthreads();
          if (!ok || (blockIdx.x == 0 && L.ackbad)) {
            ok = false;
            break;
          }
        } else {
          if (threadIdx.x == 0) {
            const int bad = !fg_wait_geq(&C->sm_signal, sm_seen, C->bar + FG_BAR_STRIDE, 4096);
            L.flag = bad;
          }
          __syncthreads();
          if (L.flag) {
            ok = false;
            break;
          }
          const MpCtl* cc = C;
          it = cc->tp_it;
          qsel = cc->tp_qsel;
          fsel = cc->tp_fsel;
          nl = cc->tp_levels;
          force_full = cc->tp_force;
          swait = cc->tp_swait;
          qlen = cc->tp_qlen;
          plen = cc->tp_plen;
          live = cc->tp_live;
          nearl = cc->tp_nearl;
          __builtin_amdgcn_s_waitcnt(0);  // every wave has its copy
          __syncthreads();
          if (threadIdx.x == 0) fg_handoff_ack(&C->sm_ack);
        }
        k += nl - 1;  // the loop adds the last one
        continue;
      }
    }
    force_full = 0;
    const int s = k % 3;
    ull idle = live & ~nearl;  // lanes with an empty near frontier
    if (idle && plen == 0) {
      live &= ~idle;  // empty near frontier and nothing far: finished
      idle = 0;
      if (!live) break;
    }
    ull sl = 0;  // lanes that split in this iteration
    if (idle) {
      if (__popcll(idle) >= P.split_lanes || (live & nearl) == 0 || swait + 1 >= P.split_wait) {
        sl = idle;
        swait = 0;
      } else {
        swait++;
      }
    }
    if (tid == 0) {
      const int s1 = (k + 1) % 3;
      __hip_atomic_store(&C->qcnt[s1].v, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&C->dcnt[s1].v, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&C->fcnt[s1].v, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&C->nearw[s1].v, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&C->stayw[s1].v, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (blockIdx.x == 0 && threadIdx.x < MAXL)
      __hip_atomic_store(&C->minst[(k + 1) % 3][threadIdx.x], DIST_INF, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    if (threadIdx.x < MAXL) L.minl[threadIdx.x] = DIST_INF;
    const ull kbase = fbase + (ull)plen;  // farpos value at the start of this iteration
    Out O;
    O.Fn = P.F[fsel ^ 1];
    O.Qn = P.q[qsel ^ 1];
    O.qcnt = &C->qcnt[s].v;
    O.pile = sl ? P.far[psel ^ 1] : P.far[psel];
    O.fpos = &C->farpos.v;
    O.fcnt = &C->fcnt[s].v;
    O.fbase = sl ? kbase : fbase;
    WaveStage<int32_t, STAGE> st{L.stage[wid], 0};
    PileStage fst{L.fstage[wid], 0};
    ull nearb = 0, stayb = 0;
    __syncthreads();  // minl initialised

    // ---- near frontier, 64 list entries per wave.  A vertex with many
    // frontier lanes is relaxed lane-parallel (one wave, coalesced distance
    // rows); the (edge, lane) pairs of the others are spread over the wave's
    // threads by a scan; vertices of high degree go to edge chunks.
    {
      const int32_t* Qc = P.q[qsel];
      ull* Fc = P.F[fsel];
      int32_t* sc = L.w_sc[wid];
      int32_t* su = L.w_u[wid];
      int32_t* sb = L.w_b[wid];
      int32_t* sd = L.w_d[wid];
      ull* sm = L.w_m[wid];
      for (int64_t base = gw * FG_WAVE; base < qlen; base += W * FG_WAVE) {
        const int64_t i = base + lane;
        int32_t u = 0, b = 0, d = 0;
        ull m = 0;
        if (i < qlen) {
          u = Qc[i];
          m = Fc[u];
          if (m) {
            fg_st_shared(&Fc[u], 0ull);  // only this thread reads u's word in this iteration
            b = P.off[u];
            d = P.off[u + 1] - b;
          }
        }
        const int pc = __popcll(m);
        edges += (ull)d;
        edge_lanes += (ull)d * (ull)pc;
        const bool big = d >= P.big_deg;
        const bool dense = !big && d > 0 && pc >= P.dense;
        // edge chunks
        const int32_t nch = big ? (d + CHS - 1) / CHS : 0;
        const int32_t chi = fg_wave_incl_scan(nch);
        const int32_t NC = __shfl(chi, FG_WAVE - 1, FG_WAVE);
        if (NC > 0) {
          ull d0 = 0;
          if (lane == 0) d0 = atomicAdd(&C->dcnt[s].v, (ull)NC);
          d0 = __shfl(d0, 0, FG_WAVE);
          wave_lds_fence();
          sc[lane] = chi - nch;
          su[lane] = u;
          sb[lane] = b;
          sm[lane] = m;
          wave_lds_fence();
          for (int32_t t = lane; t < NC; t += FG_WAVE) {
            const int32_t j = upper_idx(sc, FG_WAVE, t);
            const ull mj = sm[j];
            fg_st_shared(&P.desc[d0 + t],
                         make_int4(su[j], sb[j] + (t - sc[j]) * CHS, (int32_t)(uint32_t)mj,
                                   (int32_t)(uint32_t)(mj >> 32)));
          }
          wave_lds_fence();
        }
        // lane-parallel vertices
        ull dm = __ballot(dense);
        while (dm) {
          const int j = __builtin_ctzll(dm);
          dm &= dm - 1;
          const int32_t uj = __builtin_amdgcn_readlane(u, j);
          const int32_t bj = __builtin_amdgcn_readlane(b, j);
          const int32_t dj = __builtin_amdgcn_readlane(d, j);
          const ull mj = fg_readlane64(m, j);
          relax_edges(P, L, uj, bj, bj + dj, mj, O, st, fst, nearb, ovf);
        }
        // (edge, lane) pairs of the sparse vertices
        const int32_t items = (!big && !dense) ? d * pc : 0;
        const int32_t inc = fg_wave_incl_scan(items);
        const int32_t T = __shfl(inc, FG_WAVE - 1, FG_WAVE);
        if (T == 0) continue;
        wave_lds_fence();
        sc[lane] = inc - items;
        su[lane] = u;
        sb[lane] = b;
        sd[lane] = d;
        sm[lane] = m;
        wave_lds_fence();
        for (int32_t t0 = 0; t0 < T; t0 += FG_WAVE) {
          const int32_t t = t0 + lane;
          bool fn = false, ff = false;
          int32_t v = 0;
          if (t < T) {
            const int32_t j = upper_idx(sc, FG_WAVE, t);
            const int32_t r = t - sc[j];
            const int32_t dj = sd[j];
            const int32_t li = r / dj;
            relax_one(P, L, su[j], kth_bit(sm[j], li), sb[j] + (r - li * dj), O, fn, ff, v,
                      nearb, ovf);
          }
          st.push(fn, v, O.qcnt, 0ull, O.Qn);
          fst.push(ff, v, O.fpos, O.fcnt, O.fbase, O.pile);
        }
      }
    }
    // ---- splits of the lanes with an empty near frontier
    if (sl) {
      const int32_t* pile = P.far[psel];
      for (int64_t base = tid - lane; base < plen; base += nth) {
        const int64_t i = base + lane;
        int32_t v = 0;
        bool keep = false, first = false;
        if (i < plen) {
          v = pile[i];
          const ull f = P.Ff[v];
          ull fb = f & sl;
          ull clr = 0, mv = 0;
          while (fb) {
            const int l = __builtin_ctzll(fb);
            fb &= fb - 1;
            const uint32_t d = P.dist[(int64_t)v * MAXL + l];
            if (d < L.Tnext[l]) {
              clr |= 1ull << l;
              if (d >= L.T[l]) mv |= 1ull << l;
            } else {
              stayb |= 1ull << l;
              atomicMin(&L.minl[l], d);
            }
          }
          ull rest = f;
          if (clr) rest = atomicAnd(&P.Ff[v], ~clr) & ~clr;
          keep = rest != 0ull;
          if (mv) {
            first = atomicOr(&O.Fn[v], mv) == 0ull;
            nearb |= mv;
          }
        }
        st.push(first, v, O.qcnt, 0ull, O.Qn);
        fst.push(keep, v, O.fpos, O.fcnt, O.fbase, O.pile);
      }
    }
    st.flush(O.qcnt, 0ull, O.Qn);
    fst.flush(O.fpos, O.fcnt, O.fbase, O.pile);
    {
      const ull bn = block_or(nearb, L.redu);
      const ull bs = block_or(stayb, L.redu);
      if (threadIdx.x == 0) {
        if (bn) atomicOr(&C->nearw[s].v, bn);
        if (bs) atomicOr(&C->stayw[s].v, bs);
      }
      if (threadIdx.x < MAXL && ((bs >> threadIdx.x) & 1ull))
        atomicMin(&C->minst[s][threadIdx.x], L.minl[threadIdx.x]);
    }
    if (!(ok = gs.sync_acquire(&L.flag))) break;
    // ---- edge chunks of high-degree vertices: one chunk per wave
    const int64_t nd = (int64_t)fg_atomic_load_u64(&C->dcnt[s].v);
    if (nd > 0) {
      ull nb2 = 0;
      for (int64_t i = gw; i < nd; i += W) {
        const int4 dsc = P.desc[i];
        const ull m = (ull)(uint32_t)dsc.z | ((ull)(uint32_t)dsc.w << 32);
        const int32_t e_end = P.off[dsc.x + 1];
        const int32_t e1 = dsc.y + CHS < e_end ? dsc.y + CHS : e_end;
        if (__popcll(m) >= P.dense) {
          relax_edges(P, L, dsc.x, dsc.y, e1, m, O, st, fst, nb2, ovf);
          continue;
        }
        // few lanes: one edge per thread, lane after lane
        ull mm = m;
        while (mm) {
          const int l = __builtin_ctzll(mm);
          mm &= mm - 1;
          const int32_t e = dsc.y + lane;
          bool fn = false, ff = false;
          int32_t v = 0;
          if (e < e1) relax_one(P, L, dsc.x, l, e, O, fn, ff, v, nb2, ovf);
          st.push(fn, v, O.qcnt, 0ull, O.Qn);
          fst.push(ff, v, O.fpos, O.fcnt, O.fbase, O.pile);
        }
      }
      st.flush(O.qcnt, 0ull, O.Qn);
      fst.flush(O.fpos, O.fcnt, O.fbase, O.pile);
      const ull bn = block_or(nb2, L.redu);
      if (threadIdx.x == 0 && bn) atomicOr(&C->nearw[s].v, bn);
      if (!(ok = gs.sync_acquire(&L.flag))) break;
    }
    // ---- next state (identical in every workgroup)
    const ull nw = fg_atomic_load_u64(&C->nearw[s].v);
    const ull sw = fg_atomic_load_u64(&C->stayw[s].v);
    qlen = (int64_t)fg_atomic_load_u64(&C->qcnt[s].v);
    const int64_t fa = (int64_t)fg_atomic_load_u64(&C->fcnt[s].v);
    if (sl) {
      fbase = kbase;
      plen = fa;
      psel ^= 1;
    } else {
      plen += fa;
    }
    qsel ^= 1;
    fsel ^= 1;
    if (sl) {
      __syncthreads();
      if (threadIdx.x < MAXL && ((sl >> threadIdx.x) & 1ull)) {
        const int l = threadIdx.x;
        const uint32_t Tn = L.Tnext[l];
        L.T[l] = Tn;
        if ((nw >> l) & 1ull) {
          L.Tnext[l] = sat_add(Tn, P.delta);
        } else if ((sw >> l) & 1ull) {
          const uint32_t mk = __hip_atomic_load(&C->minst[s][l], __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
          L.Tnext[l] = sat_add(mk, P.delta);
        }
      }
      live &= ~(sl & ~nw & ~sw);  // nothing moved, nothing kept: finished
      __syncthreads();
    }
    nearl = nw;
    it++;
  }
  // ---- statistics and state
  {
    const int64_t be = fg_block_sum<PB>((int64_t)edges, L.red64);
    const int64_t bl = fg_block_sum<PB>((int64_t)edge_lanes, L.red64);
    if (threadIdx.x == 0) {
      if (be) atomicAdd(&C->edges.v, (ull)be);
      if (bl) atomicAdd(&C->edge_lanes.v, (ull)bl);
    }
    if (ovf) atomicOr(&C->pub_ovf, 1u);
  }
  const bool ok2 = gs.sync(&L.flag);
  if (blockIdx.x == 0) {
    MpState* S = P.state;
    if (threadIdx.x == 0) {
      S->it = it;
      S->qsel = qsel;
      S->fsel = fsel;
      S->psel = psel;
      S->qlen = qlen;
      S->plen = plen;
      S->live = (ok && ok2) ? live : 0ull;
      S->used = used;
      S->nearl = nearl;
      S->swait = swait;
      S->edges += fg_atomic_load_u64(&C->edges.v);
      S->edge_lanes += fg_atomic_load_u64(&C->edge_lanes.v);
      const uint32_t o = __hip_atomic_load(&C->pub_ovf, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (o || !(ok && ok2)) S->overflow = o ? 1u : 2u;
    }
    if (threadIdx.x < MAXL) {
      S->T[threadIdx.x] = L.T[threadIdx.x];
      S->Tnext[threadIdx.x] = L.Tnext[threadIdx.x];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t done = __hip_atomic_fetch_add(&C->exit_count, 1u, __ATOMIC_ACQ_REL,
                                                 __HIP_MEMORY_SCOPE_AGENT);
    L.flag = done == gridDim.x - 1;
  }
  __syncthreads();
  if (L.flag) {
    uint32_t* wv = (uint32_t*)C;
    for (int i = threadIdx.x; i < (int)(sizeof(MpCtl) / 4); i += PB) wv[i] = 0u;
  }
}

// out[v] = dist[v][lane]
__global__ void mssp_read_kernel(const uint32_t* __restrict__ dist, int32_t n, int32_t lane,
                                 uint32_t* __restrict__ out) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x)
    out[v] = dist[v * MAXL + lane];
}

struct MpLayout {
  MpState* state;
  MpCtl* ctl;
  uint32_t* dist;
  ull* F[2];
  ull* Ff;
  int32_t* q[2];
  int32_t* far[2];
  int4* desc;
  size_t bytes;
};

MpLayout mp_layout(const fg_graph* g, void* ws) {
  fg_carver c(ws);
  MpLayout L;
  L.state = c.take<MpState>(1);
  L.ctl = c.take<MpCtl>(1);
  L.dist = c.take<uint32_t>((size_t)g->n * MAXL);
  L.F[0] = c.take<ull>(g->n);
  L.F[1] = c.take<ull>(g->n);
  L.Ff = c.take<ull>(g->n);
  // + 64: admissions list their sources even when a reused lane's cleared
  // bits leave listed vertices without lanes
  L.q[0] = c.take<int32_t>((size_t)g->n + MAXL);
  L.q[1] = c.take<int32_t>((size_t)g->n + MAXL);
  L.far[0] = c.take<int32_t>(g->n);
  L.far[1] = c.take<int32_t>(g->n);
  L.desc = c.take<int4>((size_t)(g->m / CHS) + (size_t)g->n + 64);
  L.bytes = c.used;
  return L;
}

int g_mp_occ[64];

uint32_t default_delta(const fg_graph* g) {
  if (g->m <= 0 || g->nonzero_degree <= 0) return 1u;
  const double d = 64.0 * ((double)g->w_sum / (double)g->m) /
                   ((double)g->m / (double)g->nonzero_degree);
  if (d >= 4294967295.0) return DIST_INF;
  return d < 1.0 ? 1u : (uint32_t)(d + 0.5);
}

}  // namespace

struct fg_mssp {
  const fg_graph* g = nullptr;
  int32_t lanes = 0;
  MpLayout lay;
  int32_t npend = 0;
  int32_t pend_lane[MAXL];
  int32_t pend_src[MAXL];
  uint64_t admitted = 0;
  fg_mssp_opts opts;
};

size_t fg_mssp_workspace_bytes(const fg_graph* g) { return mp_layout(g, nullptr).bytes; }

extern "C" void fg_mssp_opts_default(fg_mssp_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
}

extern "C" fg_status fg_mssp_open(const fg_graph* g, int32_t lanes, void* ws, size_t ws_bytes,
                                  const fg_mssp_opts* opts, void* stream, fg_mssp** out) {
  if (!out) return fg_set_error(FG_EINVAL, "fg_mssp_open: out is NULL");
  *out = nullptr;
  if (!g || !ws) return fg_set_error(FG_EINVAL, "fg_mssp_open: NULL graph or workspace");
  if (!g->w) return fg_set_error(FG_EINVAL, "fg_mssp_open: the graph was loaded without weights");
  if (lanes < 1 || lanes > MAXL)
    return fg_set_error(FG_EINVAL, "fg_mssp_open: lanes=%d outside [1, 64]", lanes);
  MpLayout lay = mp_layout(g, ws);
  FG_CHECK_WS_ALIGN(ws, "fg_mssp_open");
  if (ws_bytes < lay.bytes)
    return fg_set_error(FG_ENOMEM, "fg_mssp_open: workspace of %zu bytes < required %zu", ws_bytes,
                        lay.bytes);
  hipStream_t s = (hipStream_t)stream;
  FG_HIP_TRY(hipMemsetAsync(lay.state, 0, sizeof(MpState), s));
  FG_HIP_TRY(hipMemsetAsync(lay.ctl, 0, sizeof(MpCtl), s));
  FG_HIP_TRY(hipMemsetAsync(lay.F[0], 0, sizeof(ull) * (size_t)g->n, s));
  FG_HIP_TRY(hipMemsetAsync(lay.F[1], 0, sizeof(ull) * (size_t)g->n, s));
  FG_HIP_TRY(hipMemsetAsync(lay.Ff, 0, sizeof(ull) * (size_t)g->n, s));
  fg_mssp* b = new fg_mssp();
  b->g = g;
  b->lanes = lanes;
  b->lay = lay;
  if (opts) b->opts = *opts; else fg_mssp_opts_default(&b->opts);
  *out = b;
  return FG_OK;
}

extern "C" fg_status fg_mssp_close(fg_mssp* b) {
  delete b;
  return FG_OK;
}

extern "C" fg_status fg_mssp_admit(fg_mssp* b, int32_t lane, int32_t src) {
  if (!b) return fg_set_error(FG_EINVAL, "fg_mssp_admit: batch is NULL");
  if (lane < 0 || lane >= b->lanes)
    return fg_set_error(FG_EINVAL, "fg_mssp_admit: lane=%d outside [0, %d)", lane, b->lanes);
  if (src < 0 || src >= b->g->n)
    return fg_set_error(FG_EINVAL, "fg_mssp_admit: src=%d outside [0, %d)", src, b->g->n);
  for (int i = 0; i < b->npend; ++i)
    if (b->pend_lane[i] == lane)
      return fg_set_error(FG_EINVAL, "fg_mssp_admit: lane %d already pending", lane);
  b->pend_lane[b->npend] = lane;
  b->pend_src[b->npend] = src;
  b->npend++;
  b->admitted |= 1ull << lane;
  return FG_OK;
}

extern "C" fg_status fg_mssp_step(fg_mssp* b, int32_t k_iters, void* stream) {
  if (!b) return fg_set_error(FG_EINVAL, "fg_mssp_step: batch is NULL");
  if (k_iters < 0) return fg_set_error(FG_EINVAL, "fg_mssp_step: negative k_iters");
  int dev = 0;
  FG_HIP_TRY(hipGetDevice(&dev));
  fg_device_props pr = fg_props(dev);
  if (!pr.coop) return fg_set_error(FG_EUNSUPPORTED, "fg_mssp_step: no cooperative launch");
  if (dev >= 0 && dev < 64 && g_mp_occ[dev] == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, mssp_persistent<true>, PB, 0) !=
            hipSuccess ||
        nb < 1)
      nb = 1;
    g_mp_occ[dev] = nb;
  }
  int bpc = (dev >= 0 && dev < 64) ? g_mp_occ[dev] : 1;
  if (bpc > 2) bpc = 2;
  if (b->opts.blocks_per_cu > 0 && b->opts.blocks_per_cu < bpc) bpc = b->opts.blocks_per_cu;
  const fg_graph* g = b->g;
  MpParams P;
  memset(&P, 0, sizeof(P));
  P.off = g->off;
  P.col = g->col;
  P.w = g->w;
  P.n = g->n;
  P.dist = b->lay.dist;
  P.F[0] = b->lay.F[0];
  P.F[1] = b->lay.F[1];
  P.Ff = b->lay.Ff;
  P.q[0] = b->lay.q[0];
  P.q[1] = b->lay.q[1];
  P.far[0] = b->lay.far[0];
  P.far[1] = b->lay.far[1];
  P.desc = b->lay.desc;
  P.state = b->lay.state;
  P.ctl = b->lay.ctl;
  P.k_iters = k_iters;
  P.npend = b->npend;
  for (int i = 0; i < b->npend; ++i) {
    P.pend_lane[i] = b->pend_lane[i];
    P.pend_src[i] = b->pend_src[i];
  }
  // on graphs of mean degree > 8 a batch wants a coarser step than one
  // source (R-MAT 22, 64 lanes: 81 ms at the one-source step, 66 ms at
  // twice it); on grids the one-source step is best
  const bool low_deg = g->m <= (int64_t)TEAM_AUTO_DEG * g->n;
  uint32_t dd = default_delta(g);
  if (!low_deg && dd < DIST_INF / 2) dd *= 2;
  P.delta = b->opts.delta > 0 ? b->opts.delta : dd;
  P.big_deg = b->opts.big_degree > 0 ? b->opts.big_degree : 4 * CHS;
  if (P.big_deg > 65536) P.big_deg = 65536;  // keeps a wave's (edge, lane) count in int32
  P.dense = b->opts.dense_lanes > 0 ? b->opts.dense_lanes : 16;
  // defaults by graph shape: on graphs of mean degree <= 8 (grids,
  // road-like graphs: long, thin near frontiers) idle lanes wait to split
  // together and near iterations of medium frontiers run as a team; on
  // others a lane splits as soon as its near frontier is empty (waiting
  // makes the other lanes' iterations expand more vertices there) and the
  // kernel without the team runs
  P.split_lanes = b->opts.split_lanes > 0 ? b->opts.split_lanes : 8;
  P.split_wait = b->opts.split_wait > 0 ? b->opts.split_wait : (low_deg ? 8 : 1);
  void* args[] = {&P};
  int grid = pr.cus * bpc;
  if (b->opts.grid_blocks > 0 && b->opts.grid_blocks < grid) grid = b->opts.grid_blocks;
  const int lanes_in = __builtin_popcountll(b->admitted);
  P.team = b->opts.team_blocks > 0 ? b->opts.team_blocks
           : (b->opts.team_blocks < 0 || !low_deg) ? 1
           : (lanes_in >= 4 ? DEF_TEAM_WIDE : DEF_TEAM);
  if (P.team > TEAM_MAX) P.team = TEAM_MAX;
  if (P.team > grid) P.team = grid;
  P.team_e = b->opts.team_edges > 0 ? b->opts.team_edges : DEF_TEAM_E;
  if (P.team_e > TW_CAP - 1) P.team_e = TW_CAP - 1;

  const void* kern = P.team > 1 ? (const void*)mssp_persistent<true>
                                : (const void*)mssp_persistent<false>;
  FG_HIP_TRY(hipLaunchCooperativeKernel(kern, dim3(grid), dim3(PB), args, 0,
                                        (hipStream_t)stream));
  b->npend = 0;
  return FG_OK;
}

extern "C" fg_status fg_mssp_poll(fg_mssp* b, uint64_t* done_lanes, int32_t* iterations,
                                  void* stream) {
  if (!b) return fg_set_error(FG_EINVAL, "fg_mssp_poll: batch is NULL");
  MpState hs;
  hipStream_t s = (hipStream_t)stream;
  FG_HIP_TRY(hipMemcpyAsync(&hs, b->lay.state, sizeof(MpState), hipMemcpyDeviceToHost, s));
  FG_HIP_TRY(hipStreamSynchronize(s));
  uint64_t pend = 0;
  for (int i = 0; i < b->npend; ++i) pend |= 1ull << b->pend_lane[i];
  if (done_lanes) *done_lanes = b->admitted & ~hs.live & ~pend;
  if (iterations) *iterations = hs.it;
  if (hs.overflow == 1u)
    return fg_set_error(FG_EOVERFLOW, "fg_mssp_poll: a distance reached 2^32 - 1");
  if (hs.overflow)
    return fg_set_error(FG_EDEVICE, "fg_mssp_poll: the traversal stopped (barrier abort)");
  return FG_OK;
}

extern "C" fg_status fg_mssp_counts(fg_mssp* b, uint64_t* edges, uint64_t* edge_lanes,
                                    void* stream) {
  if (!b) return fg_set_error(FG_EINVAL, "fg_mssp_counts: batch is NULL");
  MpState hs;
  hipStream_t s = (hipStream_t)stream;
  FG_HIP_TRY(hipMemcpyAsync(&hs, b->lay.state, sizeof(MpState), hipMemcpyDeviceToHost, s));
  FG_HIP_TRY(hipStreamSynchronize(s));
  if (edges) *edges = hs.edges;
  if (edge_lanes) *edge_lanes = hs.edge_lanes;
  return FG_OK;
}

extern "C" fg_status fg_mssp_read(fg_mssp* b, int32_t lane, uint32_t* dist, void* stream) {
  if (!b || !dist) return fg_set_error(FG_EINVAL, "fg_mssp_read: NULL argument");
  if (lane < 0 || lane >= b->lanes)
    return fg_set_error(FG_EINVAL, "fg_mssp_read: lane=%d outside [0, %d)", lane, b->lanes);
  int blocks = (int)((b->g->n + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  mssp_read_kernel<<<blocks, 256, 0, (hipStream_t)stream>>>(b->lay.dist, b->g->n, lane, dist);
  FG_HIP_TRY(hipGetLastError());
  return FG_OK;
}

extern "C" fg_status fg_mssp_release(fg_mssp* b, int32_t lane) {
  if (!b) return fg_set_error(FG_EINVAL, "fg_mssp_release: batch is NULL");
  if (lane < 0 || lane >= b->lanes)
    return fg_set_error(FG_EINVAL, "fg_mssp_release: lane=%d outside [0, %d)", lane, b->lanes);
  b->admitted &= ~(1ull << lane);
  return FG_OK;
}
