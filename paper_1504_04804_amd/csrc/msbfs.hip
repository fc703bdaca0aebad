// Batched multi-source BFS: up to 64 independent BFS queries (lanes) share
// one traversal.  Every vertex holds a 64-bit word per structure, one bit per
// lane: `visit` (lanes that reached it), and two frontier words F[0] / F[1]
// (lanes for which it is in the current / next frontier).  Each lane's
// depths equal those of a single-source BFS from its source; lanes can be
// admitted at any step boundary (continuous batching) and retire when their
// frontier empties.
//
// Per iteration, on the device, one of two directions (as in Sec. VI-A):
//   push: for every active vertex u and edge u->v, the lanes of F[u] not yet
//         in visit[v] are claimed with a 64-bit atomicOr on visit[v]; the
//         lanes this thread claimed get their depth and go into next[v]
//         (atomicOr); a vertex whose next word was 0 joins the next active
//         list.  Each active vertex clears its own current word, so one grid
//         barrier ends a push iteration.
//   pull: every vertex with unvisited live lanes ORs F[u] over its neighbours
//         in CSR order and stops as soon as every wanted lane is covered;
//         whole-word writes, no atomics.
// Push load balance reuses the scan-gather + edge-chunk descriptors of the
// BFS kernel.  Data layout in HBM (caller workspace):
//   state   iteration counter, direction, live / used lanes, lane start
//           iterations (persists across steps)
//   visit, F[0], F[1]   uint64[n]
//   queue   2 x int32[n]        active vertices (push)
//   desc    int4[m/CH + n + 64]  {vertex, first edge, lanes (lo, hi)}
//   depth   int32[lanes][n]     lane-major, so each lane's result is contiguous
//   control barrier and counters of one launch (cleared on exit)
#include <string.h>

#include "frontier.h"

namespace {
using namespace fgk;

constexpr int PB = 1024;
constexpr int PWAVES = PB / FG_WAVE;
constexpr int CH = 256;
constexpr int STAGE = 512;
constexpr int DSTAGE = 64;
constexpr int MAXL = 64;
// Pull: vertices with more than LONG_PULL unresolved entries are not scanned
// by their own wave (the hubs of an R-MAT graph sit in the first bitmap
// words, so one wave would scan them all); they are listed and their lists
// cut into CH-entry chunks that every wave takes in turn.
constexpr int32_t LONG_PULL = 64;
// Team mode (push levels of medium frontiers; see team_levels): LDS queue
// entries per member, widest team, packed team word fields, frontier shape.
constexpr int QCAP = 2048;
constexpr int TEAM_MAX = 64;
constexpr int TW_CNT = 25, TW_FLAG = 50, TW_ARR = 57;
constexpr int64_t TW_CAP = (1 << 19) - 1;
constexpr int LDS_MEAN_DEG = 64;
constexpr int TPV = 4;
// default team: 32 workgroups for up to 3 lanes, 64 for more (their union
// frontier is wider); degree sums up to 2^18 per level
constexpr int32_t DEF_TEAM = 32;
constexpr int32_t DEF_TEAM_WIDE = 64;
constexpr int64_t DEF_TEAM_E = 1 << 18;
constexpr int64_t TEAM_AUTO_DEG = 8;
constexpr int32_t TEAM_MIN_Q = 1;

struct MsState {
  int32_t it;      // global iteration counter
  int32_t mode;    // 0 push (active list valid), 1 pull
  int32_t qsel;    // queue of the current active list
  int32_t fsel;    // F array of the current frontier
  int64_t qlen;    // active vertices of the current frontier
  ull live;        // lanes with a non-empty current frontier
  ull used;        // lanes admitted at least once
  int32_t start[MAXL];
  ull edges;  // adjacency entries read since open (push: whole lists; pull:
              // up to the early exit)
  ull verts;  // vertex visits since open (push: active; pull: every vertex)
  int32_t aborted;  // a step stopped early (a workgroup wait hit its limit)
  int32_t pad[11];
};

// Monotone counters of one iteration parity (see the BFS kernel).
struct CtrSlot {
  Line64 q;
  Line64 desc;
  Line64 cnt;
};

struct alignas(256) MsCtl {
  uint32_t bar[FG_BAR_WORDS];
  uint32_t exit_count;
  uint32_t pad0[63];
  CtrSlot slot[2];
  // OR of the lanes discovered in iteration k lives in livew[k % 3]; it is
  // zeroed at the start of iteration k-1, after its previous use (k-3) was
  // read by every workgroup
  Line64 livew[3];
  int64_t pub_qlen;
  ull pub_live;
  // team mode: hand-back signal to the waiting workgroups, team barrier,
  // per-member records, level words, overflow counter, episode live words
  uint32_t sm_signal;
  uint32_t pad1[63];
  uint32_t sm_ack;  // waiters that have read a hand-back (monotone)
  uint32_t pad1b[63];
  uint32_t team_arrive;
  uint32_t pad2[63];
  ull team_rec[2][TEAM_MAX][2];
  Line64 team_word[3];
  Line64 team_ovf;
  int32_t pub_it, pub_qsel, pub_fsel, pub_levels, pub_force;
  int64_t pub_tqlen;
  ull pub_tlive;
};

struct MsParams {
  const int32_t* __restrict__ off;
  const int32_t* __restrict__ col;
  const int4* __restrict__ head;  // first four neighbours per vertex
  int32_t n;
  int64_t m;
  int32_t lanes;
  ull* visit;
  ull* F[2];
  int32_t* q[2];
  int4* desc;
  int32_t* depth;  // [lanes][n]
  MsState* state;
  MsCtl* ctl;
  int32_t k_iters;
  int32_t npend;
  int32_t pend_lane[MAXL];
  int32_t pend_src[MAXL];
  int32_t big_deg;
  int32_t pull_div;  // push -> pull when active vertices > n / pull_div
  int32_t push_div;  // pull -> push when active vertices < n / push_div
  int32_t team;      // workgroups of a team (<= 1: no team mode)
  int64_t team_e;    // largest frontier degree sum a team takes
};

struct Lds {
  int32_t stage[PWAVES][STAGE];
  int4 dstage[PWAVES][DSTAGE];
  ull w_f[PWAVES][FG_WAVE];
  int32_t w_sc[PWAVES][FG_WAVE];
  int32_t w_u[PWAVES][FG_WAVE];
  int32_t w_b[PWAVES][FG_WAVE];
  int64_t red[PWAVES + 1];
  int32_t red32[PWAVES + 1];
  ull redu[PWAVES + 1];
  int32_t flag;
  int32_t ackbad;  // workgroup 0: a hand-off acknowledgement wait failed
  int64_t bcast[4];
  int32_t start[MAXL];  // iteration at which each lane was admitted
  // team mode: this member's share of the frontier (vertex, first edge, end
  // edge) for the current and the next level; counters over three slots
  int32_t lq_v[2][QCAP];
  int32_t lq_b[2][QCAP];
  int32_t lq_e[2][QCAP];
  int32_t lq_cnt[3];
  int32_t lq_deg[3];
  int32_t lq_big[3];
  int32_t tsum[6];
  int32_t b_sc[PB];
  int32_t b_u[PB];
  int32_t b_b[PB];
  ull b_f[PB];
};


__device__ __forceinline__ ull block_or(ull x, ull* scratch) {
#pragma unroll
  for (int d = FG_WAVE / 2; d > 0; d >>= 1) x |= __shfl_xor(x, d, FG_WAVE);
  const int wid = threadIdx.x / FG_WAVE;
  __syncthreads();
  if (fg_lane() == 0) scratch[wid] = x;
  __syncthreads();
  ull s = 0;
#pragma unroll
  for (int i = 0; i < PWAVES; ++i) s |= scratch[i];
  return s;
}

// depth[l][v] = d for every lane l set in `bits`.
__device__ __forceinline__ void write_depths(const MsParams& P, int32_t v, ull bits, int32_t it1) {
  while (bits) {
    const int l = __builtin_ctzll(bits);
    bits &= bits - 1;
    P.depth[(int64_t)l * P.n + v] = it1 - P.state->start[l];
  }
}

__device__ __forceinline__ int4 make_desc(int32_t u, int32_t e0, ull f) {
  return make_int4(u, e0, (int32_t)(uint32_t)f, (int32_t)(uint32_t)(f >> 32));
}
__device__ __forceinline__ ull desc_lanes(const int4& d) {
  return (ull)(uint32_t)d.z | ((ull)(uint32_t)d.w << 32);
}

// Claim the lanes `fu` for v: the ones not yet visited get depth it1 and go
// into next[v]; returns true when v's next word was 0 (v joins the list).
// `got` accumulates the lanes claimed.
__device__ __forceinline__ bool claim(const MsParams& P, ull* Fn, int32_t v, ull fu, int32_t it1,
                                      const int32_t* start, ull& got) {
  const ull nb = fu & ~P.visit[v];
  if (!nb) return false;
  const ull nw = nb & ~atomicOr(&P.visit[v], nb);
  if (!nw) return false;
  got |= nw;
  ull bits = nw;
  while (bits) {
    const int l = __builtin_ctzll(bits);
    bits &= bits - 1;
    P.depth[(int64_t)l * P.n + v] = it1 - start[l];
  }
  return atomicOr(&Fn[v], nw) == 0ull;
}

// ---- push expansion (scan-gather for low degree, descriptors for high)
__device__ void push_expand(const MsParams& P, const MsState& S, int32_t k, int64_t qlen,
                            ull qbase, ull dbase, Lds& L, ull& got, uint32_t& ecnt, uint32_t& vcnt) {
  const int lane = fg_lane();
  const int wid = threadIdx.x / FG_WAVE;
  const int32_t* Qin = P.q[S.qsel];
  int32_t* Qout = P.q[S.qsel ^ 1];
  ull* Fc = P.F[S.fsel];
  ull* Fn = P.F[S.fsel ^ 1];
  int32_t* sc = L.w_sc[wid];
  int32_t* su = L.w_u[wid];
  int32_t* sb = L.w_b[wid];
  ull* sf = L.w_f[wid];
  const int32_t it1 = S.it + 1;
  CtrSlot& C = P.ctl->slot[k & 1];
  WaveStage<int32_t, STAGE> st{L.stage[wid], 0};
  WaveStage<int4, DSTAGE> dst{L.dstage[wid], 0};
  const int64_t gw = (int64_t)blockIdx.x * PWAVES + wid;
  const int64_t W = (int64_t)gridDim.x * PWAVES;
  for (int64_t base = gw * FG_WAVE; base < qlen; base += W * FG_WAVE) {
    const int64_t i = base + lane;
    int32_t u = 0, b = 0, deg = 0;
    ull fu = 0;
    if (i < qlen) {
      u = Qin[i];
      b = P.off[u];
      deg = P.off[u + 1] - b;
      fu = Fc[u];
      fg_st_shared(&Fc[u], 0ull);  // only this thread reads u's word in this iteration
      if (fu == 0ull) deg = 0;  // listed but without lanes
      ecnt += (uint32_t)deg;
      vcnt += fu != 0ull;
    }
    const bool big = deg >= P.big_deg;
    const int32_t nd = big ? (deg + CH - 1) / CH : 0;
    const int32_t ndi = fg_wave_incl_scan(nd);
    const int32_t ND = __shfl(ndi, FG_WAVE - 1, FG_WAVE);
    if (ND > 0) {
      wave_lds_fence();
      sc[lane] = ndi - nd;
      su[lane] = u;
      sb[lane] = b;
      sf[lane] = fu;
      wave_lds_fence();
      for (int32_t t0 = 0; t0 < ND; t0 += FG_WAVE) {
        const int32_t t = t0 + lane;
        int4 dsc = make_int4(0, 0, 0, 0);
        if (t < ND) {
          const int32_t j = upper_idx(sc, FG_WAVE, t);
          dsc = make_desc(su[j], sb[j] + (t - sc[j]) * CH, sf[j]);
        }
        dst.push(t < ND, dsc, &C.desc.v, dbase, P.desc);
      }
    }
    const int32_t d = big ? 0 : deg;
    const int32_t inc = fg_wave_incl_scan(d);
    const int32_t T = __shfl(inc, FG_WAVE - 1, FG_WAVE);
    if (T == 0) continue;
    wave_lds_fence();
    sc[lane] = inc - d;
    su[lane] = u;
    sb[lane] = b;
    sf[lane] = fu;
    wave_lds_fence();
    for (int32_t t0 = 0; t0 < T; t0 += FG_WAVE) {
      const int32_t t = t0 + lane;
      bool first = false;
      int32_t v = 0;
      if (t < T) {
        const int32_t j = upper_idx(sc, FG_WAVE, t);
        v = P.col[sb[j] + (t - sc[j])];
        first = claim(P, Fn, v, sf[j], it1, L.start, got);
      }
      st.push(first, v, &C.q.v, qbase, Qout);
    }
  }
  st.flush(&C.q.v, qbase, Qout);
  dst.flush(&C.desc.v, dbase, P.desc);
}

__device__ void push_desc(const MsParams& P, const MsState& S, int32_t k, int64_t ndesc,
                          ull qbase, Lds& L, ull& got) {
  const int lane = fg_lane();
  const int wid = threadIdx.x / FG_WAVE;
  const int64_t gw = (int64_t)blockIdx.x * PWAVES + wid;
  const int64_t W = (int64_t)gridDim.x * PWAVES;
  int32_t* Qout = P.q[S.qsel ^ 1];
  ull* Fn = P.F[S.fsel ^ 1];
  const int32_t it1 = S.it + 1;
  CtrSlot& C = P.ctl->slot[k & 1];
  WaveStage<int32_t, STAGE> st{L.stage[wid], 0};
  for (int64_t i = gw; i < ndesc; i += W) {
    const int4 dsc = P.desc[i];
    const int32_t u = dsc.x;
    const int32_t e_end = P.off[u + 1];
    const int32_t e1 = dsc.y + CH < e_end ? dsc.y + CH : e_end;
    const ull fu = desc_lanes(dsc);
    int32_t vv[CH / FG_WAVE];
#pragma unroll
    for (int r = 0; r < CH / FG_WAVE; ++r) {
      const int32_t e = dsc.y + r * FG_WAVE + lane;
      vv[r] = e < e1 ? P.col[e] : -1;
    }
#pragma unroll
    for (int r = 0; r < CH / FG_WAVE; ++r) {
      const int32_t v = vv[r];
      const bool first = v >= 0 && claim(P, Fn, v, fu, it1, L.start, got);
      st.push(first, v, &C.q.v, qbase, Qout);
    }
  }
  st.flush(&C.q.v, qbase, Qout);
}


// ---------------------------------------------------------------- team mode
//
// Push levels of medium frontiers (at least TEAM_MIN_Q and at most
// QCAP * T / 2 vertices, mean degree <= LDS_MEAN_DEG, degree sum <= team_e)
// run as a team of T workgroups from LDS queues, as in the single-source
// kernels: each member keeps its share of the active vertices as (vertex,
// first edge, end edge) in LDS, takes a vertex's lanes with an agent-scope
// exchange of its current word (the word is complete: all claims of the
// previous level came before the team exchange), claims the lanes of each
// neighbour with atomicOr on visit (writing their depths), and appends a
// neighbour whose next word was 0 (offsets loaded alongside) to its next
// LDS queue.  Members share only visit and the frontier words, touched by
// atomics.  Per level the members add one packed word to the level's team
// word and poll it; exact per-member counts (tagged records) are read when
// the episode ends or a share is uneven.  On exit the members write their
// LDS queues to the global queue and meet at a team barrier; the live lanes
// are taken as before the episode (lanes only finish; the next full-grid
// level recomputes them) unless the frontier emptied.  The other
// workgroups sleep.
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

__device__ __forceinline__ ull team_clear_next(const MsParams& P, uint32_t level) {
  if (blockIdx.x == 0 && threadIdx.x == 0)
    return __hip_atomic_exchange(&P.ctl->team_word[(level + 1) % 3].v, 0ull, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
  return 0;
}

__device__ bool team_fast(const MsParams& P, Lds& L, uint32_t T, uint32_t level, int32_t bcnt,
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
    L.flag = bad;
  }
  __syncthreads();
  return L.flag == 0;
}

__device__ bool team_records(const MsParams& P, Lds& L, uint32_t T, uint32_t seq, int odd) {
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

// Claim of team mode: the lanes of `fu` not yet in visit[v] (agent-scope
// atomics only).  Returns true when v's next word was 0.
__device__ __forceinline__ bool claim_team(const MsParams& P, ull* Fn, int32_t v, ull fu,
                                           int32_t it1, const int32_t* start, ull& got) {
  const ull nb = fu & ~__hip_atomic_load(&P.visit[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (!nb) return false;
  const ull nw = nb & ~atomicOr(&P.visit[v], nb);
  if (!nw) return false;
  got |= nw;
  ull bits = nw;
  while (bits) {
    const int l = __builtin_ctzll(bits);
    bits &= bits - 1;
    P.depth[(int64_t)l * P.n + v] = it1 - start[l];
  }
  return atomicOr(&Fn[v], nw) == 0ull;
}

// Runs push levels as a team of T members while the frontier suits the
// mode, at most `budget` levels.  Returns false on a device error.
// *levels = levels run; *handback = 1 when the frontier met on entry does
// not suit the mode.  On return S describes the frontier in Q[qsel] (and
// S.live the lanes of its words).
__device__ bool team_levels(const MsParams& P, MsState& S, Lds& L, uint32_t T, TeamSync& ts,
                            TeamBases& tb, int32_t budget, int32_t kbase, int32_t* levels,
                            int* handback, uint32_t& ecnt, uint32_t& vcnt) {
  const int tid = threadIdx.x;
  const int lane = fg_lane();
  ull* ovf = &P.ctl->team_ovf.v;
  ull ovf_base = tb.ovf;
  int cur = 0, ci = 0, ni = 1, ri = 2;
  *levels = 0;
  *handback = 0;
  // my even slice of the global frontier -> LDS queue `cur`
  {
    const int32_t* Qg = P.q[S.qsel];
    const int64_t lo = S.qlen * blockIdx.x / T, hi = S.qlen * (blockIdx.x + 1) / T;
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
      L.lq_big[ni] = 0;
    }
    const int32_t bsd = fg_block_sum<PB>(sd, L.red32);
    if (!team_fast(P, L, T, tb.levels, cnt, bsd, QCAP, team_clear_next(P, tb.levels)))
      return false;
    tb.levels++;
    const int64_t qd = fg_uni(L.tsum[1]);
    if (qd > LDS_MEAN_DEG * S.qlen || qd > P.team_e) {
      *handback = 1;  // nothing changed; the queue and the words are intact
      return true;
    }
    __syncthreads();
  }
  for (;;) {
    int32_t* Qo = P.q[S.qsel ^ 1];
    const int nxt = cur ^ 1;
    const int32_t cnt = L.lq_cnt[ci];
    const ull cleared2 = team_clear_next(P, tb.levels);
    if (tid == 0) {
      L.lq_cnt[ri] = 0;
      L.lq_deg[ri] = 0;
      L.lq_big[ri] = 0;
    }
    ull* Fc = P.F[S.fsel];
    ull* Fn = P.F[S.fsel ^ 1];
    const int32_t it1 = S.it + 1;
    ull got = 0;
    bool big = false;
    // vertices of degree <= TPV: TPV lanes per vertex, one edge each; the
    // first takes (and clears) the vertex's current word
    for (int32_t c0 = 0; c0 < cnt; c0 += PB / TPV) {
      const int32_t i = c0 + tid / TPV;
      const int32_t j = tid % TPV;
      int32_t u = 0, b = 0, d = 0;
      ull fu = 0;
      if (i < cnt) {
        u = L.lq_v[cur][i];
        b = L.lq_b[cur][i];
        d = L.lq_e[cur][i] - b;
        if (j == 0 && d <= TPV) {
          // vertices of degree > TPV take their word in the scan-gather below
          fu = __hip_atomic_exchange(&Fc[u], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ecnt += (uint32_t)d;
          vcnt += fu != 0ull;
        }
      }
      // the word to the vertex's other lanes (the first lane of the group)
      fu = __shfl(fu, (int)(threadIdx.x % FG_WAVE) & ~(TPV - 1), FG_WAVE);
      big |= d > TPV;
      bool won = false;
      int32_t v = 0, vb = 0, ve = 0;
      if (d <= TPV && j < d && fu) {
        v = P.col[b + j];
        vb = P.off[v];
        ve = P.off[v + 1];
        won = claim_team(P, Fn, v, fu, it1, L.start, got);
      }
      const int32_t pos = wave_reserve(won ? 1 : 0, &L.lq_cnt[ni]);
      const int32_t wdeg = fg_wave_sum(won ? ve - vb : 0);
      if (lane == 0 && wdeg) atomicAdd(&L.lq_deg[ni], wdeg);
      wave_put(L, nxt, won, pos, v, vb, ve, Qo, ovf, ovf_base);
    }
    if (big) L.lq_big[ni] = 1;
    __syncthreads();
    if (L.lq_big[ni]) {
      // vertices of degree > TPV: block scan-gather over their edges
      for (int32_t c0 = 0; c0 < cnt; c0 += PB) {
        const int32_t i = c0 + tid;
        int32_t u = 0, b = 0, d = 0;
        ull fu = 0;
        if (i < cnt) {
          u = L.lq_v[cur][i];
          b = L.lq_b[cur][i];
          d = L.lq_e[cur][i] - b;
          if (d > TPV) {
            fu = __hip_atomic_exchange(&Fc[u], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ecnt += (uint32_t)d;
            vcnt += fu != 0ull;
          }
        }
        if (d <= TPV || !fu) d = 0;
        int32_t Tn = 0;
        const int32_t ex = fg_block_excl_scan<PB>(d, L.red32, &Tn);
        L.b_sc[tid] = ex;
        L.b_u[tid] = u;
        L.b_b[tid] = b;
        L.b_f[tid] = fu;
        __syncthreads();
        const int32_t nc = cnt - c0 < PB ? cnt - c0 : PB;
        for (int32_t t0 = 0; t0 < Tn; t0 += PB) {
          const int32_t t = t0 + tid;
          bool won = false;
          int32_t v = 0, vb = 0, ve = 0;
          if (t < Tn) {
            const int32_t jj = upper_idx(L.b_sc, nc, t);
            v = P.col[L.b_b[jj] + (t - L.b_sc[jj])];
            vb = P.off[v];
            ve = P.off[v + 1];
            won = claim_team(P, Fn, v, L.b_f[jj], it1, L.start, got);
          }
          const int32_t pos = wave_reserve(won ? 1 : 0, &L.lq_cnt[ni]);
          const int32_t wdeg = fg_wave_sum(won ? ve - vb : 0);
          if (lane == 0 && wdeg) atomicAdd(&L.lq_deg[ni], wdeg);
          wave_put(L, nxt, won, pos, v, vb, ve, Qo, ovf, ovf_base);
        }
        __syncthreads();
      }
    }
    const int32_t bcnt = L.lq_cnt[ni];
    const int32_t bdeg = L.lq_deg[ni];
    if (tid == 0) {
      ull* rr = P.ctl->team_rec[S.it & 1][blockIdx.x];
      const ull tag = (ull)((uint32_t)S.it + 1u) << 32;
      __hip_atomic_store(rr, tag | (uint32_t)bcnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const int64_t lim = (5 * S.qlen / T + 64) / 4;
    if (!team_fast(P, L, T, tb.levels, bcnt, bdeg, (int32_t)(lim < QCAP ? lim : QCAP), cleared2))
      return false;
    tb.levels++;
    const int64_t nq = fg_uni(L.tsum[0]);
    const int64_t nqdeg = fg_uni(L.tsum[1]);
    const int64_t nflag = fg_uni(L.tsum[2]);
    S.it = it1;
    S.qlen = nq;
    S.fsel ^= 1;
    (*levels)++;
    bool stay = nq >= TEAM_MIN_Q && nqdeg <= LDS_MEAN_DEG * nq && nqdeg <= P.team_e &&
                nq <= (int64_t)QCAP * T / 2 && nq <= P.n / P.pull_div && *levels < budget;
    int64_t nover = bcnt > QCAP ? bcnt - QCAP : 0, before = 0;
    bool rebalance = false;
    if (!stay || nflag) {
      if (!team_records(P, L, T, (uint32_t)S.it, (S.it - 1) & 1)) return false;
      nover = fg_uni(L.tsum[3]);
      before = fg_uni(L.tsum[4]);
      stay = stay && fg_uni(L.tsum[2]) == 0;
      rebalance = stay && 4 * fg_uni(L.tsum[5]) * (int64_t)T > 5 * nq + 64 * (int64_t)T;
    }
    if (!stay || rebalance) {
      // global queue: the overflow entries, then every member's LDS queue
      // in member order
      const int32_t nloc = bcnt < QCAP ? bcnt : QCAP;
      int32_t* dst = Qo + nover + before;
      for (int32_t i = tid; i < nloc; i += PB) dst[i] = L.lq_v[nxt][i];
      ovf_base += (ull)nover;
      tb.ovf = ovf_base;
      // the live word of the next full-grid level starts at zero (cleared
      // before the barrier, which every member passes before using it)
      if (!stay && blockIdx.x == 0 && threadIdx.x == 0)
        __hip_atomic_store(&P.ctl->livew[(kbase + *levels) % 3].v, 0ull, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      if (!ts.sync(&L.flag)) return false;
      S.qsel ^= 1;
      if (!stay) {
        if (nq == 0) S.live = 0ull;
        return true;
      }
      // reload an even share from the global queue
      {
        const int32_t* Qg = P.q[S.qsel];
        const int64_t lo = S.qlen * blockIdx.x / T, hi = S.qlen * (blockIdx.x + 1) / T;
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
    }
    cur = nxt;
    const int t3 = ci;
    ci = ni;
    ni = ri;
    ri = t3;
  }
}

// TEAM = false compiles the kernel without the team episodes, whose code
// raises the register pressure (and the spills) of the whole kernel.
template <bool TEAM>
__global__ __launch_bounds__(PB) void msbfs_persistent(MsParams P) {
  __shared__ Lds L;
  fg_grid_sync gs{P.ctl->bar, gridDim.x, 0u};
  const int64_t tid = (int64_t)blockIdx.x * PB + threadIdx.x;
  const int64_t nth = (int64_t)gridDim.x * PB;
  const int lane = fg_lane();
  const int wid = threadIdx.x / FG_WAVE;
  const int64_t gw = (int64_t)blockIdx.x * PWAVES + wid;
  const int64_t W = (int64_t)gridDim.x * PWAVES;
  MsState S = *P.state;  // read by every workgroup before anyone writes it
  bool ok = gs.sync(&L.flag);
  // per-parity bases of the monotone counters, as scalars (a dynamically
  // indexed array would live in scratch memory)
  ull qb0 = 0, qb1 = 0, db0 = 0, db1 = 0, cb0 = 0, cb1 = 0;

  // ---- admissions: clear reused lanes, fill their depth rows, seed sources
  if (ok && P.npend > 0) {
    ull mask = 0;
    for (int i = 0; i < P.npend; ++i) mask |= 1ull << P.pend_lane[i];
    const ull reused = mask & S.used;
    if (reused) {
      for (int64_t v = tid; v < P.n; v += nth) {
        P.visit[v] &= ~reused;
        P.F[0][v] &= ~reused;
        P.F[1][v] &= ~reused;
      }
    }
    for (int i = 0; i < P.npend; ++i) {
      int32_t* row = P.depth + (int64_t)P.pend_lane[i] * P.n;
      for (int64_t v = tid; v < P.n; v += nth) row[v] = -1;
    }
    ok = gs.sync(&L.flag);
    if (ok && tid == 0) {
      MsState* st = P.state;
      int64_t ql = S.qlen;
      for (int i = 0; i < P.npend; ++i) {
        const int32_t l = P.pend_lane[i], s = P.pend_src[i];
        const ull bit = 1ull << l;
        P.visit[s] |= bit;
        if (S.mode == 0 && P.F[S.fsel][s] == 0ull) P.q[S.qsel][ql++] = s;
        P.F[S.fsel][s] |= bit;
        P.depth[(int64_t)l * P.n + s] = 0;
        st->start[l] = S.it;
      }
      if (S.mode == 1) ql = S.qlen + P.npend;  // pull: an estimate is enough
      S.qlen = ql;
      S.live |= mask;
      S.used |= mask;
      P.ctl->pub_qlen = ql;
      P.ctl->pub_live = S.live;
    }
    ok = ok && gs.sync(&L.flag);
    S.qlen = P.ctl->pub_qlen;
    S.live = P.ctl->pub_live;
    S.used |= mask;
  }

  if (threadIdx.x < MAXL) L.start[threadIdx.x] = P.state->start[threadIdx.x];
  __syncthreads();
  uint32_t ecnt = 0, vcnt = 0;  // per-thread counts stay far below 2^32
  TeamSync ts{&P.ctl->team_arrive, P.ctl->bar + FG_BAR_STRIDE, (uint32_t)(P.team > 1 ? P.team : 1),
              0u};
  TeamBases tb = {};
  uint32_t sm_seen = 0;
  uint32_t ack_need = 0;  // workgroup 0: acknowledgements of the hand-backs so far
  int force_full = 0;
  for (int32_t k = 0; ok && k < P.k_iters && S.live != 0ull; ++k) {
    const int32_t it1 = S.it + 1;
    const bool want_pull = S.mode == 0 ? S.qlen > P.n / P.pull_div : S.qlen >= P.n / P.push_div;
    // ---- push levels of medium frontiers as a team (the others sleep)
    if (TEAM && !force_full && S.mode == 0 && !want_pull && P.team > 1 && S.qlen >= TEAM_MIN_Q &&
        S.qlen <= (int64_t)QCAP * P.team / 2) {
      sm_seen++;
      int32_t nl = 0;
      if (blockIdx.x < (uint32_t)P.team) {
        int hb = 0;
        if (!team_levels(P, S, L, (uint32_t)P.team, ts, tb, P.k_iters - k, k, &nl, &hb, ecnt,
                         vcnt))
          ok = false;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
          MsCtl* c = P.ctl;
          // every waiter of the previous hand-back has read it (on a
          // timeout the abort flag is set and every wait ends)
          L.ackbad = !fg_wait_geq(&c->sm_ack, ack_need, c->bar + FG_BAR_STRIDE, 1);
          // a failed wait has set the abort flag: publish nothing (a slow
          // waiter may still be reading the previous hand-off); the waiters
          // see the flag and leave
          if (!L.ackbad) {
            c->pub_it = S.it;
            c->pub_qsel = S.qsel;
            c->pub_fsel = S.fsel;
            c->pub_levels = nl;
            c->pub_force = hb;
            c->pub_tqlen = S.qlen;
            c->pub_tlive = S.live;
            __hip_atomic_fetch_add(&c->sm_signal, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
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
          const int bad = !fg_wait_geq(&P.ctl->sm_signal, sm_seen, P.ctl->bar + FG_BAR_STRIDE, 4096);
          L.flag = bad;
          if (!bad) {
            const MsCtl* c = P.ctl;
            L.bcast[0] = c->pub_it;
            L.bcast[1] = c->pub_qsel | ((int64_t)c->pub_fsel << 8) | ((int64_t)c->pub_force << 16);
            L.bcast[2] = c->pub_levels;
            L.bcast[3] = c->pub_tqlen;
            L.redu[0] = c->pub_tlive;
            fg_handoff_ack(&P.ctl->sm_ack);
          }
        }
        __syncthreads();
        if (L.flag) {
          ok = false;
          break;
        }
        S.it = (int32_t)L.bcast[0];
        S.qsel = (int32_t)(L.bcast[1] & 0xff);
        S.fsel = (int32_t)((L.bcast[1] >> 8) & 0xff);
        force_full = (int)((L.bcast[1] >> 16) & 0xff);
        nl = (int32_t)L.bcast[2];
        S.qlen = L.bcast[3];
        S.live = L.redu[0];
        __syncthreads();
      }
      k += nl - 1;  // the loop adds the last one
      continue;
    }
    force_full = 0;
    CtrSlot& C = P.ctl->slot[k & 1];
    const bool odd = k & 1;
    const ull msk = 0ull - (ull)odd;
    ull qbp = (qb1 & msk) | (qb0 & ~msk);
    ull dbp = (db1 & msk) | (db0 & ~msk);
    ull cbp = (cb1 & msk) | (cb0 & ~msk);
    ull* livew = &P.ctl->livew[k % 3].v;
    if (tid == 0)
      __hip_atomic_store(&P.ctl->livew[(k + 1) % 3].v, 0ull, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    if (!want_pull && S.mode == 1) {
      // pull -> push: list the active vertices, clear the next F array
      const ull* Fc = P.F[S.fsel];
      ull* Fn = P.F[S.fsel ^ 1];
      WaveStage<int32_t, STAGE> st{L.stage[wid], 0};
      for (int64_t v0 = gw * FG_WAVE; v0 < P.n; v0 += W * FG_WAVE) {
        const int64_t v = v0 + lane;
        bool act = false;
        if (v < P.n) {
          act = Fc[v] != 0ull;
          fg_st_shared(&Fn[v], 0ull);
        }
        st.push(act, (int32_t)v, &C.cnt.v, cbp, P.q[S.qsel]);
      }
      st.flush(&C.cnt.v, cbp, P.q[S.qsel]);
      if (!(ok = gs.sync_acquire(&L.flag))) break;
      const ull ct = fg_atomic_load_u64(&C.cnt.v);
      S.qlen = (int64_t)(ct - cbp);
      cbp = ct;
      S.mode = 0;
    }
    if (want_pull) {
      // ---- pull: lane per vertex, early exit when every wanted lane is
      // seen.  The first four neighbours come from the head table (one
      // coalesced load); lists of up to 32 go on four entries at a time,
      // longer ones are scanned by the whole wave, 64 entries per step.
      const ull* Fc = P.F[S.fsel];
      ull* Fn = P.F[S.fsel ^ 1];
      int32_t* Qlong = P.q[S.qsel ^ 1];  // queues are idle while pulling
      ull lor = 0;
      int32_t act = 0;
      for (int64_t v0 = gw * FG_WAVE; v0 < P.n; v0 += W * FG_WAVE) {
        const int64_t v = v0 + lane;
        ull vis = ~0ull, nw = 0;
        int32_t b = 0, e = 0;
        int4 hd = make_int4(0, 0, 0, 0);
        if (v < P.n) {
          vis = P.visit[v];
          b = P.off[v];
          e = P.off[v + 1];
          hd = P.head[v];
        }
        const ull want = S.live & ~vis;
        vcnt += v < P.n;
        if (want && e > b) {
          const int32_t d = e - b;
          ecnt += (uint32_t)(d < 4 ? d : 4);
          const ull f0 = Fc[hd.x], f1 = Fc[hd.y], f2 = Fc[hd.z], f3 = Fc[hd.w];
          nw = (f0 | (d > 1 ? f1 : 0ull) | (d > 2 ? f2 : 0ull) | (d > 3 ? f3 : 0ull)) & want;
        }
        bool shortl = want && nw != want && e - b > 4 && e - b <= 32;
        for (int32_t i0 = 4; i0 < 32 && __ballot(shortl); i0 += 4) {
          if (shortl) {
            const int32_t i = b + i0, l = e - 1;
            const int32_t u0 = P.col[i], u1 = P.col[i + 1 < l ? i + 1 : l],
                          u2 = P.col[i + 2 < l ? i + 2 : l], u3 = P.col[i + 3 < l ? i + 3 : l];
            const ull g = Fc[u0] | Fc[u1] | Fc[u2] | Fc[u3];
            ecnt += (uint32_t)(e - i < 4 ? e - i : 4);
            nw |= g & want;
            if (nw == want || i + 4 >= e) shortl = false;
          }
        }
        const bool lng = want && nw != want && e - b > LONG_PULL;
        if (lng) {
          // listed for the chunked scan; the lanes found so far stay in Fn
          const int32_t nch = (e - b - 4 + CH - 1) / CH;
          fg_st_shared(&Qlong[atomicAdd(&C.q.v, 1ull) - qbp], (int32_t)v);
          const int64_t d0 = (int64_t)(atomicAdd(&C.desc.v, (ull)nch) - dbp);
          for (int32_t c = 0; c < nch; ++c)
            fg_st_shared(&P.desc[d0 + c], make_int4((int32_t)v, b + 4 + c * CH, 0, 0));
        }
        uint64_t pend = __ballot(want && nw != want && e - b > 32 && !lng);
        while (pend) {
          const int l = __builtin_ctzll(pend);
          pend &= pend - 1;
          const int32_t lb = __builtin_amdgcn_readlane(b, l) + 4;
          const int32_t le = __builtin_amdgcn_readlane(e, l);
          const ull lw = fg_readlane64(want, l);
          ull acc = fg_readlane64(nw, l);
          for (int32_t i0 = lb; i0 < le && (acc & lw) != lw; i0 += FG_WAVE) {
            const int32_t i = i0 + lane;
            ull x = 0;
            if (i < le) x = Fc[P.col[i]] & lw;
            if (lane == 0) ecnt += (uint32_t)(le - i0 < FG_WAVE ? le - i0 : FG_WAVE);
            acc |= fg_wave_or64(x);
          }
          if (lane == l) nw = acc & lw;
        }
        if (v < P.n) {
          if (nw && !lng) fg_st_shared(&P.visit[v], vis | nw);
          fg_st_shared(&Fn[v], nw);
        }
        if (lng) nw = 0;  // finished after the chunked scan
        // depths, lane by lane over the wave's union: coalesced row stores
        ull uni = fg_wave_or64(nw);
        while (uni) {
          const int l = __builtin_ctzll(uni);
          uni &= uni - 1;
          if ((nw >> l) & 1ull) P.depth[(int64_t)l * P.n + v] = it1 - L.start[l];
        }
        lor |= nw;
        act += nw != 0ull;
      }
      {
        const ull bor = block_or(lor, L.redu);
        const int32_t bact = fg_block_sum<PB>(act, L.red32);
        if (threadIdx.x == 0) {
          if (bor) atomicOr(livew, bor);
          if (bact) atomicAdd(&C.cnt.v, (ull)bact);
        }
      }
      if (!(ok = gs.sync_acquire(&L.flag))) break;
      // ---- listed long vertices (if any): chunked scan by every wave, then
      // finalise; without them the level costs one grid barrier as before
      {
        const ull lt = fg_atomic_load_u64(&C.q.v);
        const ull dt = fg_atomic_load_u64(&C.desc.v);
        const int64_t nlong = (int64_t)(lt - qbp), nch = (int64_t)(dt - dbp);
        qbp = lt;
        dbp = dt;
        if (nch > 0) {
          for (int64_t i = gw; i < nch; i += W) {
            const int4 dsc = P.desc[i];
            const int32_t v = dsc.x;
            const ull want = S.live & ~P.visit[v];
            const ull cur = fg_uni(__hip_atomic_load(&Fn[v], __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT));
            if ((cur & want) == want) continue;  // every wanted lane already found
            const int32_t e1 = min(dsc.y + CH, P.off[v + 1]);
            if (lane == 0) ecnt += (uint32_t)(e1 - dsc.y);
            ull x = 0;
#pragma unroll
            for (int r = 0; r < CH / FG_WAVE; ++r) {
              const int32_t i2 = dsc.y + r * FG_WAVE + lane;
              if (i2 < e1) x |= Fc[P.col[i2]];
            }
            x = fg_wave_or64(x & want);
            if (lane == 0 && (x & ~cur)) atomicOr(&Fn[v], x);
          }
          if (!(ok = gs.sync_acquire(&L.flag))) break;
          ull lor2 = 0;
          int32_t act2 = 0;
          for (int64_t i = tid; i < nlong; i += nth) {
            const int32_t v = Qlong[i];
            const ull vis = P.visit[v];
            const ull nw = Fn[v] & S.live & ~vis;
            fg_st_shared(&Fn[v], nw);
            if (nw) {
              fg_st_shared(&P.visit[v], vis | nw);
              write_depths(P, v, nw, it1);
            }
            lor2 |= nw;
            act2 += nw != 0ull;
          }
          const ull bor = block_or(lor2, L.redu);
          const int32_t bact = fg_block_sum<PB>(act2, L.red32);
          if (threadIdx.x == 0) {
            if (bor) atomicOr(livew, bor);
            if (bact) atomicAdd(&C.cnt.v, (ull)bact);
          }
          if (!(ok = gs.sync_acquire(&L.flag))) break;
        }
      }
      const ull lv = fg_atomic_load_u64(livew);
      const ull ct = fg_atomic_load_u64(&C.cnt.v);
      S.qlen = (int64_t)(ct - cbp);
      cbp = ct;
      S.live = lv;
      S.fsel ^= 1;
      S.mode = 1;
    } else {
      // ---- push
      ull got = 0;
      push_expand(P, S, k, S.qlen, qbp, dbp, L, got, ecnt, vcnt);
      {
        const ull bor = block_or(got, L.redu);
        if (threadIdx.x == 0 && bor) atomicOr(livew, bor);
      }
      if (!(ok = gs.sync_acquire(&L.flag))) break;
      const ull dt = fg_atomic_load_u64(&C.desc.v);
      const int64_t ndesc = (int64_t)(dt - dbp);
      if (ndesc > 0) {
        ull got2 = 0;
        push_desc(P, S, k, ndesc, qbp, L, got2);
        const ull bor = block_or(got2, L.redu);
        if (threadIdx.x == 0 && bor) atomicOr(livew, bor);
        if (!(ok = gs.sync_acquire(&L.flag))) break;
      }
      dbp = dt;
      const ull qt = fg_atomic_load_u64(&C.q.v);
      const int64_t qn = (int64_t)(qt - qbp);
      qbp = qt;
      S.live = fg_atomic_load_u64(livew);
      S.qlen = qn;
      S.qsel ^= 1;
      S.fsel ^= 1;
      S.mode = 0;
    }
    qb1 = (qbp & msk) | (qb1 & ~msk);
    qb0 = (qb0 & msk) | (qbp & ~msk);
    db1 = (dbp & msk) | (db1 & ~msk);
    db0 = (db0 & msk) | (dbp & ~msk);
    cb1 = (cbp & msk) | (cb1 & ~msk);
    cb0 = (cb0 & msk) | (cbp & ~msk);
    S.it = it1;
  }
  {
    // work counters: every workgroup adds its own (the host reads them after
    // the launch)
    const int64_t be = fg_block_sum<PB>((int64_t)ecnt, L.red);
    const int64_t bv = fg_block_sum<PB>((int64_t)vcnt, L.red);
    if (threadIdx.x == 0) {
      if (be) atomicAdd(&P.state->edges, (ull)be);
      if (bv) atomicAdd(&P.state->verts, (ull)bv);
    }
  }
  if (tid == 0) {
    MsState* st = P.state;
    st->it = S.it;
    st->mode = S.mode;
    st->qsel = S.qsel;
    st->fsel = S.fsel;
    st->qlen = S.qlen;
    st->live = ok ? S.live : 0ull;
    st->used = S.used;
    if (!ok) st->aborted = 1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t done = __hip_atomic_fetch_add(&P.ctl->exit_count, 1u, __ATOMIC_ACQ_REL,
                                                 __HIP_MEMORY_SCOPE_AGENT);
    L.flag = done == gridDim.x - 1;
  }
  __syncthreads();
  if (L.flag) {
    uint32_t* w = (uint32_t*)P.ctl;
    for (int i = threadIdx.x; i < (int)(sizeof(MsCtl) / 4); i += PB) w[i] = 0u;
  }
}

struct MsLayout {
  MsState* state;
  MsCtl* ctl;
  ull* visit;
  ull* F[2];
  int32_t* q[2];
  int4* desc;
  int32_t* depth;
  size_t bytes;
};

MsLayout ms_layout(const fg_graph* g, int32_t lanes, void* ws) {
  fg_carver c(ws);
  MsLayout L;
  L.state = c.take<MsState>(1);
  L.ctl = c.take<MsCtl>(1);
  L.visit = c.take<ull>(g->n);
  L.F[0] = c.take<ull>(g->n);
  L.F[1] = c.take<ull>(g->n);
  // + 64: admissions list their sources even when a reused lane's cleared
  // bits leave listed vertices without lanes
  L.q[0] = c.take<int32_t>((size_t)g->n + MAXL);
  L.q[1] = c.take<int32_t>((size_t)g->n + MAXL);
  L.desc = c.take<int4>((size_t)(g->m / CH) + (size_t)g->n + 64);
  L.depth = c.take<int32_t>((size_t)lanes * (size_t)g->n);
  L.bytes = c.used;
  return L;
}

int g_ms_occ[64];

}  // namespace

struct fg_msbfs {
  const fg_graph* g = nullptr;
  int32_t lanes = 0;
  MsLayout lay;
  int32_t npend = 0;
  int32_t pend_lane[MAXL];
  int32_t pend_src[MAXL];
  uint64_t admitted = 0;  // lanes holding a query (host view)
  fg_msbfs_opts opts;
};

size_t fg_msbfs_workspace_bytes(const fg_graph* g, int32_t lanes) {
  return ms_layout(g, lanes, nullptr).bytes;
}

extern "C" void fg_msbfs_opts_default(fg_msbfs_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
}

extern "C" fg_status fg_msbfs_open(const fg_graph* g, int32_t lanes, void* ws, size_t ws_bytes,
                                   const fg_msbfs_opts* opts, void* stream, fg_msbfs** out) {
  if (!out) return fg_set_error(FG_EINVAL, "fg_msbfs_open: out is NULL");
  *out = nullptr;
  if (!g || !ws) return fg_set_error(FG_EINVAL, "fg_msbfs_open: NULL graph or workspace");
  if (lanes < 1 || lanes > MAXL)
    return fg_set_error(FG_EINVAL, "fg_msbfs_open: lanes=%d outside [1, 64]", lanes);
  MsLayout lay = ms_layout(g, lanes, ws);
  FG_CHECK_WS_ALIGN(ws, "fg_msbfs_open");
  if (ws_bytes < lay.bytes)
    return fg_set_error(FG_ENOMEM, "fg_msbfs_open: workspace of %zu bytes < required %zu",
                        ws_bytes, lay.bytes);
  hipStream_t s = (hipStream_t)stream;
  // fresh state: visit / F all zero, no lanes
  FG_HIP_TRY(hipMemsetAsync(lay.state, 0, sizeof(MsState), s));
  FG_HIP_TRY(hipMemsetAsync(lay.ctl, 0, sizeof(MsCtl), s));
  FG_HIP_TRY(hipMemsetAsync(lay.visit, 0, sizeof(ull) * (size_t)g->n, s));
  FG_HIP_TRY(hipMemsetAsync(lay.F[0], 0, sizeof(ull) * (size_t)g->n, s));
  FG_HIP_TRY(hipMemsetAsync(lay.F[1], 0, sizeof(ull) * (size_t)g->n, s));
  fg_msbfs* b = new fg_msbfs();
  b->g = g;
  b->lanes = lanes;
  b->lay = lay;
  if (opts) b->opts = *opts; else fg_msbfs_opts_default(&b->opts);
  *out = b;
  return FG_OK;
}

extern "C" fg_status fg_msbfs_close(fg_msbfs* b) {
  delete b;
  return FG_OK;
}

extern "C" fg_status fg_msbfs_admit(fg_msbfs* b, int32_t lane, int32_t src) {
  if (!b) return fg_set_error(FG_EINVAL, "fg_msbfs_admit: batch is NULL");
  if (lane < 0 || lane >= b->lanes)
    return fg_set_error(FG_EINVAL, "fg_msbfs_admit: lane=%d outside [0, %d)", lane, b->lanes);
  if (src < 0 || src >= b->g->n)
    return fg_set_error(FG_EINVAL, "fg_msbfs_admit: src=%d outside [0, %d)", src, b->g->n);
  for (int i = 0; i < b->npend; ++i)
    if (b->pend_lane[i] == lane)
      return fg_set_error(FG_EINVAL, "fg_msbfs_admit: lane %d already pending", lane);
  b->pend_lane[b->npend] = lane;
  b->pend_src[b->npend] = src;
  b->npend++;
  b->admitted |= 1ull << lane;
  return FG_OK;
}

extern "C" fg_status fg_msbfs_step(fg_msbfs* b, int32_t k_iters, void* stream) {
  if (!b) return fg_set_error(FG_EINVAL, "fg_msbfs_step: batch is NULL");
  if (k_iters < 0) return fg_set_error(FG_EINVAL, "fg_msbfs_step: negative k_iters");
  int dev = 0;
  FG_HIP_TRY(hipGetDevice(&dev));
  fg_device_props pr = fg_props(dev);
  if (!pr.coop) return fg_set_error(FG_EUNSUPPORTED, "fg_msbfs_step: no cooperative launch");
  if (dev >= 0 && dev < 64 && g_ms_occ[dev] == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, msbfs_persistent<true>, PB, 0) !=
            hipSuccess ||
        nb < 1)
      nb = 1;
    g_ms_occ[dev] = nb;
  }
  int bpc = (dev >= 0 && dev < 64) ? g_ms_occ[dev] : 1;
  if (bpc > 2) bpc = 2;
  if (b->opts.blocks_per_cu > 0 && b->opts.blocks_per_cu < bpc) bpc = b->opts.blocks_per_cu;
  const fg_graph* g = b->g;
  MsParams P;
  memset(&P, 0, sizeof(P));
  P.off = g->off;
  P.col = g->col;
  P.head = g->head;
  P.n = g->n;
  P.m = g->m;
  P.lanes = b->lanes;
  P.visit = b->lay.visit;
  P.F[0] = b->lay.F[0];
  P.F[1] = b->lay.F[1];
  P.q[0] = b->lay.q[0];
  P.q[1] = b->lay.q[1];
  P.desc = b->lay.desc;
  P.depth = b->lay.depth;
  P.state = b->lay.state;
  P.ctl = b->lay.ctl;
  P.k_iters = k_iters;
  P.npend = b->npend;
  for (int i = 0; i < b->npend; ++i) {
    P.pend_lane[i] = b->pend_lane[i];
    P.pend_src[i] = b->pend_src[i];
  }
  P.big_deg = b->opts.big_degree > 0 ? b->opts.big_degree : 64;
  P.pull_div = b->opts.pull_div > 0 ? b->opts.pull_div : 64;
  // back to push at the same size as the switch to pull (grid 2048², 64
  // lanes: 105 ms, against 125 ms at n / 512; R-MAT 23 flat at 6.8-7.0 ms)
  P.push_div = b->opts.push_div > 0 ? b->opts.push_div : 64;
  void* args[] = {&P};
  int grid = pr.cus * bpc;
  if (b->opts.grid_blocks > 0 && b->opts.grid_blocks < grid) grid = b->opts.grid_blocks;
  // by default the team kernel runs on graphs of mean degree <= 8 (grids,
  // road-like graphs: long, thin push frontiers)
  const int lanes_in = __builtin_popcountll(b->admitted);
  const bool low_deg = g->m <= (int64_t)TEAM_AUTO_DEG * g->n;
  const int32_t tbo = b->opts.team_blocks;
  P.team = tbo > 1 ? tbo
           : (tbo == 1 || (tbo == 0 && low_deg)) ? (lanes_in >= 4 ? DEF_TEAM_WIDE : DEF_TEAM)
           : 1;
  if (P.team > TEAM_MAX) P.team = TEAM_MAX;
  if (P.team > grid) P.team = grid;
  P.team_e = b->opts.team_edges > 0 ? b->opts.team_edges : DEF_TEAM_E;
  if (P.team_e > TW_CAP - 1) P.team_e = TW_CAP - 1;

  const void* kern = P.team > 1 ? (const void*)msbfs_persistent<true>
                                : (const void*)msbfs_persistent<false>;
  FG_HIP_TRY(hipLaunchCooperativeKernel(kern, dim3(grid), dim3(PB), args, 0,
                                        (hipStream_t)stream));
  b->npend = 0;
  return FG_OK;
}

extern "C" fg_status fg_msbfs_poll(fg_msbfs* b, uint64_t* done_lanes, int32_t* iterations,
                                   void* stream) {
  if (!b) return fg_set_error(FG_EINVAL, "fg_msbfs_poll: batch is NULL");
  MsState hs;
  hipStream_t s = (hipStream_t)stream;
  FG_HIP_TRY(hipMemcpyAsync(&hs, b->lay.state, sizeof(MsState), hipMemcpyDeviceToHost, s));
  FG_HIP_TRY(hipStreamSynchronize(s));
  uint64_t pend = 0;
  for (int i = 0; i < b->npend; ++i) pend |= 1ull << b->pend_lane[i];
  if (done_lanes) *done_lanes = b->admitted & ~hs.live & ~pend;
  if (iterations) *iterations = hs.it;
  if (hs.aborted)
    return fg_set_error(FG_EDEVICE, "fg_msbfs_poll: a step stopped early (barrier abort)");
  return FG_OK;
}

extern "C" fg_status fg_msbfs_counts(fg_msbfs* b, uint64_t* edges, uint64_t* verts, void* stream) {
  if (!b) return fg_set_error(FG_EINVAL, "fg_msbfs_counts: batch is NULL");
  MsState hs;
  hipStream_t s = (hipStream_t)stream;
  FG_HIP_TRY(hipMemcpyAsync(&hs, b->lay.state, sizeof(MsState), hipMemcpyDeviceToHost, s));
  FG_HIP_TRY(hipStreamSynchronize(s));
  if (edges) *edges = hs.edges;
  if (verts) *verts = hs.verts;
  return FG_OK;
}

extern "C" fg_status fg_msbfs_read(fg_msbfs* b, int32_t lane, int32_t* depth, void* stream) {
  if (!b || !depth) return fg_set_error(FG_EINVAL, "fg_msbfs_read: NULL argument");
  if (lane < 0 || lane >= b->lanes)
    return fg_set_error(FG_EINVAL, "fg_msbfs_read: lane=%d outside [0, %d)", lane, b->lanes);
  FG_HIP_TRY(hipMemcpyAsync(depth, b->lay.depth + (size_t)lane * b->g->n,
                            sizeof(int32_t) * (size_t)b->g->n, hipMemcpyDeviceToDevice,
                            (hipStream_t)stream));
  return FG_OK;
}

extern "C" fg_status fg_msbfs_release(fg_msbfs* b, int32_t lane) {
  if (!b) return fg_set_error(FG_EINVAL, "fg_msbfs_release: batch is NULL");
  if (lane < 0 || lane >= b->lanes)
    return fg_set_error(FG_EINVAL, "fg_msbfs_release: lane=%d outside [0, %d)", lane, b->lanes);
  b->admitted &= ~(1ull << lane);
  return FG_OK;
}
