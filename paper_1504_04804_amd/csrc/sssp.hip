// Single-source shortest paths with non-negative integer weights (Table I:
// SSSP is a frontier traversal whose advance relaxes edges, W in O(b|E_i|)).
//
// Frontier relaxation on one GPU in one cooperative launch.  Each vertex
// keeps a packed 64-bit key (distance << 32 | predecessor); a relaxation is
// one 64-bit atomicMin, so at convergence the key holds the shortest
// distance and the smallest-id tight predecessor (every tight predecessor
// relaxes the vertex with its final distance at least once, and only tight
// ones can produce the final distance).
//
// Work ordering (near-far): only vertices whose distance is below a
// threshold T are relaxed ("near").  A vertex whose distance strictly
// improved to d < T joins the next frontier once (test-and-set membership
// bitmap); one improved to d >= T is appended once to the far pile
// (test-and-set membership bitmap of its own).  When the near frontier
// empties, T grows by delta and the pile is split: entries now below T form
// the next frontier, entries below the old T are stale (their vertex was
// relaxed as a near vertex since) and are dropped, the rest stay.  Every
// vertex is relaxed after its last improvement, so distances and parents are
// those of any other correct order; delta = UINT32_MAX never splits and
// gives plain frontier Bellman-Ford.  A smaller delta trades iterations for
// fewer re-relaxations (on a grid with weights in [1, 64] Bellman-Ford
// relaxes every edge about a hundred times).
//
// Load balance, small-frontier mode and the barrier follow the BFS push
// kernel.  Data layout in HBM (caller workspace, 256-B aligned):
//   key     uint64[n]                 packed distance / predecessor
//   inq     2 x uint32[ceil(n/32)]    membership of the next frontier
//   infar   uint32[ceil(n/32)]        membership of the far pile
//   queue   2 x int32[n]              input / output frontier
//   far     2 x int32[n]              far pile (entries are unique)
//   desc    int2[m/CH + n + 64]       edge-chunk descriptors
//   control barrier, counters, small-frontier hand-back state
#include <string.h>

#include "frontier.h"

namespace {
using namespace fgk;

constexpr int PB = 1024;
constexpr int PWAVES = PB / FG_WAVE;
constexpr int CH = 256;
constexpr int STAGE = 512;
constexpr int DSTAGE = 128;
constexpr int32_t DEF_SMALL_Q = 1024;
constexpr int64_t DEF_SMALL_E = 4096;
constexpr int32_t DEF_BIG_DEG = 64;
constexpr ull KEY_INF = ~0ull;
constexpr uint32_t DIST_INF = 0xFFFFFFFFu;
constexpr int FSTAGE = 256;
constexpr int64_t SMALL_FAR = 4 * PB;  // piles workgroup 0 splits alone
// Team mode (medium frontiers; see team_mode): LDS queue entries per member,
// widest team, packed team word fields, and the frontier shape it takes.
constexpr int QCAP = 2048;
constexpr int TEAM_MAX = 64;
constexpr int TW_CNT = 25, TW_FLAG = 50, TW_ARR = 57;
constexpr int64_t TW_CAP = (1 << 19) - 1;
constexpr int LDS_MEAN_DEG = 64;
constexpr int TPV = 4;
constexpr int32_t DEF_TEAM = 32;
constexpr int64_t DEF_TEAM_E = 65536;
constexpr int64_t TEAM_AUTO_DEG = 8;

struct CtrSlot {
  Line64 q;
  Line64 desc;
  Line64 insp;
};

// Zero when a launch starts (fresh workspaces are zero-filled; the last
// workgroup of each launch clears it again).
struct alignas(256) SsspCtl {
  uint32_t bar[FG_BAR_WORDS];
  uint32_t sm_signal;
  uint32_t pad0[63];
  uint32_t sm_ack;  // waiters that have read a hand-back (monotone)
  uint32_t pad0b[63];
  uint32_t exit_count;
  uint32_t pad1[63];
  uint32_t overflow;
  uint32_t pad2[63];
  Line64 reached;
  // Full-grid phases (near iterations and splits) are numbered ph = 0, 1, ..
  // and count into slot ph % 3, which phase ph - 1 cleared: a slot is read
  // after its phase's barrier and written again two barriers later, so no
  // workgroup reads a count that the next phase is already changing.
  Line64 farpos;    // positions in the far piles (monotone within a launch)
  Line64 fcnt[3];   // far-pile appends of the phase
  Line64 sqcnt[3];  // frontier entries made by a split
  CtrSlot slot[2];
  uint32_t fmin[3];  // smallest distance among the entries a split keeps
  uint32_t pad3[61];
  // team mode: arrivals of the team barrier, per-member records, the
  // level words, and the overflow counter of the global queue
  uint32_t team_arrive;
  uint32_t pad4[63];
  ull team_rec[2][TEAM_MAX][2];
  Line64 team_word[3];
  Line64 team_ovf;
  int32_t pub_k, pub_qsel, pub_force, pub_fsel;
  int64_t pub_qlen, pub_insp_sum, pub_flen;
  ull pub_fbase;
  uint32_t pub_T, pub_Tnext;
};

struct SsspParams {
  const int32_t* __restrict__ off;
  const int32_t* __restrict__ col;
  const uint32_t* __restrict__ w;
  int32_t n;
  int32_t nw32;  // ceil(n / 32)
  int32_t src;
  uint32_t* dist;
  int32_t* parent;
  ull* key;
  uint32_t* inq[2];
  uint32_t* infar;
  int32_t* q[2];
  int32_t* far[2];
  int2* desc;
  SsspCtl* ctl;
  uint32_t delta;
  fg_run_stats* stats;
  int32_t small_q;
  int64_t small_e;
  int32_t big_deg;
  int32_t clock_khz;
  int32_t team;     // workgroups of a team (<= 1: no team mode)
  int64_t team_e;   // largest frontier degree sum a team takes
};

struct St {
  int32_t k;
  int32_t qsel;
  int64_t qlen;
  int64_t insp_sum;
  ull b0q, b0desc, b0insp;
  ull b1q, b1desc, b1insp;
  uint32_t T;      // near threshold: distances below it are relaxed
  uint32_t Tnext;  // threshold of the next split
  int32_t fsel;    // pile holding the far entries
  int32_t ph;      // full-grid phases so far
  ull fbase;       // farpos value at which the current pile starts
  int64_t flen;    // entries in the current pile
};

// Far-pile appends staged per wave: positions come from one monotone
// counter, and the number appended is added to the phase's count slot.
template <int CAP>
struct PileStage {
  int32_t* buf;
  int32_t cnt;

  __device__ __forceinline__ void flush(ull* pos_ctr, ull* count, ull base, int32_t* out) {
    if (cnt == 0) return;
    wave_lds_fence();
    ull pos = 0;
    if (fg_lane() == 0) {
      pos = atomicAdd(pos_ctr, (ull)cnt);
      if (count) atomicAdd(count, (ull)cnt);
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
    if (cnt + c > CAP) flush(pos_ctr, count, base, out);
    if (keep) buf[cnt + fg_mbcnt(mask)] = x;
    cnt += c;
  }
};

__device__ __forceinline__ uint32_t sat_add(uint32_t a, uint32_t b) {
  const ull s = (ull)a + (ull)b;
  return s >= (ull)DIST_INF ? DIST_INF : (uint32_t)s;
}

struct Bases {
  ull q, desc, insp;
};

__device__ __forceinline__ ull sel(bool odd, ull a1, ull a0) {
  const ull m = 0ull - (ull)odd;
  return (a1 & m) | (a0 & ~m);
}
__device__ __forceinline__ Bases get_bases(const St& S) {
  const bool odd = S.k & 1;
  return Bases{sel(odd, S.b1q, S.b0q), sel(odd, S.b1desc, S.b0desc), sel(odd, S.b1insp, S.b0insp)};
}
__device__ __forceinline__ void set_bases(St& S, const Bases& b) {
  const bool odd = S.k & 1;
  S.b1q = sel(odd, b.q, S.b1q);
  S.b1desc = sel(odd, b.desc, S.b1desc);
  S.b1insp = sel(odd, b.insp, S.b1insp);
  S.b0q = sel(odd, S.b0q, b.q);
  S.b0desc = sel(odd, S.b0desc, b.desc);
  S.b0insp = sel(odd, S.b0insp, b.insp);
}

struct Lds {
  int32_t stage[PWAVES][STAGE];
  int2 dstage[PWAVES][DSTAGE];
  int32_t w_sc[PWAVES][FG_WAVE];
  int32_t w_u[PWAVES][FG_WAVE];
  int32_t w_b[PWAVES][FG_WAVE];
  uint32_t w_d[PWAVES][FG_WAVE];
  int32_t fstage[PWAVES][FSTAGE];
  uint32_t redm[PWAVES];
  int32_t b_sc[PB];
  int32_t b_u[PB];
  int32_t b_b[PB];
  uint32_t b_d[PB];
  int64_t red[PWAVES + 1];
  int32_t red32[PWAVES + 1];
  int32_t newcnt;
  int32_t flag;
  int32_t ackbad;  // workgroup 0: a hand-off acknowledgement wait failed
  int64_t bcast[8];
  uint32_t bcast2[2];
  // team mode: this member's share of the frontier, (vertex, first edge,
  // end edge), for the current and the next level; counters rotate over
  // three slots (input, output, cleared for the level after)
  int32_t lq_v[2][QCAP];
  int32_t lq_b[2][QCAP];
  int32_t lq_e[2][QCAP];
  int32_t lq_cnt[3];
  int32_t lq_deg[3];
  int32_t lq_big[3];
  int32_t tsum[6];
};

__device__ __forceinline__ void trace_iter(const St& S, const SsspParams& P) {
  if (blockIdx.x == 0 && threadIdx.x == 0 && P.stats && S.k < FG_TRACE_MAX) {
    P.stats->dir[S.k] = 0;
    P.stats->frontier[S.k] = S.qlen;
  }
}

__device__ __forceinline__ void trace_insp(int32_t k, int64_t insp, const SsspParams& P) {
  if (blockIdx.x == 0 && threadIdx.x == 0 && P.stats && k < FG_TRACE_MAX) {
    P.stats->inspected[k] = insp;
    P.stats->t_end[k] = (int64_t)wall_clock64();
  }
}

// Clears the count slot of the next full-grid phase.
__device__ __forceinline__ void clear_slot(SsspCtl* c, int s) {
  __hip_atomic_store(&c->fcnt[s].v, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&c->sqcnt[s].v, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&c->fmin[s], DIST_INF, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Block-wide minimum (every thread of the block calls it).
__device__ __forceinline__ uint32_t block_min(uint32_t x, uint32_t* scratch) {
#pragma unroll
  for (int d = FG_WAVE / 2; d > 0; d >>= 1) {
    const uint32_t o = __shfl_xor(x, d, FG_WAVE);
    x = o < x ? o : x;
  }
  const int wid = threadIdx.x / FG_WAVE;
  __syncthreads();
  if (fg_lane() == 0) scratch[wid] = x;
  __syncthreads();
  uint32_t m = DIST_INF;
#pragma unroll
  for (int i = 0; i < PWAVES; ++i) m = scratch[i] < m ? scratch[i] : m;
  return m;
}

enum { R_NONE = 0, R_NEAR = 1, R_FAR = 2 };

// Relax v through u with candidate distance du + wt.  Returns R_NEAR when
// v's distance strictly improved to below T and v was not yet in the next
// frontier, R_FAR when it improved to T or more and v was not yet in the far
// pile, R_NONE otherwise.
__device__ __forceinline__ int relax(int32_t v, int32_t u, uint32_t du, uint32_t wt, uint32_t T,
                                     uint32_t* inq_next, const SsspParams& P) {
  const ull nd = (ull)du + (ull)wt;
  if (nd >= 0xFFFFFFFFull) {
    P.ctl->overflow = 1u;  // distance does not fit the uint32 output
    return R_NONE;
  }
  const ull nk = (nd << 32) | (ull)(uint32_t)u;
  // the source keeps (0, src): with zero-weight edges a neighbour at
  // distance 0 would otherwise replace its predecessor
  if (v == P.src || nk >= P.key[v]) return R_NONE;  // plain pre-check; keys only decrease
  const ull old = atomicMin(&P.key[v], nk);
  if (nd >= (old >> 32)) return R_NONE;  // no distance improvement (maybe a better parent)
  const uint32_t bit = 1u << (v & 31);
  if (nd < (ull)T) {
    const uint32_t o = atomicOr(&inq_next[v >> 5], bit);
    return (o & bit) ? R_NONE : R_NEAR;
  }
  const uint32_t o = atomicOr(&P.infar[v >> 5], bit);
  return (o & bit) ? R_NONE : R_FAR;
}

// Full grid, phase A: 64-entry frontier chunks per wave; low-degree vertices
// by scan-gather, high-degree ones into CH-edge descriptors.  Each frontier
// vertex also clears its word of the current membership bitmap (every bit
// set there belongs to a current frontier vertex, and nothing sets bits in
// it during this iteration).
__device__ void phase_a(const SsspParams& P, const St& S, Lds& L) {
  const int lane = fg_lane();
  const int wid = threadIdx.x / FG_WAVE;
  const int32_t* Qin = P.q[S.qsel];
  int32_t* Qout = P.q[S.qsel ^ 1];
  uint32_t* inq_cur = P.inq[S.k & 1];
  uint32_t* inq_nxt = P.inq[(S.k + 1) & 1];
  int32_t* sc = L.w_sc[wid];
  int32_t* su = L.w_u[wid];
  int32_t* sb = L.w_b[wid];
  uint32_t* sd = L.w_d[wid];
  CtrSlot& C = P.ctl->slot[S.k & 1];
  const Bases B = get_bases(S);
  WaveStage<int32_t, STAGE> st{L.stage[wid], 0};
  PileStage<FSTAGE> fst{L.fstage[wid], 0};
  WaveStage<int2, DSTAGE> dst{L.dstage[wid], 0};
  int32_t* pile = P.far[S.fsel];
  ull* fpos = &P.ctl->farpos.v;
  ull* fcnt = &P.ctl->fcnt[S.ph % 3].v;
  const int64_t gw = (int64_t)blockIdx.x * PWAVES + wid;
  const int64_t W = (int64_t)gridDim.x * PWAVES;
  int64_t insp = 0;
  for (int64_t base = gw * FG_WAVE; base < S.qlen; base += W * FG_WAVE) {
    const int64_t i = base + lane;
    int32_t u = 0, b = 0, deg = 0;
    uint32_t du = 0;
    if (i < S.qlen) {
      u = Qin[i];
      b = P.off[u];
      deg = P.off[u + 1] - b;
      du = (uint32_t)(P.key[u] >> 32);
      fg_st_shared(&inq_cur[u >> 5], 0u);
    }
    insp += deg;
    const bool big = deg >= P.big_deg;
    const int32_t nd = big ? (deg + CH - 1) / CH : 0;
    const int32_t ndi = fg_wave_incl_scan(nd);
    const int32_t ND = __shfl(ndi, FG_WAVE - 1, FG_WAVE);
    if (ND > 0) {
      wave_lds_fence();
      sc[lane] = ndi - nd;
      su[lane] = u;
      sb[lane] = b;
      wave_lds_fence();
      for (int32_t t0 = 0; t0 < ND; t0 += FG_WAVE) {
        const int32_t t = t0 + lane;
        int2 dsc = make_int2(0, 0);
        if (t < ND) {
          const int32_t j = upper_idx(sc, FG_WAVE, t);
          dsc = make_int2(su[j], sb[j] + (t - sc[j]) * CH);
        }
        dst.push(t < ND, dsc, &C.desc.v, B.desc, P.desc);
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
    sd[lane] = du;
    wave_lds_fence();
    for (int32_t t0 = 0; t0 < T; t0 += FG_WAVE) {
      const int32_t t = t0 + lane;
      int r = R_NONE;
      int32_t v = 0;
      if (t < T) {
        const int32_t j = upper_idx(sc, FG_WAVE, t);
        const int32_t e = sb[j] + (t - sc[j]);
        v = P.col[e];
        r = relax(v, su[j], sd[j], P.w[e], S.T, inq_nxt, P);
      }
      st.push(r == R_NEAR, v, &C.q.v, B.q, Qout);
      fst.push(r == R_FAR, v, fpos, fcnt, S.fbase, pile);
    }
  }
  st.flush(&C.q.v, B.q, Qout);
  fst.flush(fpos, fcnt, S.fbase, pile);
  dst.flush(&C.desc.v, B.desc, P.desc);
  const int64_t tot = fg_block_sum<PB>(insp, L.red);
  if (threadIdx.x == 0 && tot) atomicAdd(&C.insp.v, (ull)tot);
}

// Full grid, phase B: descriptors taken by every wave in turn.
__device__ void phase_b(const SsspParams& P, const St& S, int64_t ndesc, Lds& L) {
  const int lane = fg_lane();
  const int wid = threadIdx.x / FG_WAVE;
  const int64_t gw = (int64_t)blockIdx.x * PWAVES + wid;
  const int64_t W = (int64_t)gridDim.x * PWAVES;
  int32_t* Qout = P.q[S.qsel ^ 1];
  uint32_t* inq_nxt = P.inq[(S.k + 1) & 1];
  CtrSlot& C = P.ctl->slot[S.k & 1];
  const Bases B = get_bases(S);
  WaveStage<int32_t, STAGE> st{L.stage[wid], 0};
  PileStage<FSTAGE> fst{L.fstage[wid], 0};
  int32_t* pile = P.far[S.fsel];
  ull* fpos = &P.ctl->farpos.v;
  ull* fcnt = &P.ctl->fcnt[S.ph % 3].v;
  for (int64_t i = gw; i < ndesc; i += W) {
    const int2 dsc = P.desc[i];
    const int32_t u = dsc.x;
    const int32_t e_end = P.off[u + 1];
    const int32_t e1 = dsc.y + CH < e_end ? dsc.y + CH : e_end;
    const uint32_t du = (uint32_t)(P.key[u] >> 32);
    int32_t vv[CH / FG_WAVE];
    uint32_t ww[CH / FG_WAVE];
#pragma unroll
    for (int r = 0; r < CH / FG_WAVE; ++r) {
      const int32_t e = dsc.y + r * FG_WAVE + lane;
      vv[r] = e < e1 ? P.col[e] : -1;
      ww[r] = e < e1 ? P.w[e] : 0u;
    }
#pragma unroll
    for (int r = 0; r < CH / FG_WAVE; ++r) {
      const int32_t v = vv[r];
      const int rr = v >= 0 ? relax(v, u, du, ww[r], S.T, inq_nxt, P) : R_NONE;
      st.push(rr == R_NEAR, v, &C.q.v, B.q, Qout);
      fst.push(rr == R_FAR, v, fpos, fcnt, S.fbase, pile);
    }
  }
  st.flush(&C.q.v, B.q, Qout);
  fst.flush(fpos, fcnt, S.fbase, pile);
}

// Split of the far pile by the whole grid (the current frontier is empty):
// entries with T <= dist < Tnew go to the current queue, stale ones (dist <
// T) are dropped, the rest move to the other pile.  Their smallest distance
// goes to fmin[ph % 3].
__device__ void split_full(const SsspParams& P, const St& S, uint32_t Tnew, Lds& L) {
  const int lane = fg_lane();
  const int wid = threadIdx.x / FG_WAVE;
  const int32_t* pile = P.far[S.fsel];
  int32_t* keep = P.far[S.fsel ^ 1];
  int32_t* Q = P.q[S.qsel];
  const ull kbase = S.fbase + (ull)S.flen;
  WaveStage<int32_t, STAGE> st{L.stage[wid], 0};
  PileStage<FSTAGE> fst{L.fstage[wid], 0};
  const int64_t gw = (int64_t)blockIdx.x * PWAVES + wid;
  const int64_t W = (int64_t)gridDim.x * PWAVES;
  ull* sq = &P.ctl->sqcnt[S.ph % 3].v;
  ull* fpos = &P.ctl->farpos.v;
  ull* fcnt = &P.ctl->fcnt[S.ph % 3].v;
  uint32_t mn = DIST_INF;
  for (int64_t base = gw * FG_WAVE; base < S.flen; base += W * FG_WAVE) {
    const int64_t i = base + lane;
    int r = R_NONE;
    int32_t v = 0;
    if (i < S.flen) {
      v = pile[i];
      const uint32_t d = (uint32_t)(P.key[v] >> 32);
      if (d >= Tnew) {
        r = R_FAR;
        mn = d < mn ? d : mn;
      } else {
        atomicAnd(&P.infar[v >> 5], ~(1u << (v & 31)));
        r = d >= S.T ? R_NEAR : R_NONE;
      }
    }
    st.push(r == R_NEAR, v, sq, 0ull, Q);
    fst.push(r == R_FAR, v, fpos, fcnt, kbase, keep);
  }
  st.flush(sq, 0ull, Q);
  fst.flush(fpos, fcnt, kbase, keep);
  const uint32_t bm = block_min(mn, L.redm);
  if (threadIdx.x == 0 && bm != DIST_INF) atomicMin(&P.ctl->fmin[S.ph % 3], bm);
}

// The same split by workgroup 0 alone (small piles, inside small mode).
__device__ void split_small(const SsspParams& P, St& S, Lds& L) {
  const int tid = threadIdx.x;
  const int lane = fg_lane();
  const uint32_t Tnew = S.Tnext;
  const int32_t* pile = P.far[S.fsel];
  int32_t* keep = P.far[S.fsel ^ 1];
  int32_t* Q = P.q[S.qsel];
  const ull kbase = S.fbase + (ull)S.flen;
  if (tid == 0) L.newcnt = 0;
  __syncthreads();
  uint32_t mn = DIST_INF;
  for (int64_t c0 = 0; c0 < S.flen; c0 += PB) {
    const int64_t i = c0 + tid;
    int r = R_NONE;
    int32_t v = 0;
    if (i < S.flen) {
      v = pile[i];
      const uint32_t d = (uint32_t)(P.key[v] >> 32);
      if (d >= Tnew) {
        r = R_FAR;
        mn = d < mn ? d : mn;
      } else {
        atomicAnd(&P.infar[v >> 5], ~(1u << (v & 31)));
        r = d >= S.T ? R_NEAR : R_NONE;
      }
    }
    const uint64_t nm = __ballot(r == R_NEAR);
    if (nm) {
      int32_t pos = 0;
      if (lane == 0) pos = atomicAdd(&L.newcnt, __popcll(nm));
      pos = __shfl(pos, 0, FG_WAVE);
      if (r == R_NEAR) Q[pos + fg_mbcnt(nm)] = v;
    }
    const uint64_t fm = __ballot(r == R_FAR);
    if (fm) {
      ull pos = 0;
      if (lane == 0) pos = atomicAdd(&P.ctl->farpos.v, (ull)__popcll(fm));
      pos = __shfl(pos, 0, FG_WAVE) - kbase;
      if (r == R_FAR) keep[pos + fg_mbcnt(fm)] = v;
    }
  }
  // block_min has barriers: newcnt and farpos are final (workgroup 0 is the
  // only one running)
  const uint32_t bm = block_min(mn, L.redm);
  S.qlen = L.newcnt;
  S.fbase = kbase;
  S.flen = (int64_t)(fg_atomic_load_u64(&P.ctl->farpos.v) - kbase);
  S.fsel ^= 1;
  S.T = Tnew;
  S.Tnext = S.qlen > 0 ? sat_add(Tnew, P.delta) : sat_add(bm, P.delta);
  __syncthreads();
}

// Workgroup 0 alone while the frontier is small (see the BFS kernel).
__device__ void small_mode(const SsspParams& P, St& S, Lds& L, int* force_full) {
  const int tid = threadIdx.x;
  *force_full = 0;
  for (;;) {
    if (S.qlen == 0) {
      // near frontier empty: split the pile here if it is small
      if (S.flen == 0 || S.flen > SMALL_FAR) return;
      split_small(P, S, L);
      trace_iter(S, P);
      if (S.qlen > P.small_q) return;
      continue;
    }
    const int32_t* Qin = P.q[S.qsel];
    int32_t* Qout = P.q[S.qsel ^ 1];
    uint32_t* inq_cur = P.inq[S.k & 1];
    uint32_t* inq_nxt = P.inq[(S.k + 1) & 1];
    int64_t s = 0;
    for (int64_t i = tid; i < S.qlen; i += PB) {
      const int32_t u = Qin[i];
      s += P.off[u + 1] - P.off[u];
    }
    const int64_t sum = fg_block_sum<PB>(s, L.red);
    if (sum > P.small_e) {
      *force_full = 1;
      return;
    }
    if (tid == 0) L.newcnt = 0;
    for (int64_t c0 = 0; c0 < S.qlen; c0 += PB) {
      const int64_t i = c0 + tid;
      int32_t u = 0, b = 0, d = 0;
      uint32_t du = 0;
      if (i < S.qlen) {
        u = Qin[i];
        b = P.off[u];
        d = P.off[u + 1] - b;
        du = (uint32_t)(P.key[u] >> 32);
        inq_cur[u >> 5] = 0u;
      }
      int32_t T = 0;
      const int32_t ex = fg_block_excl_scan<PB>(d, L.red32, &T);
      L.b_sc[tid] = ex;
      L.b_u[tid] = u;
      L.b_b[tid] = b;
      L.b_d[tid] = du;
      __syncthreads();
      const int32_t cnt = (int32_t)((S.qlen - c0) < PB ? (S.qlen - c0) : PB);
      for (int32_t t0 = 0; t0 < T; t0 += PB) {
        const int32_t t = t0 + tid;
        int r = R_NONE;
        int32_t v = 0;
        if (t < T) {
          const int32_t j = upper_idx(L.b_sc, cnt, t);
          const int32_t e = L.b_b[j] + (t - L.b_sc[j]);
          v = P.col[e];
          r = relax(v, L.b_u[j], L.b_d[j], P.w[e], S.T, inq_nxt, P);
        }
        const uint64_t mask = __ballot(r == R_NEAR);
        if (mask) {
          int32_t pos = 0;
          if (fg_lane() == 0) pos = atomicAdd(&L.newcnt, __popcll(mask));
          pos = __shfl(pos, 0, FG_WAVE);
          if (r == R_NEAR) Qout[pos + fg_mbcnt(mask)] = v;
        }
        const uint64_t fm = __ballot(r == R_FAR);
        if (fm) {
          ull pos = 0;
          if (fg_lane() == 0) pos = atomicAdd(&P.ctl->farpos.v, (ull)__popcll(fm));
          pos = __shfl(pos, 0, FG_WAVE) - S.fbase;
          if (r == R_FAR) P.far[S.fsel][pos + fg_mbcnt(fm)] = v;
        }
      }
      __syncthreads();
    }
    const int64_t nq = L.newcnt;
    S.flen = (int64_t)(fg_atomic_load_u64(&P.ctl->farpos.v) - S.fbase);
    trace_insp(S.k, sum, P);
    S.insp_sum += sum;
    S.k++;
    S.qsel ^= 1;
    S.qlen = nq;
    trace_iter(S, P);
    __syncthreads();
    if (nq > P.small_q) return;
  }
}


// ---------------------------------------------------------------- team mode
//
// A team of T workgroups runs near iterations back to back while the
// frontier is of medium size (more than one workgroup's worth, at most
// QCAP * T / 2 vertices, mean degree <= LDS_MEAN_DEG, degree sum <= team_e).
// Each member keeps its share of the frontier in LDS as (vertex, first edge,
// end edge); a vertex it moves into the next frontier goes to its own next
// LDS queue with the offsets loaded alongside the relaxation.  Far-pile
// appends go to the global pile as elsewhere.  Per iteration the members
// add one packed word (arrival | overflow flag | count | capped degree sum)
// to the level's team word and poll it.  Members share the keys and the
// membership bitmaps, touched only by atomics here: a vertex's own distance
// is read with an agent-scope atomic load (another member may just have
// lowered it) and membership words are cleared with agent-scope atomic
// stores.  Exact per-member counts (tagged records) are read when the
// episode ends or a member's share is uneven; the shares are then evened
// out through the global queue.  The other workgroups sleep meanwhile.
struct TeamSync {
  uint32_t* arrive;
  uint32_t* abort_flag;
  uint32_t T;
  uint32_t count;

  // Without the L2 write-back: for data the members write with
  // fg_st_shared or atomics.
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

struct TeamBases {
  ull ovf;          // team_ovf value at which the current global queue starts
  uint32_t levels;  // team word exchanges so far
};

// Workgroup 0 clears the team word of exchange `level + 1` (its last
// readers have all arrived at this exchange).
__device__ __forceinline__ ull team_clear_next(const SsspParams& P, uint32_t level) {
  if (blockIdx.x == 0 && threadIdx.x == 0)
    return __hip_atomic_exchange(&P.ctl->team_word[(level + 1) % 3].v, 0ull, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
  return 0;
}

// One exchange: add this member's word, wait for all T.  L.tsum: [0] count,
// [1] degree sum, [2] members that flagged themselves (count > lim).
__device__ bool team_fast(const SsspParams& P, Lds& L, uint32_t T, uint32_t level, int32_t bcnt,
                          int32_t bdeg, int32_t lim, ull cleared) {
  if (threadIdx.x == 0) {
    ull* w = &P.ctl->team_word[level % 3].v;
    const ull g = bdeg < TW_CAP ? (ull)bdeg : (ull)TW_CAP;
    const ull add = (1ull << TW_ARR) | ((ull)(bcnt > lim) << TW_FLAG) | ((ull)bcnt << TW_CNT) | g;
    // the clear's old value is consumed before the arrival is issued
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

// Exact per-member counts (records tagged with the level; re-read until
// current).  L.tsum: [2] members over QCAP, [3] overflow entries in all,
// [4] entries kept in LDS by the members before this one, [5] largest count.
__device__ bool team_records(const SsspParams& P, Lds& L, uint32_t T, uint32_t seq, int odd) {
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

// `w` consecutive slots per lane behind the LDS counter, one atomic per
// wave; returns this lane's first slot.  Every lane of the wave takes part.
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

// Stores a won vertex at slot `pos` of the next LDS queue; slots past QCAP
// go to the global queue, one atomic per wave.  Every lane takes part.
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
    if (over) fg_st_shared(&Qo[base - ovf_base + fg_mbcnt(om)], v);
  }
}

// Far-pile append of a wave's far vertices (one atomic per wave).
__device__ __forceinline__ void far_put(const SsspParams& P, bool put, int32_t v, int32_t* pile,
                                        ull fbase) {
  const uint64_t m = __ballot(put);
  if (m) {
    ull base = 0;
    if (fg_lane() == 0) base = atomicAdd(&P.ctl->farpos.v, (ull)__popcll(m));
    base = fg_uni(base);
    if (put) fg_st_shared(&pile[base - fbase + fg_mbcnt(m)], v);
  }
}

// The relaxation of team mode: no pre-check load (latency matters more than
// atomic traffic at these frontier sizes).
__device__ __forceinline__ int relax_team(int32_t v, int32_t u, uint32_t du, uint32_t wt, uint32_t T,
                                          uint32_t* inq_next, const SsspParams& P) {
  const ull nd = (ull)du + (ull)wt;
  if (nd >= 0xFFFFFFFFull) {
    __hip_atomic_store(&P.ctl->overflow, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return R_NONE;
  }
  if (v == P.src) return R_NONE;
  const ull nk = (nd << 32) | (ull)(uint32_t)u;
  const ull old = atomicMin(&P.key[v], nk);
  if (nd >= (old >> 32)) return R_NONE;
  const uint32_t bit = 1u << (v & 31);
  if (nd < (ull)T) {
    const uint32_t o = atomicOr(&inq_next[v >> 5], bit);
    return (o & bit) ? R_NONE : R_NEAR;
  }
  const uint32_t o = atomicOr(&P.infar[v >> 5], bit);
  return (o & bit) ? R_NONE : R_FAR;
}

// Runs near iterations as a team of T members (blockIdx.x < T).  Returns
// false on a device error.  *handback = 1 when the frontier met on entry
// does not suit the mode (the caller runs the next iteration on the full
// grid).  On return S describes the frontier in the global queue Q[qsel].
__device__ bool team_mode(const SsspParams& P, St& S, Lds& L, uint32_t T, TeamSync& ts,
                          TeamBases& tb, int* handback) {
  const int tid = threadIdx.x;
  const int lane = fg_lane();
  ull* ovf = &P.ctl->team_ovf.v;
  ull ovf_base = tb.ovf;
  int cur = 0, ci = 0, ni = 1, ri = 2;
  bool load = true;
  int64_t lvl_deg = 0;  // degree sum of the current level's frontier
  *handback = 0;
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
      lvl_deg = fg_uni(L.tsum[1]);
      if (lvl_deg > LDS_MEAN_DEG * S.qlen || lvl_deg > P.team_e) {
        *handback = 1;  // the global queue is untouched
        return true;
      }
      __syncthreads();
    }
    const int nxt = cur ^ 1;
    const int32_t cnt = L.lq_cnt[ci];
    // issued now, so that it is done by the time this level's exchange
    // needs it
    const ull cleared = team_clear_next(P, tb.levels);
    if (tid == 0) {
      L.lq_cnt[ri] = 0;
      L.lq_deg[ri] = 0;
      L.lq_big[ri] = 0;
    }
    uint32_t* inq_cur = P.inq[S.k & 1];
    uint32_t* inq_nxt = P.inq[(S.k + 1) & 1];
    int32_t* pile = P.far[S.fsel];
    bool big = false;
    // vertices of degree <= TPV: TPV consecutive lanes per vertex, one edge
    // each; every vertex clears its word of the current membership bitmap
    for (int32_t c0 = 0; c0 < cnt; c0 += PB / TPV) {
      const int32_t i = c0 + tid / TPV;
      const int32_t j = tid % TPV;
      int32_t u = 0, b = 0, d = 0;
      if (i < cnt) {
        u = L.lq_v[cur][i];
        b = L.lq_b[cur][i];
        d = L.lq_e[cur][i] - b;
        if (j == 0)
          __hip_atomic_store(&inq_cur[u >> 5], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      big |= d > TPV;
      int r = R_NONE;
      int32_t v = 0, vb = 0, ve = 0;
      if (d <= TPV && j < d) {
        const int32_t e = b + j;
        v = P.col[e];
        const uint32_t wt = P.w[e];
        vb = P.off[v];
        ve = P.off[v + 1];
        const uint32_t du = (uint32_t)(__hip_atomic_load(&P.key[u], __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT) >> 32);
        r = relax_team(v, u, du, wt, S.T, inq_nxt, P);
      }
      const bool won = r == R_NEAR;
      const int32_t pos = wave_reserve(won ? 1 : 0, &L.lq_cnt[ni]);
      const int32_t wdeg = fg_wave_sum(won ? ve - vb : 0);
      if (lane == 0 && wdeg) atomicAdd(&L.lq_deg[ni], wdeg);
      wave_put(L, nxt, won, pos, v, vb, ve, Qo, ovf, ovf_base);
      far_put(P, r == R_FAR, v, pile, S.fbase);
    }
    if (big) L.lq_big[ni] = 1;
    __syncthreads();
    if (L.lq_big[ni]) {
      // vertices of degree > TPV: block scan-gather over their edges
      for (int32_t c0 = 0; c0 < cnt; c0 += PB) {
        const int32_t i = c0 + tid;
        int32_t u = 0, b = 0, d = 0;
        uint32_t du = 0;
        if (i < cnt) {
          u = L.lq_v[cur][i];
          b = L.lq_b[cur][i];
          d = L.lq_e[cur][i] - b;
        }
        if (d <= TPV) d = 0;
        if (d)
          du = (uint32_t)(__hip_atomic_load(&P.key[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >>
                          32);
        int32_t Tn = 0;
        const int32_t ex = fg_block_excl_scan<PB>(d, L.red32, &Tn);
        L.b_sc[tid] = ex;
        L.b_u[tid] = u;
        L.b_b[tid] = b;
        L.b_d[tid] = du;
        __syncthreads();
        const int32_t nc = cnt - c0 < PB ? cnt - c0 : PB;
        for (int32_t t0 = 0; t0 < Tn; t0 += PB) {
          const int32_t t = t0 + tid;
          int r = R_NONE;
          int32_t v = 0, vb = 0, ve = 0;
          if (t < Tn) {
            const int32_t jj = upper_idx(L.b_sc, nc, t);
            const int32_t e = L.b_b[jj] + (t - L.b_sc[jj]);
            v = P.col[e];
            const uint32_t wt = P.w[e];
            vb = P.off[v];
            ve = P.off[v + 1];
            r = relax_team(v, L.b_u[jj], L.b_d[jj], wt, S.T, inq_nxt, P);
          }
          const bool won = r == R_NEAR;
          const int32_t pos = wave_reserve(won ? 1 : 0, &L.lq_cnt[ni]);
          const int32_t wdeg = fg_wave_sum(won ? ve - vb : 0);
          if (lane == 0 && wdeg) atomicAdd(&L.lq_deg[ni], wdeg);
          wave_put(L, nxt, won, pos, v, vb, ve, Qo, ovf, ovf_base);
          far_put(P, r == R_FAR, v, pile, S.fbase);
        }
        __syncthreads();
      }
    }
    const int32_t bcnt = L.lq_cnt[ni];
    const int32_t bdeg = L.lq_deg[ni];
    if (tid == 0) {
      // the record behind the word, read only on the slow path
      ull* rr = P.ctl->team_rec[S.k & 1][blockIdx.x];
      const ull tag = (ull)((uint32_t)S.k + 1u) << 32;
      __hip_atomic_store(rr, tag | (uint32_t)bcnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const int64_t lim = (5 * S.qlen / T + 64) / 4;
    if (!team_fast(P, L, T, tb.levels, bcnt, bdeg, (int32_t)(lim < QCAP ? lim : QCAP), cleared))
      return false;
    tb.levels++;
    const int64_t nq = fg_uni(L.tsum[0]);
    const int64_t nqdeg = fg_uni(L.tsum[1]);
    const int64_t nflag = fg_uni(L.tsum[2]);
    trace_insp(S.k, lvl_deg, P);
    S.insp_sum += lvl_deg;
    S.k++;
    S.qlen = nq;
    lvl_deg = nqdeg;
    trace_iter(S, P);
    bool stay = nq > 0 && nqdeg <= LDS_MEAN_DEG * nq && nqdeg <= P.team_e &&
                nq <= (int64_t)QCAP * T / 2 && !(nq <= P.small_q && nqdeg <= P.small_e);
    int64_t nover = bcnt > QCAP ? bcnt - QCAP : 0, before = 0;
    bool rebalance = false;
    if (!stay || nflag) {
      if (!team_records(P, L, T, (uint32_t)S.k, (S.k - 1) & 1)) return false;
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
      for (int32_t i = tid; i < nloc; i += PB) fg_st_shared(&dst[i], L.lq_v[nxt][i]);
      ovf_base += (ull)nover;
      tb.ovf = ovf_base;
      if (!ts.sync_acquire(&L.flag)) return false;
      S.qsel ^= 1;
      if (!stay) {
        // the far pile grew by the members' appends (all done before the
        // barrier above)
        S.flen = (int64_t)(fg_atomic_load_u64(&P.ctl->farpos.v) - S.fbase);
        return true;
      }
      load = true;
    }
    cur = nxt;
    const int t3 = ci;
    ci = ni;
    ni = ri;
    ri = t3;
  }
}

// TEAM = false compiles the kernel without the team episodes: their code
// raises the register pressure (and the spills) of the whole kernel, which
// is not worth it on graphs whose frontiers rarely suit a team.
template <bool TEAM>
__global__ __launch_bounds__(PB) void sssp_persistent(SsspParams P) {
  __shared__ Lds L;
  fg_grid_sync gs{P.ctl->bar, gridDim.x, 0u};
  St S = {};
  S.qlen = 1;
  S.T = P.delta;
  S.Tnext = sat_add(P.delta, P.delta);
  uint32_t sm_seen = 0;
  uint32_t ack_need = 0;  // workgroup 0: acknowledgements of the hand-backs so far
  int force_full = 0;
  bool ok = true;
  TeamSync ts{&P.ctl->team_arrive, P.ctl->bar + FG_BAR_STRIDE, (uint32_t)(P.team > 1 ? P.team : 1),
              0u};
  TeamBases tb = {};
  const int64_t tid = (int64_t)blockIdx.x * PB + threadIdx.x;
  const int64_t nth = (int64_t)gridDim.x * PB;
  // init: every key infinite except the source, membership bitmaps clear
  if (blockIdx.x == 0 && P.stats) {
    uint32_t* sw = (uint32_t*)P.stats;
    for (int i = threadIdx.x; i < (int)(sizeof(fg_run_stats) / 4); i += PB) sw[i] = 0u;
  }
  for (int64_t v = tid; v < P.n; v += nth)
    P.key[v] = v == P.src ? (ull)(uint32_t)P.src : KEY_INF;
  for (int64_t i = tid; i < P.nw32; i += nth) {
    P.inq[0][i] = 0u;
    P.inq[1][i] = 0u;
    P.infar[i] = 0u;
  }
  if (tid == 0) {
    P.q[0][0] = P.src;
    P.ctl->fmin[0] = DIST_INF;
  }
  if (!gs.sync(&L.flag)) ok = false;
  if (blockIdx.x == 0 && threadIdx.x == 0 && P.stats) {
    P.stats->t_start = (int64_t)wall_clock64();
    P.stats->clock_khz = P.clock_khz;
  }
  trace_iter(S, P);
  while (ok && (S.qlen > 0 || S.flen > 0)) {
    const bool small = S.qlen == 0 ? S.flen <= SMALL_FAR : (!force_full && S.qlen <= P.small_q);
    const bool team = TEAM && !small && S.qlen > 0 && !force_full && P.team > 1 &&
                      S.qlen <= (int64_t)QCAP * P.team / 2;
    if (small || team) {
      sm_seen++;
      const bool member = small ? blockIdx.x == 0 : blockIdx.x < (uint32_t)P.team;
      if (member) {
        int ff = 0;
        if (small) {
          small_mode(P, S, L, &ff);
        } else if (!team_mode(P, S, L, (uint32_t)P.team, ts, tb, &ff)) {
          ok = false;
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) {
          SsspCtl* c = P.ctl;
          // every waiter of the previous hand-back has read it (on a
          // timeout the abort flag is set and every wait ends)
          L.ackbad = !fg_wait_geq(&c->sm_ack, ack_need, c->bar + FG_BAR_STRIDE, 1);
          // a failed wait has set the abort flag: publish nothing (a slow
          // waiter may still be reading the previous hand-off); the waiters
          // see the flag and leave
          if (!L.ackbad) {
            c->pub_k = S.k;
            c->pub_qsel = S.qsel;
            c->pub_force = ff;
            c->pub_qlen = S.qlen;
            c->pub_insp_sum = S.insp_sum;
            c->pub_fsel = S.fsel;
            c->pub_flen = S.flen;
            c->pub_fbase = S.fbase;
            c->pub_T = S.T;
            c->pub_Tnext = S.Tnext;
            __hip_atomic_fetch_add(&c->sm_signal, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            ack_need += gridDim.x - (small ? 1u : (uint32_t)P.team);
          }
        }
        force_full = ff;
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
            const SsspCtl* c = P.ctl;
            L.bcast[0] = c->pub_k;
            L.bcast[1] = c->pub_qsel;
            L.bcast[2] = c->pub_force;
            L.bcast[3] = c->pub_qlen;
            L.bcast[4] = c->pub_insp_sum;
            L.bcast[5] = c->pub_fsel;
            L.bcast[6] = c->pub_flen;
            L.bcast[7] = (int64_t)c->pub_fbase;
            L.bcast2[0] = c->pub_T;
            L.bcast2[1] = c->pub_Tnext;
            fg_handoff_ack(&P.ctl->sm_ack);
          }
        }
        __syncthreads();
        if (L.flag) {
          ok = false;
          break;
        }
        S.k = (int32_t)L.bcast[0];
        S.qsel = (int32_t)L.bcast[1];
        force_full = (int)L.bcast[2];
        S.qlen = L.bcast[3];
        S.insp_sum = L.bcast[4];
        S.fsel = (int32_t)L.bcast[5];
        S.flen = L.bcast[6];
        S.fbase = (ull)L.bcast[7];
        S.T = L.bcast2[0];
        S.Tnext = L.bcast2[1];
        __syncthreads();
      }
      continue;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) clear_slot(P.ctl, (S.ph + 1) % 3);
    if (S.qlen == 0) {
      // full-grid split of a large pile
      const uint32_t Tnew = S.Tnext;
      split_full(P, S, Tnew, L);
      if (!(ok = gs.sync_acquire(&L.flag))) break;
      const int sl = S.ph % 3;
      const ull sq = fg_atomic_load_u64(&P.ctl->sqcnt[sl].v);
      const ull fc = fg_atomic_load_u64(&P.ctl->fcnt[sl].v);
      const uint32_t mn = __hip_atomic_load(&P.ctl->fmin[sl], __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
      S.qlen = (int64_t)sq;
      S.fbase += (ull)S.flen;
      S.flen = (int64_t)fc;
      S.fsel ^= 1;
      S.ph++;
      S.T = Tnew;
      S.Tnext = S.qlen > 0 ? sat_add(Tnew, P.delta) : sat_add(mn, P.delta);
      trace_iter(S, P);
      continue;
    }
    force_full = 0;
    CtrSlot& C = P.ctl->slot[S.k & 1];
    Bases B = get_bases(S);
    phase_a(P, S, L);
    if (!(ok = gs.sync_acquire(&L.flag))) break;
    const ull dt = fg_atomic_load_u64(&C.desc.v);
    const int64_t ndesc = (int64_t)(dt - B.desc);
    if (ndesc > 0) {
      phase_b(P, S, ndesc, L);
      if (!(ok = gs.sync_acquire(&L.flag))) break;
    }
    B.desc = dt;
    const ull qt = fg_atomic_load_u64(&C.q.v);
    const ull it = fg_atomic_load_u64(&C.insp.v);
    const ull fc = fg_atomic_load_u64(&P.ctl->fcnt[S.ph % 3].v);
    const int64_t nq = (int64_t)(qt - B.q);
    const int64_t insp = (int64_t)(it - B.insp);
    B.q = qt;
    B.insp = it;
    set_bases(S, B);
    trace_insp(S.k, insp, P);
    S.insp_sum += insp;
    S.k++;
    S.qsel ^= 1;
    S.qlen = nq;
    S.flen += (int64_t)fc;
    S.ph++;
    trace_iter(S, P);
  }
  // unpack keys into the outputs, count reached vertices
  int32_t reached = 0;
  if (ok) {
    for (int64_t v = tid; v < P.n; v += nth) {
      const ull kk = P.key[v];
      const bool r = kk != KEY_INF;
      P.dist[v] = r ? (uint32_t)(kk >> 32) : 0xFFFFFFFFu;
      if (P.parent) P.parent[v] = r ? (int32_t)(uint32_t)kk : -1;
      reached += r;
    }
  }
  const int32_t rb = fg_block_sum<PB>(reached, L.red32);
  if (threadIdx.x == 0 && rb) atomicAdd(&P.ctl->reached.v, (ull)rb);
  const bool ok2 = gs.sync(&L.flag);
  if (blockIdx.x == 0 && threadIdx.x == 0 && P.stats) {
    fg_run_stats* stt = P.stats;
    const uint32_t ovf = __hip_atomic_load(&P.ctl->overflow, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    stt->status = (ok && ok2) ? (ovf ? FG_EOVERFLOW : FG_OK) : FG_EDEVICE;
    stt->iterations = S.k;
    stt->reached = (int64_t)fg_atomic_load_u64(&P.ctl->reached.v);
    stt->edges_inspected = S.insp_sum;
    stt->grid_blocks = (int32_t)gridDim.x;
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
    for (int i = threadIdx.x; i < (int)(sizeof(SsspCtl) / 4); i += PB) w[i] = 0u;
  }
}

struct SsspLayout {
  SsspCtl* ctl;
  ull* key;
  uint32_t* inq[2];
  uint32_t* infar;
  int32_t* q[2];
  int32_t* far[2];
  int2* desc;
  size_t bytes;
};

SsspLayout sssp_layout(const fg_graph* g, void* ws) {
  fg_carver c(ws);
  SsspLayout L;
  L.ctl = c.take<SsspCtl>(1);
  L.key = c.take<ull>(g->n);
  const size_t nw32 = ((size_t)g->n + 31) / 32;
  L.inq[0] = c.take<uint32_t>(nw32);
  L.inq[1] = c.take<uint32_t>(nw32);
  L.infar = c.take<uint32_t>(nw32);
  L.q[0] = c.take<int32_t>(g->n);
  L.q[1] = c.take<int32_t>(g->n);
  L.far[0] = c.take<int32_t>(g->n);
  L.far[1] = c.take<int32_t>(g->n);
  L.desc = c.take<int2>((size_t)(g->m / CH) + (size_t)g->n + 64);
  L.bytes = c.used;
  return L;
}

int g_sssp_occ[64];

// Default near-far step: 64 (the wave width) times the mean edge weight over
// the mean degree of the vertices with edges, so one step of the threshold
// admits about a wave's worth of edges per frontier vertex; at least 1.
uint32_t fg_sssp_default_delta(const fg_graph* g) {
  if (g->m <= 0 || g->nonzero_degree <= 0) return 1u;
  const double mean_w = (double)g->w_sum / (double)g->m;
  const double mean_deg = (double)g->m / (double)g->nonzero_degree;
  const double d = 64.0 * mean_w / mean_deg;
  if (d >= 4294967295.0) return DIST_INF;
  return d < 1.0 ? 1u : (uint32_t)(d + 0.5);
}

}  // namespace

size_t fg_sssp_workspace_bytes(const fg_graph* g) { return sssp_layout(g, nullptr).bytes; }

extern "C" void fg_sssp_opts_default(fg_sssp_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
}

extern "C" fg_status fg_sssp(const fg_graph* g, int32_t src, const fg_sssp_opts* opts, void* ws,
                             size_t ws_bytes, uint32_t* dist, int32_t* parent,
                             fg_run_stats* stats, void* stream) {
  if (!g) return fg_set_error(FG_EINVAL, "fg_sssp: graph is NULL");
  if (src < 0 || src >= g->n)
    return fg_set_error(FG_EINVAL, "fg_sssp: src=%d outside [0, %d)", src, g->n);
  if (!dist) return fg_set_error(FG_EINVAL, "fg_sssp: dist is NULL");
  if (!ws) return fg_set_error(FG_EINVAL, "fg_sssp: workspace is NULL");
  if (!g->w) return fg_set_error(FG_EINVAL, "fg_sssp: the graph was loaded without weights");
  fg_sssp_opts o;
  if (opts) o = *opts; else fg_sssp_opts_default(&o);
  SsspLayout lay = sssp_layout(g, ws);
  FG_CHECK_WS_ALIGN(ws, "fg_sssp");
  if (ws_bytes < lay.bytes)
    return fg_set_error(FG_ENOMEM, "fg_sssp: workspace of %zu bytes < required %zu", ws_bytes,
                        lay.bytes);
  int dev = 0;
  FG_HIP_TRY(hipGetDevice(&dev));
  fg_device_props pr = fg_props(dev);
  if (!pr.coop) return fg_set_error(FG_EUNSUPPORTED, "fg_sssp: device lacks cooperative launch");
  if (dev >= 0 && dev < 64 && g_sssp_occ[dev] == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, sssp_persistent<true>, PB, 0) !=
            hipSuccess ||
        nb < 1)
      nb = 1;
    g_sssp_occ[dev] = nb;
  }
  int bpc = (dev >= 0 && dev < 64) ? g_sssp_occ[dev] : 1;
  if (o.blocks_per_cu > 0 && o.blocks_per_cu < bpc) bpc = o.blocks_per_cu;
  if (o.blocks_per_cu == 0 && bpc > 2) bpc = 2;
  int grid = pr.cus * bpc;
  if (o.grid_blocks > 0 && o.grid_blocks < grid) grid = o.grid_blocks;

  SsspParams P;
  memset(&P, 0, sizeof(P));
  P.off = g->off;
  P.col = g->col;
  P.w = g->w;
  P.n = g->n;
  P.nw32 = (int32_t)(((int64_t)g->n + 31) / 32);
  P.src = src;
  P.dist = dist;
  P.parent = parent;
  P.key = lay.key;
  P.inq[0] = lay.inq[0];
  P.inq[1] = lay.inq[1];
  P.infar = lay.infar;
  P.q[0] = lay.q[0];
  P.q[1] = lay.q[1];
  P.far[0] = lay.far[0];
  P.far[1] = lay.far[1];
  P.desc = lay.desc;
  P.ctl = lay.ctl;
  P.stats = stats;
  P.small_q = o.small_frontier > 0 ? o.small_frontier : DEF_SMALL_Q;
  if (P.small_q > PB) P.small_q = PB;
  P.small_e = o.small_edges > 0 ? o.small_edges : DEF_SMALL_E;
  P.big_deg = o.big_degree > 0 ? o.big_degree : DEF_BIG_DEG;
  P.delta = o.delta > 0 ? o.delta : fg_sssp_default_delta(g);
  // by default the team kernel runs on graphs of mean degree <= 8 (grids,
  // road-like graphs), where near frontiers are long and thin
  const bool low_deg = g->m <= (int64_t)TEAM_AUTO_DEG * g->n;
  P.team = o.team_blocks > 0 ? o.team_blocks : (o.team_blocks < 0 || !low_deg ? 1 : DEF_TEAM);
  if (P.team > TEAM_MAX) P.team = TEAM_MAX;
  if (P.team > grid) P.team = grid;
  P.team_e = o.team_edges > 0 ? o.team_edges : DEF_TEAM_E;
  if (P.team_e > TW_CAP - 1) P.team_e = TW_CAP - 1;
  P.clock_khz = pr.clock_khz;
  void* args[] = {&P};
  const void* kern = P.team > 1 ? (const void*)sssp_persistent<true>
                                : (const void*)sssp_persistent<false>;
  FG_HIP_TRY(hipLaunchCooperativeKernel(kern, dim3(grid), dim3(PB), args, 0, (hipStream_t)stream));
  return FG_OK;
}
