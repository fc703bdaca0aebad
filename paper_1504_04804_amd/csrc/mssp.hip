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
    for (int i = fg_lane(); i < cnt; i += FG_WAVE) out[pos + i] = buf[i];
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
  for (int32_t k = 0; ok && k < P.k_iters && live != 0ull; ++k) {
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
            Fc[u] = 0ull;  // only this thread reads u's word in this iteration
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
            P.desc[d0 + t] = make_int4(su[j], sb[j] + (t - sc[j]) * CHS, (int32_t)(uint32_t)mj,
                                       (int32_t)(uint32_t)(mj >> 32));
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
    if (!(ok = gs.sync(&L.flag))) break;
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
      if (!(ok = gs.sync(&L.flag))) break;
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
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, mssp_persistent, PB, 0) != hipSuccess ||
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
  P.delta = b->opts.delta > 0 ? b->opts.delta : default_delta(g);
  P.big_deg = b->opts.big_degree > 0 ? b->opts.big_degree : 4 * CHS;
  if (P.big_deg > 65536) P.big_deg = 65536;  // keeps a wave's (edge, lane) count in int32
  P.dense = b->opts.dense_lanes > 0 ? b->opts.dense_lanes : 16;
  P.split_lanes = b->opts.split_lanes > 0 ? b->opts.split_lanes : 8;
  P.split_wait = b->opts.split_wait > 0 ? b->opts.split_wait : 8;
  void* args[] = {&P};
  int grid = pr.cus * bpc;
  if (b->opts.grid_blocks > 0 && b->opts.grid_blocks < grid) grid = b->opts.grid_blocks;
  FG_HIP_TRY(hipLaunchCooperativeKernel((const void*)mssp_persistent, dim3(grid),
                                        dim3(PB), args, 0, (hipStream_t)stream));
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
