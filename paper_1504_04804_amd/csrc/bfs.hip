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
//   desc      int2[m/CH + n + 64]     edge-chunk descriptors {vertex, first edge}
//   control   barrier, counters, hand-back state of the small-frontier mode
#include <string.h>

#include "frontier.h"

namespace {
using namespace fgk;

constexpr int PB = 1024;          // persistent workgroup size
constexpr int PWAVES = PB / FG_WAVE;
constexpr int CH = 256;           // edges per descriptor
constexpr int DIR_PUSH = 0, DIR_PULL = 1;

constexpr int32_t DEF_SMALL_Q = 1024;
constexpr int64_t DEF_SMALL_E = 4096;
constexpr int32_t DEF_BIG_DEG = 64;
constexpr int32_t DEF_TEAM = 16;
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
  uint32_t exit_count;         // workgroups that left the launch
  uint32_t pad3[63];
  uint32_t team_arrive;        // barrier of the team (workgroups 0..team-1)
  uint32_t pad4[63];
  Line64 aux;                  // entries written by bitmap -> queue conversion
  CtrSlot slot[2];
  // state published by workgroup 0 when a small-frontier / team episode ends
  int32_t pub_k, pub_dir, pub_prevdir, pub_switched, pub_qsel, pub_force;
  int64_t pub_qlen, pub_p, pub_insp_sum;
  int32_t pub_switches;
  int64_t pub_qdeg;
  ull pub_b[8];
};

struct BfsParams {
  const int32_t* __restrict__ off;
  const int32_t* __restrict__ col;
  const uint64_t* __restrict__ nz;
  int32_t n;
  int32_t nwords;
  int64_t m;
  int32_t src;
  int32_t mode;
  int32_t* depth;
  int32_t* parent;
  uint64_t* vis[2];
  int32_t* q[2];
  int2* desc;
  BfsCtl* ctl;
  fg_run_stats* stats;
  uint32_t a_num, a_den, b_num, b_den;
  int32_t small_q;
  int64_t small_e;
  int32_t big_deg;
  int32_t clock_khz;
  int32_t team;     // workgroups of the team mode (0 = off)
  int64_t team_e;   // team mode while the frontier's degree sum <= team_e
};

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

__device__ __forceinline__ void trace_iter(const St& S, const BfsParams& P) {
  if (blockIdx.x == 0 && threadIdx.x == 0 && P.stats && S.k < FG_TRACE_MAX) {
    P.stats->dir[S.k] = (int8_t)S.dir;
    P.stats->frontier[S.k] = S.qlen;
  }
}

__device__ __forceinline__ void trace_insp(int32_t k, int64_t insp, const BfsParams& P) {
  if (blockIdx.x == 0 && threadIdx.x == 0 && P.stats && k < FG_TRACE_MAX) {
    P.stats->inspected[k] = insp;
    P.stats->t_end[k] = (int64_t)wall_clock64();
  }
}

// Filter step fused into the advance: test-and-set of the visited bit.
__device__ __forceinline__ bool try_visit(int32_t v, int32_t src, int32_t d,
                                          uint32_t* vis32, const BfsParams& P) {
  const uint32_t bit = 1u << (v & 31);
  uint32_t* wp = vis32 + (v >> 5);
  if (*wp & bit) return false;  // plain pre-check; a stale 0 only costs the atomic
  const uint32_t old = atomicOr(wp, bit);
  if (old & bit) return false;
  P.depth[v] = d;
  if (P.parent) P.parent[v] = src;
  return true;
}

constexpr int STAGE = 512;   // per-wave LDS staging of discovered vertices
constexpr int DSTAGE = 128;  // per-wave LDS staging of descriptors

struct Lds {
  int32_t stage[PWAVES][STAGE];
  int2 dstage[PWAVES][DSTAGE];
  // per-wave scan-gather staging (push, full grid)
  int32_t w_sc[PWAVES][FG_WAVE];
  int32_t w_u[PWAVES][FG_WAVE];
  int32_t w_b[PWAVES][FG_WAVE];
  // block-level staging (small-frontier mode)
  int32_t b_sc[PB];
  int32_t b_u[PB];
  int32_t b_b[PB];
  int64_t red[PWAVES + 1];
  int32_t red32[PWAVES + 1];
  int32_t newcnt;
  int32_t flag;
  int64_t bcast[20];
};

// ---- push, full grid, phase A: each wave takes 64-entry chunks of the
// frontier (static stride).  Vertices below big_deg are expanded by a
// wave-level scan-gather; the others become CH-edge descriptors.
__device__ void push_phase_a(const BfsParams& P, const St& S, Lds& L, uint32_t nblocks) {
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
  WaveStage<int2, DSTAGE> dst{L.dstage[wid], 0};
  const int64_t gw = (int64_t)blockIdx.x * PWAVES + wid;
  const int64_t W = (int64_t)nblocks * PWAVES;
  int64_t insp = 0, ndeg = 0;
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
    for (int32_t t0 = 0; t0 < T; t0 += FG_WAVE) {
      const int32_t t = t0 + lane;
      bool won = false;
      int32_t v = 0;
      if (t < T) {
        const int32_t j = upper_idx(sc, FG_WAVE, t);
        v = P.col[sb[j] + (t - sc[j])];
        won = try_visit(v, su[j], d_new, vis32, P);
        if (won) ndeg += P.off[v + 1] - P.off[v];
      }
      st.push(won, v, &C.q.v, B.q, Qout);
    }
  }
  st.flush(&C.q.v, B.q, Qout);
  dst.flush(&C.desc.v, B.desc, P.desc);
  const int64_t tot = fg_block_sum<PB>(insp, L.red);
  const int64_t tdeg = fg_block_sum<PB>(ndeg, L.red);
  if (threadIdx.x == 0) {
    if (tot) atomicAdd(&C.insp.v, (ull)tot);
    if (tdeg) atomicAdd(&C.deg.v, (ull)tdeg);
  }
}

// ---- push, full grid, phase B: waves take descriptors in turn; the CH
// edges of a descriptor are contiguous, so each round is one coalesced read
// of 64 column indices and no search is needed.
__device__ void push_phase_b(const BfsParams& P, const St& S, int64_t ndesc, Lds& L,
                             uint32_t nblocks) {
  const int lane = fg_lane();
  const int wid = threadIdx.x / FG_WAVE;
  const int64_t gw = (int64_t)blockIdx.x * PWAVES + wid;
  const int64_t W = (int64_t)nblocks * PWAVES;
  int64_t ndeg = 0;
  int32_t* Qout = P.q[S.qsel ^ 1];
  uint32_t* vis32 = (uint32_t*)P.vis[S.cur];
  const int32_t d_new = S.k + 1;
  CtrSlot& C = P.ctl->slot[S.k & 1];
  const Bases B = get_bases(S);
  WaveStage<int32_t, STAGE> st{L.stage[wid], 0};
  for (int64_t i = gw; i < ndesc; i += W) {
    const int2 dsc = P.desc[i];
    const int32_t u = dsc.x;
    const int32_t e_end = P.off[u + 1];
    const int32_t e1 = dsc.y + CH < e_end ? dsc.y + CH : e_end;
    // CH / 64 rounds, loads first so the rounds' reads overlap
    int32_t vv[CH / FG_WAVE];
#pragma unroll
    for (int r = 0; r < CH / FG_WAVE; ++r) {
      const int32_t e = dsc.y + r * FG_WAVE + lane;
      vv[r] = e < e1 ? P.col[e] : -1;
    }
#pragma unroll
    for (int r = 0; r < CH / FG_WAVE; ++r) {
      const int32_t v = vv[r];
      const bool won = v >= 0 && try_visit(v, u, d_new, vis32, P);
      if (won) ndeg += P.off[v + 1] - P.off[v];
      st.push(won, v, &C.q.v, B.q, Qout);
    }
  }
  st.flush(&C.q.v, B.q, Qout);
  const int64_t tdeg = fg_block_sum<PB>(ndeg, L.red);
  if (threadIdx.x == 0 && tdeg) atomicAdd(&C.deg.v, (ull)tdeg);
}

// ---- pull, full grid: each wave owns 64 consecutive vertices (one bitmap
// word).  An unvisited vertex of nonzero degree scans its CSR row in order
// and stops at the first visited neighbour: for an unvisited v every
// visited neighbour has depth exactly k (depths differ by at most one across
// an edge), so that neighbour is in the current frontier.  The next bitmap
// word is written whole, so no atomics are needed.
__device__ void pull_phase(const BfsParams& P, const St& S, Lds& L) {
  const int lane = fg_lane();
  const int wid = threadIdx.x / FG_WAVE;
  const int64_t gw = (int64_t)blockIdx.x * PWAVES + wid;
  const int64_t W = (int64_t)gridDim.x * PWAVES;
  const uint64_t* Vin = P.vis[S.cur];
  uint64_t* Vout = P.vis[S.cur ^ 1];
  const int32_t d_new = S.k + 1;
  int64_t insp = 0, ndeg = 0;
  int32_t nnew = 0;
  for (int64_t w = gw; w < P.nwords; w += W) {
    const uint64_t vis = Vin[w];
    const uint64_t act = P.nz[w] & ~vis;
    uint64_t nb = 0;
    if (act) {
      const int32_t v = (int32_t)(w * 64 + lane);
      bool found = false;
      int32_t pu = -1;
      if ((act >> lane) & 1ull) {
        const int32_t b0 = P.off[v];
        const int32_t e = P.off[v + 1];
        for (int32_t i = b0; i < e; ++i) {
          const int32_t u = P.col[i];
          insp++;
          if ((Vin[u >> 6] >> (u & 63)) & 1ull) {
            found = true;
            pu = u;
            break;
          }
        }
        if (found) ndeg += e - b0;
      }
      nb = __ballot(found);
      if (found) {
        P.depth[v] = d_new;
        if (P.parent) P.parent[v] = pu;
      }
      nnew += __popcll(nb);
    }
    if (lane == 0) Vout[w] = vis | nb;
  }
  if (lane != 0) nnew = 0;
  const int64_t tot = fg_block_sum<PB>(insp, L.red);
  const int64_t tdeg = fg_block_sum<PB>(ndeg, L.red);
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
__device__ void bitmap_diff_to_queue(const BfsParams& P, const St& S) {
  const int lane = fg_lane();
  const uint64_t* Vnew = P.vis[S.cur];
  const uint64_t* Vold = P.vis[S.cur ^ 1];
  int32_t* Q = P.q[S.qsel];
  const int64_t tid = (int64_t)blockIdx.x * PB + threadIdx.x;
  const int64_t nth = (int64_t)gridDim.x * PB;
  for (int64_t w0 = tid - lane; w0 < P.nwords; w0 += nth) {
    const int64_t w = w0 + lane;
    uint64_t diff = 0;
    if (w < P.nwords) diff = Vnew[w] & ~Vold[w];
    const int32_t c = __popcll(diff);
    const int32_t inc = fg_wave_incl_scan(c);
    const int32_t tot = __shfl(inc, FG_WAVE - 1, FG_WAVE);
    ull base = 0;
    if (lane == FG_WAVE - 1 && tot) base = atomicAdd(&P.ctl->aux.v, (ull)tot);
    base = __shfl(base, FG_WAVE - 1, FG_WAVE) - S.auxbase;
    int64_t pos = (int64_t)base + inc - c;
    while (diff) {
      const int bit = __builtin_ctzll(diff);
      diff &= diff - 1;
      Q[pos++] = (int32_t)(w * 64 + bit);
    }
  }
}

// ---- small-frontier mode, workgroup 0 only: push levels run back to back
// with workgroup barriers while |Q| <= small_q and the frontier's degree sum
// <= small_e.  Returns with S describing the next iteration.
template <int MODE>
__device__ void small_mode(const BfsParams& P, St& S, Lds& L) {
  const int tid = threadIdx.x;
  for (;;) {
    const int32_t* Qin = P.q[S.qsel];
    int32_t* Qout = P.q[S.qsel ^ 1];
    uint32_t* vis32 = (uint32_t*)P.vis[S.cur];
    if (tid == 0) L.newcnt = 0;
    const int32_t d_new = S.k + 1;
    int64_t ndeg = 0;
    for (int64_t c0 = 0; c0 < S.qlen; c0 += PB) {
      const int64_t i = c0 + tid;
      int32_t u = 0, b = 0, d = 0;
      if (i < S.qlen) {
        u = Qin[i];
        b = P.off[u];
        d = P.off[u + 1] - b;
      }
      int32_t T = 0;
      const int32_t ex = fg_block_excl_scan<PB>(d, L.red32, &T);
      L.b_sc[tid] = ex;
      L.b_u[tid] = u;
      L.b_b[tid] = b;
      __syncthreads();
      const int32_t cnt = (int32_t)((S.qlen - c0) < PB ? (S.qlen - c0) : PB);
      for (int32_t t0 = 0; t0 < T; t0 += PB) {
        const int32_t t = t0 + tid;
        bool won = false;
        int32_t v = 0;
        if (t < T) {
          const int32_t j = upper_idx(L.b_sc, cnt, t);
          v = P.col[L.b_b[j] + (t - L.b_sc[j])];
          won = try_visit(v, L.b_u[j], d_new, vis32, P);
          if (won) ndeg += P.off[v + 1] - P.off[v];
        }
        const uint64_t mask = __ballot(won);
        if (mask) {
          int32_t pos = 0;
          if (fg_lane() == 0) pos = atomicAdd(&L.newcnt, __popcll(mask));
          pos = __shfl(pos, 0, FG_WAVE);
          if (won) Qout[pos + fg_mbcnt(mask)] = v;
        }
      }
      __syncthreads();
    }
    const int64_t nqdeg = fg_uni(fg_block_sum<PB>(ndeg, L.red));
    const int64_t nq = fg_uni((int64_t)L.newcnt);
    trace_insp(S.k, S.qdeg, P);
    S.insp_sum += S.qdeg;
    S.k++;
    S.qsel ^= 1;
    S.qlen = nq;
    S.qdeg = nqdeg;
    S.p += nq;
    decide<MODE>(S, P);
    trace_iter(S, P);
    __syncthreads();
    if (nq == 0 || S.dir != DIR_PUSH || nq > P.small_q || nqdeg > P.small_e) return;
  }
}

// ---- team mode: workgroups 0..team-1 run push levels back to back with a
// barrier among themselves while the frontier's degree sum is at most
// team_e (and above the small-frontier limits); the other workgroups wait.
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

template <int MODE>
__device__ bool team_mode(const BfsParams& P, St& S, Lds& L, TeamSync& ts) {
  for (;;) {
    CtrSlot& C = P.ctl->slot[S.k & 1];
    Bases B = get_bases(S);
    push_phase_a(P, S, L, ts.T);
    if (!ts.sync(&L.flag)) return false;
    const ull dt = fg_atomic_load_u64(&C.desc.v);
    const int64_t ndesc = (int64_t)(dt - B.desc);
    if (ndesc > 0) {
      push_phase_b(P, S, ndesc, L, ts.T);
      if (!ts.sync(&L.flag)) return false;
    }
    B.desc = dt;
    const ull qt = fg_atomic_load_u64(&C.q.v);
    const ull it = fg_atomic_load_u64(&C.insp.v);
    const ull gt = fg_atomic_load_u64(&C.deg.v);
    const int64_t nq = (int64_t)(qt - B.q);
    const int64_t insp = (int64_t)(it - B.insp);
    const int64_t nqdeg = (int64_t)(gt - B.deg);
    B.q = qt;
    B.insp = it;
    B.deg = gt;
    set_bases(S, B);
    trace_insp(S.k, insp, P);
    S.insp_sum += insp;
    S.k++;
    S.qsel ^= 1;
    S.qlen = nq;
    S.qdeg = nqdeg;
    S.p += nq;
    decide<MODE>(S, P);
    trace_iter(S, P);
    if (nq == 0 || S.dir != DIR_PUSH || nqdeg > P.team_e ||
        (nq <= P.small_q && nqdeg <= P.small_e))
      return true;
  }
}

// MODE is FG_MODE_DO or FG_MODE_PUSH (one kernel per mode).
template <int MODE>
__global__ __launch_bounds__(PB) void bfs_persistent(BfsParams P) {
  __shared__ Lds L;
  fg_grid_sync gs{P.ctl->bar, gridDim.x, 0u};
  St S = {};
  S.dir = DIR_PUSH;
  S.prevdir = DIR_PUSH;
  S.qlen = 1;
  S.p = 1;
  uint32_t sm_seen = 0;
  bool ok = true;
  TeamSync ts{&P.ctl->team_arrive, P.ctl->bar + FG_BAR_STRIDE, (uint32_t)P.team, 0u};
  // a1: depth = parent = -1 except at the source, visited = {src}, Q = {src}
  {
    const int64_t tid = (int64_t)blockIdx.x * PB + threadIdx.x;
    const int64_t nth = (int64_t)gridDim.x * PB;
    const int32_t src = P.src;
    if (blockIdx.x == 0 && P.stats) {
      uint32_t* sw = (uint32_t*)P.stats;
      for (int i = threadIdx.x; i < (int)(sizeof(fg_run_stats) / 4); i += PB) sw[i] = 0u;
    }
    const bool vec = ((((uintptr_t)P.depth) | ((uintptr_t)(P.parent ? P.parent : P.depth))) & 15) == 0;
    if (vec) {
      const int64_t n4 = P.n / 4;
      int4* d4 = (int4*)P.depth;
      int4* p4 = (int4*)P.parent;
      for (int64_t i = tid; i < n4; i += nth) {
        const bool hit = (src >> 2) == i;
        const int r = src & 3;
        const int4 d = make_int4(hit && r == 0 ? 0 : -1, hit && r == 1 ? 0 : -1,
                                 hit && r == 2 ? 0 : -1, hit && r == 3 ? 0 : -1);
        const int4 pp = make_int4(hit && r == 0 ? src : -1, hit && r == 1 ? src : -1,
                                  hit && r == 2 ? src : -1, hit && r == 3 ? src : -1);
        d4[i] = d;
        if (P.parent) p4[i] = pp;
      }
      for (int64_t i = n4 * 4 + tid; i < P.n; i += nth) {
        P.depth[i] = i == src ? 0 : -1;
        if (P.parent) P.parent[i] = i == src ? src : -1;
      }
    } else {
      for (int64_t i = tid; i < P.n; i += nth) {
        P.depth[i] = i == src ? 0 : -1;
        if (P.parent) P.parent[i] = i == src ? src : -1;
      }
    }
    uint64_t* v0 = P.vis[0];
    for (int64_t w = tid; w < P.nwords; w += nth)
      v0[w] = (w == (src >> 6)) ? (1ull << (src & 63)) : 0ull;
    if (tid == 0) P.q[0][0] = src;
    if (!gs.sync(&L.flag)) ok = false;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && P.stats) {
    P.stats->t_start = (int64_t)wall_clock64();
    P.stats->clock_khz = P.clock_khz;
  }
  S.qdeg = fg_uni((int32_t)(P.off[P.src + 1] - P.off[P.src]));
  trace_iter(S, P);
  while (ok && S.qlen > 0) {
    // backward -> forward: list the last pull's discoveries first
    if (MODE == FG_MODE_DO && S.dir == DIR_PUSH && S.prevdir == DIR_PULL) {
      bitmap_diff_to_queue(P, S);
      if (!(ok = gs.sync(&L.flag))) break;
      S.auxbase = fg_atomic_load_u64(&P.ctl->aux.v);
      S.prevdir = DIR_PUSH;
    }
    const bool small_ep = S.dir == DIR_PUSH && S.qlen <= P.small_q && S.qdeg <= P.small_e;
    const bool team_ep = !small_ep && S.dir == DIR_PUSH && P.team > 1 && S.qdeg <= P.team_e;
    if (small_ep || team_ep) {
      sm_seen++;
      const bool member = small_ep ? blockIdx.x == 0 : blockIdx.x < (uint32_t)P.team;
      if (member) {
        if (small_ep) {
          small_mode<MODE>(P, S, L);
        } else if (!team_mode<MODE>(P, S, L, ts)) {
          ok = false;
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) {
          BfsCtl* c = P.ctl;
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
        }
        __syncthreads();
        if (!ok) break;
      } else {
        if (threadIdx.x == 0) {
          const int bad = !fg_wait_geq(&P.ctl->sm_signal, sm_seen, P.ctl->bar + FG_BAR_STRIDE, 64);
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
    if (MODE != FG_MODE_DO || S.dir == DIR_PUSH) {
      push_phase_a(P, S, L, gridDim.x);
      if (!(ok = gs.sync(&L.flag))) break;
      const ull dt = fg_atomic_load_u64(&C.desc.v);
      const int64_t ndesc = (int64_t)(dt - B.desc);
      if (ndesc > 0) {
        push_phase_b(P, S, ndesc, L, gridDim.x);
        if (!(ok = gs.sync(&L.flag))) break;
      }
      B.desc = dt;
      S.qsel ^= 1;
    } else {
      pull_phase(P, S, L);
      if (!(ok = gs.sync(&L.flag))) break;
      S.cur ^= 1;
    }
    const ull qt = fg_atomic_load_u64(&C.q.v);
    const ull it = fg_atomic_load_u64(&C.insp.v);
    const ull gt = fg_atomic_load_u64(&C.deg.v);
    const int64_t nq = (int64_t)(qt - B.q);
    const int64_t insp = (int64_t)(it - B.insp);
    B.q = qt;
    B.insp = it;
    S.qdeg = (int64_t)(gt - B.deg);
    B.deg = gt;
    set_bases(S, B);
    trace_insp(S.k, insp, P);
    S.insp_sum += insp;
    S.k++;
    S.qlen = nq;
    S.p += nq;
    decide<MODE>(S, P);
    trace_iter(S, P);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && P.stats) {
    fg_run_stats* st = P.stats;
    st->status = ok ? FG_OK : FG_EDEVICE;
    st->iterations = S.k;
    st->reached = S.p;
    st->edges_inspected = S.insp_sum;
    st->direction_switches = S.switches;
    st->grid_blocks = (int32_t)gridDim.x;
  }
  // the last workgroup out clears the control block for the next launch
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t done = __hip_atomic_fetch_add(&P.ctl->exit_count, 1u, __ATOMIC_ACQ_REL,
                                                 __HIP_MEMORY_SCOPE_AGENT);
    L.flag = done == gridDim.x - 1;
  }
  __syncthreads();
  if (L.flag) {
    uint32_t* w = (uint32_t*)P.ctl;
    for (int i = threadIdx.x; i < (int)(sizeof(BfsCtl) / 4); i += PB) w[i] = 0u;
  }
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
  int2* desc;
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
  L.desc = c.take<int2>((size_t)(g->m / CH) + (size_t)g->n + 64);
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
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, bfs_persistent<MODE>, PB, 0) !=
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

extern "C" fg_status fg_bfs(const fg_graph* g, int32_t src, const fg_bfs_opts* opts, void* ws,
                            size_t ws_bytes, int32_t* depth, int32_t* parent,
                            fg_run_stats* stats, void* stream) {
  if (!g) return fg_set_error(FG_EINVAL, "fg_bfs: graph is NULL");
  if (src < 0 || src >= g->n)
    return fg_set_error(FG_EINVAL, "fg_bfs: src=%d outside [0, %d)", src, g->n);
  if (!depth) return fg_set_error(FG_EINVAL, "fg_bfs: depth is NULL");
  if (!ws) return fg_set_error(FG_EINVAL, "fg_bfs: workspace is NULL");
  fg_bfs_opts o;
  if (opts) o = *opts; else fg_bfs_opts_default(&o);
  if (o.mode != FG_MODE_DO && o.mode != FG_MODE_PUSH && o.mode != FG_MODE_PUSH_UNFUSED)
    return fg_set_error(FG_EINVAL, "fg_bfs: unknown mode %d", o.mode);
  if (o.mode == FG_MODE_DO) {
    if (!g->symmetric)
      return fg_set_error(FG_EUNSUPPORTED,
                          "fg_bfs: the pull step needs an undirected graph (FG_SYMMETRIC)");
    if (o.do_a_den == 0 || o.do_b_den == 0)
      return fg_set_error(FG_EINVAL, "fg_bfs: zero denominator in do_a / do_b");
  }
  if (o.mode == FG_MODE_PUSH_UNFUSED)
    return fg_bfs_unfused(g, src, ws, ws_bytes, depth, parent, stats, (hipStream_t)stream);
  BfsLayout lay = bfs_layout(g, ws);
  if (ws_bytes < lay.bytes)
    return fg_set_error(FG_ENOMEM, "fg_bfs: workspace of %zu bytes < required %zu", ws_bytes,
                        lay.bytes);
  int dev = 0;
  FG_HIP_TRY(hipGetDevice(&dev));
  fg_device_props pr = fg_props(dev);
  if (!pr.coop) return fg_set_error(FG_EUNSUPPORTED, "fg_bfs: device lacks cooperative launch");
  int bpc = o.mode == FG_MODE_DO ? persistent_blocks_per_cu<FG_MODE_DO>(dev)
                                 : persistent_blocks_per_cu<FG_MODE_PUSH>(dev);
  if (o.blocks_per_cu > 0 && o.blocks_per_cu < bpc) bpc = o.blocks_per_cu;
  if (o.blocks_per_cu == 0 && bpc > 2) bpc = 2;
  const int grid = pr.cus * bpc;
  hipStream_t s = (hipStream_t)stream;

  BfsParams P;
  memset(&P, 0, sizeof(P));
  P.off = g->off;
  P.col = g->col;
  P.nz = g->nzmask;
  P.n = g->n;
  P.nwords = g->nwords;
  P.m = g->m;
  P.src = src;
  P.mode = o.mode;
  P.depth = depth;
  P.parent = parent;
  P.vis[0] = lay.vis[0];
  P.vis[1] = lay.vis[1];
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
  if (P.small_q > PB) P.small_q = PB;
  P.small_e = o.small_edges > 0 ? o.small_edges : DEF_SMALL_E;
  P.big_deg = o.big_degree > 0 ? o.big_degree : DEF_BIG_DEG;
  P.clock_khz = pr.clock_khz;

  void* args[] = {&P};
  const void* fn = o.mode == FG_MODE_DO ? (const void*)bfs_persistent<FG_MODE_DO>
                                        : (const void*)bfs_persistent<FG_MODE_PUSH>;
  FG_HIP_TRY(hipLaunchCooperativeKernel(fn, dim3(grid), dim3(PB), args, 0, s));
  return FG_OK;
}
