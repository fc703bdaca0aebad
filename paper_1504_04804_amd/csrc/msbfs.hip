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
  int32_t pad[12];
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
  int64_t bcast[4];
  int32_t start[MAXL];  // iteration at which each lane was admitted
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
      Fc[u] = 0ull;  // only this thread reads u's word in this iteration
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
  for (int32_t k = 0; ok && k < P.k_iters && S.live != 0ull; ++k) {
    const int32_t it1 = S.it + 1;
    const bool want_pull = S.mode == 0 ? S.qlen > P.n / P.pull_div : S.qlen >= P.n / P.push_div;
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
          Fn[v] = 0ull;
        }
        st.push(act, (int32_t)v, &C.cnt.v, cbp, P.q[S.qsel]);
      }
      st.flush(&C.cnt.v, cbp, P.q[S.qsel]);
      if (!(ok = gs.sync(&L.flag))) break;
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
          Qlong[atomicAdd(&C.q.v, 1ull) - qbp] = (int32_t)v;
          const int64_t d0 = (int64_t)(atomicAdd(&C.desc.v, (ull)nch) - dbp);
          for (int32_t c = 0; c < nch; ++c) P.desc[d0 + c] = make_int4((int32_t)v, b + 4 + c * CH, 0, 0);
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
          if (nw && !lng) P.visit[v] = vis | nw;
          Fn[v] = nw;
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
      if (!(ok = gs.sync(&L.flag))) break;
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
          if (!(ok = gs.sync(&L.flag))) break;
          ull lor2 = 0;
          int32_t act2 = 0;
          for (int64_t i = tid; i < nlong; i += nth) {
            const int32_t v = Qlong[i];
            const ull vis = P.visit[v];
            const ull nw = Fn[v] & S.live & ~vis;
            Fn[v] = nw;
            if (nw) {
              P.visit[v] = vis | nw;
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
          if (!(ok = gs.sync(&L.flag))) break;
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
      if (!(ok = gs.sync(&L.flag))) break;
      const ull dt = fg_atomic_load_u64(&C.desc.v);
      const int64_t ndesc = (int64_t)(dt - dbp);
      if (ndesc > 0) {
        ull got2 = 0;
        push_desc(P, S, k, ndesc, qbp, L, got2);
        const ull bor = block_or(got2, L.redu);
        if (threadIdx.x == 0 && bor) atomicOr(livew, bor);
        if (!(ok = gs.sync(&L.flag))) break;
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
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, msbfs_persistent, PB, 0) != hipSuccess ||
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
  P.push_div = b->opts.push_div > 0 ? b->opts.push_div : 512;
  void* args[] = {&P};
  int grid = pr.cus * bpc;
  if (b->opts.grid_blocks > 0 && b->opts.grid_blocks < grid) grid = b->opts.grid_blocks;
  FG_HIP_TRY(hipLaunchCooperativeKernel((const void*)msbfs_persistent, dim3(grid),
                                        dim3(PB), args, 0, (hipStream_t)stream));
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
