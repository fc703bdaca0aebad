// Device building blocks shared by the persistent traversal kernels
// (BFS and SSSP): padded counters, per-wave LDS staging of outputs, and the
// wave-level search used by the scan-gather expansion.
#pragma once

#include "fg_common.h"

namespace fgk {

typedef unsigned long long ull;

// One 256-byte line per counter so concurrent atomics do not share a line.
struct alignas(256) Line64 {
  ull v;
  ull pad[31];
};

// Entries are staged per wave in LDS and written out with one global atomic
// per batch, so concurrent waves do not serialise on the shared counter.
template <class T, int CAP>
struct WaveStage {
  T* buf;
  int32_t cnt;

  __device__ __forceinline__ void flush(ull* total, ull base, T* out) {
    if (cnt == 0) return;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    ull pos = 0;
    if (fg_lane() == 0) pos = atomicAdd(total, (ull)cnt);
    pos = __shfl(pos, 0, FG_WAVE) - base;
    // written through: read by other workgroups after the next barrier
    for (int i = fg_lane(); i < cnt; i += FG_WAVE) fg_st_shared(&out[pos + i], buf[i]);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    cnt = 0;
  }

  __device__ __forceinline__ void push(bool keep, const T& x, ull* total, ull base, T* out) {
    const uint64_t mask = __ballot(keep);
    if (!mask) return;
    const int32_t c = __popcll(mask);
    if (cnt + c > CAP) flush(total, base, out);
    if (keep) buf[cnt + fg_mbcnt(mask)] = x;
    cnt += c;
  }
};

__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Largest j in [0, cnt) with sc[j] <= t (sc non-decreasing).
__device__ __forceinline__ int32_t upper_idx(const int32_t* sc, int32_t cnt, int32_t t) {
  int32_t lo = 0, hi = cnt - 1;
  while (lo < hi) {
    int32_t mid = (lo + hi + 1) >> 1;
    if (sc[mid] <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}


}  // namespace fgk
