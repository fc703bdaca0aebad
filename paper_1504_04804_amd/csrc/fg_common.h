// Shared host/device helpers of libfg (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/fg.h"

// ---------------------------------------------------------------- host side

// Records a thread-local error message and returns `code`.
fg_status fg_set_error(fg_status code, const char* fmt, ...);

#define FG_HIP_TRY(expr)                                                       \
  do {                                                                         \
    hipError_t _e = (expr);                                                    \
    if (_e != hipSuccess)                                                      \
      return fg_set_error(FG_EDEVICE, "%s failed: %s (%s:%d)", #expr,          \
                          hipGetErrorString(_e), __FILE__, __LINE__);          \
  } while (0)

struct fg_graph {
  int32_t n = 0;
  int64_t m = 0;
  int32_t nwords = 0;       // ceil(n / 64)
  const int32_t* off = nullptr;
  const int32_t* col = nullptr;
  const uint32_t* w = nullptr;
  uint64_t* nzmask = nullptr;  // bit v set iff deg(v) > 0, nwords words
  int4* head = nullptr;        // first four neighbours of each vertex (see graph.hip)
  void* owned[4] = {nullptr, nullptr, nullptr, nullptr};
  int32_t symmetric = 0;
  int32_t max_degree = 0;
  int32_t nonzero_degree = 0;
  uint64_t w_sum = 0;   // sum of the weights (0 without weights)
  uint32_t w_max = 0;   // largest weight
  int32_t device = 0;
  int64_t resident_bytes = 0;
};

// Internal entry points shared between translation units.
size_t fg_bfs_workspace_bytes(const fg_graph* g);
size_t fg_ops_workspace_bytes(const fg_graph* g, bool with_bfs);
size_t fg_sssp_workspace_bytes(const fg_graph* g);
size_t fg_msbfs_workspace_bytes(const fg_graph* g, int32_t lanes);
size_t fg_mssp_workspace_bytes(const fg_graph* g);
size_t fg_pr_workspace_bytes(const fg_graph* g);
size_t fg_cc_workspace_bytes(const fg_graph* g);
void fg_bfs_launch_init(const fg_graph* g, int32_t src, int32_t* depth, int32_t* parent,
                        uint64_t* vis0, int32_t* q0, fg_run_stats* stats, hipStream_t s,
                        void* ctl, int32_t ctl_bytes);
fg_status fg_bfs_unfused(const fg_graph* g, int32_t src, void* ws, size_t ws_bytes,
                         int32_t* depth, int32_t* parent, fg_run_stats* stats, hipStream_t s);

// Device properties used for persistent launches (cached per device).
struct fg_device_props {
  int cus;
  int coop;
  int clock_khz;  // device wall clock (wall_clock64) rate
};
fg_device_props fg_props(int device);

static inline size_t fg_align(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspaces are carved into 256-byte aligned pieces from their start, so
// the start must be 256-byte aligned too (every hipMalloc allocation is).
#define FG_CHECK_WS_ALIGN(ws, fn)                                                      \
  do {                                                                                 \
    if (((uintptr_t)(ws) & 255u) != 0)                                                 \
      return fg_set_error(FG_EINVAL, fn ": workspace %p is not 256-byte aligned", (ws)); \
  } while (0)

// Carves a caller workspace into 256-byte aligned pieces.
struct fg_carver {
  char* base;
  size_t used = 0;
  explicit fg_carver(void* b) : base((char*)b) {}
  template <class T>
  T* take(size_t count) {
    T* p = base ? (T*)(base + used) : nullptr;
    used += fg_align(count * sizeof(T));
    return p;
  }
};

// ------------------------------------------------------------- device side

#define FG_WAVE 64

__device__ __forceinline__ int fg_lane() { return (int)__lane_id(); }

// Number of set bits of `mask` below the calling lane.
__device__ __forceinline__ int fg_mbcnt(uint64_t mask) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                        __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Inclusive prefix sum over the 64 lanes of a wave.
template <class T>
__device__ __forceinline__ T fg_wave_incl_scan(T x) {
  const int lane = fg_lane();
#pragma unroll
  for (int d = 1; d < FG_WAVE; d <<= 1) {
    T y = __shfl_up(x, d, FG_WAVE);
    if (lane >= d) x += y;
  }
  return x;
}

// 32-bit version through DPP row shifts and row broadcasts: six VALU
// operations and no LDS traffic (the generic one above waits on six
// dependent cross-lane permutes).  All 64 lanes must be active.
__device__ __forceinline__ int32_t fg_wave_incl_scan(int32_t x) {
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);  // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);  // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);  // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);  // row_shr:8
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15 -> rows 1, 3
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31 -> rows 2, 3
  return x;
}

template <class T>
__device__ __forceinline__ T fg_wave_sum(T x) {
#pragma unroll
  for (int d = FG_WAVE / 2; d > 0; d >>= 1) x += __shfl_xor(x, d, FG_WAVE);
  return x;
}

// 64-bit value of lane l (l wave-uniform).
__device__ __forceinline__ unsigned long long fg_readlane64(unsigned long long x, int l) {
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)x, l);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), l);
  return ((unsigned long long)hi << 32) | lo;
}

// Wave-wide OR of 32 / 64-bit values through DPP (all lanes active);
// the result is wave-uniform.
__device__ __forceinline__ uint32_t fg_wave_or32(uint32_t x) {
  int32_t y = (int32_t)x;
  y |= __builtin_amdgcn_update_dpp(0, y, 0x111, 0xf, 0xf, false);  // row_shr:1
  y |= __builtin_amdgcn_update_dpp(0, y, 0x112, 0xf, 0xf, false);  // row_shr:2
  y |= __builtin_amdgcn_update_dpp(0, y, 0x114, 0xf, 0xf, false);  // row_shr:4
  y |= __builtin_amdgcn_update_dpp(0, y, 0x118, 0xf, 0xf, false);  // row_shr:8
  y |= __builtin_amdgcn_update_dpp(0, y, 0x142, 0xa, 0xf, false);  // row_bcast:15
  y |= __builtin_amdgcn_update_dpp(0, y, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return (uint32_t)__builtin_amdgcn_readlane(y, FG_WAVE - 1);
}
__device__ __forceinline__ unsigned long long fg_wave_or64(unsigned long long x) {
  const uint32_t lo = fg_wave_or32((uint32_t)x);
  const uint32_t hi = fg_wave_or32((uint32_t)(x >> 32));
  return ((unsigned long long)hi << 32) | lo;
}

// Wave total of 32-bit values (DPP scan, then the last lane's value).
__device__ __forceinline__ int32_t fg_wave_sum(int32_t x) {
  return __builtin_amdgcn_readlane(fg_wave_incl_scan(x), FG_WAVE - 1);
}

// Wave-uniform copies (scalar registers) of values every lane holds equally.
__device__ __forceinline__ int32_t fg_uni(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t fg_uni(int64_t x) {
  const int32_t lo = __builtin_amdgcn_readfirstlane((int32_t)(uint32_t)(uint64_t)x);
  const int32_t hi = __builtin_amdgcn_readfirstlane((int32_t)(uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
__device__ __forceinline__ unsigned long long fg_uni(unsigned long long x) {
  return (unsigned long long)fg_uni((int64_t)x);
}

__device__ __forceinline__ uint32_t fg_atomic_load_u32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Relaxed load of a counter every lane reads at the same address; the result
// is made wave-uniform so the compiler keeps it in scalar registers.
__device__ __forceinline__ unsigned long long fg_atomic_load_u64(const unsigned long long* p) {
  return fg_uni((unsigned long long)__hip_atomic_load(p, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT));
}

// Bounded wait: poll `*p` (relaxed, no cache invalidation per poll) until
// (int32)(*p - target) >= 0, then one agent-scope acquire fence.  Gives up
// when `abort_flag` is set or after FG_SPIN_LIMIT polls (then sets it), so
// every workgroup leaves the kernel even if a peer never arrives.
// `sleep_cycles` sets the pause between polls: >= 4096 for waits that may
// be long (about 500 clocks for the first 64 polls, 2K for the next 192,
// then 4K), which keeps idle workgroups from hammering the counter's memory
// channel.
#define FG_SPIN_LIMIT (1u << 24)

__device__ __forceinline__ bool fg_wait_geq(const uint32_t* p, uint32_t target,
                                            uint32_t* abort_flag, int sleep_cycles) {
  uint32_t spins = 0;
  for (;;) {
    uint32_t now = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((int32_t)(now - target) >= 0) break;
    if ((++spins & 31u) == 0 &&
        __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      return false;
    if (spins > FG_SPIN_LIMIT) {
      __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    if (sleep_cycles >= 4096) {
      // long waits (a hand-off after an episode of any length): short
      // pauses first, so the end of a short episode is seen within a few
      // hundred cycles, then ever fewer polls
      if (spins < 64) __builtin_amdgcn_s_sleep(8);
      else if (spins < 256) __builtin_amdgcn_s_sleep(32);
      else __builtin_amdgcn_s_sleep(64);
    } else if (sleep_cycles > 8) {
      __builtin_amdgcn_s_sleep(8);
    } else {
      __builtin_amdgcn_s_sleep(1);
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return true;
}

// Hand-off of an episode's state (small-frontier or team episodes) from
// workgroup 0 to the workgroups that waited for it: each waiter
// acknowledges once it has read the published fields, and workgroup 0 waits
// for every acknowledgement of the previous episode before it writes the
// fields again.  Without this, two episodes that end a few microseconds
// apart let a slow waiter read the second episode's state as the first's,
// after which its iteration count, and so its barrier count, differ from
// the other workgroups'.
__device__ __forceinline__ void fg_handoff_ack(uint32_t* ack) {
  __builtin_amdgcn_s_waitcnt(0);  // the published fields have been read
  __hip_atomic_fetch_add(ack, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Stores of data that other workgroups read after a barrier which does not
// write back the L2 (fg_grid_sync::sync_acquire): agent-scope atomic stores
// write through to the point of coherence, so no dirty copy stays in one
// XCD's L2.
__device__ __forceinline__ void fg_st_shared(int32_t* p, int32_t x) {
  __hip_atomic_store(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void fg_st_shared(uint32_t* p, uint32_t x) {
  __hip_atomic_store(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void fg_st_shared(uint64_t* p, uint64_t x) {
  __hip_atomic_store(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void fg_st_shared(unsigned long long* p, unsigned long long x) {
  __hip_atomic_store(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void fg_st_shared(int2* p, const int2& x) {
  __hip_atomic_store((unsigned long long*)p, ((unsigned long long)(uint32_t)x.y << 32) | (uint32_t)x.x,
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void fg_st_shared(int4* p, const int4& x) {
  unsigned long long* q = (unsigned long long*)p;
  __hip_atomic_store(q, ((unsigned long long)(uint32_t)x.y << 32) | (uint32_t)x.x,
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(q + 1, ((unsigned long long)(uint32_t)x.w << 32) | (uint32_t)x.z,
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Device-wide barrier for cooperative (co-resident) launches, two levels:
// workgroups arrive at their group's counter (groups of FG_BAR_GROUP
// consecutive workgroups); the last arrival of a group arrives at the global
// counter, waits for every group, then releases its group through the
// group's flag.  All counters are monotone (barrier c completes when they
// reach c times the number of arrivals) and start at zero for the launch.
// `ctl` must hold FG_BAR_WORDS 32-bit words, one 256-byte line per counter.
#define FG_BAR_GROUP 32
#define FG_BAR_STRIDE 64  // words between counters (256 bytes)
#define FG_BAR_MAXG 32
#define FG_BAR_WORDS (FG_BAR_STRIDE * (2 * FG_BAR_MAXG + 2))

struct fg_grid_sync {
  uint32_t* ctl;       // [0] global arrivals, [1] abort, then per-group pairs
  uint32_t nblocks;
  uint32_t count;      // barriers passed by this workgroup

  __device__ uint32_t* abort_flag() const { return ctl + FG_BAR_STRIDE; }
  __device__ uint32_t* group_arrive(uint32_t g) const { return ctl + FG_BAR_STRIDE * (2 + 2 * g); }
  __device__ uint32_t* group_release(uint32_t g) const {
    return ctl + FG_BAR_STRIDE * (3 + 2 * g);
  }

  // Returns false if the grid was aborted.  Every thread of every workgroup
  // must call it the same number of times.
  __device__ bool sync(int* s_flag) {
    __syncthreads();
    if (threadIdx.x == 0) {
      count++;
      const uint32_t g = blockIdx.x / FG_BAR_GROUP;
      const uint32_t ngroups = (nblocks + FG_BAR_GROUP - 1) / FG_BAR_GROUP;
      const uint32_t gsize = (g + 1 < ngroups) ? FG_BAR_GROUP : nblocks - g * FG_BAR_GROUP;
      int ok = 1;
      const uint32_t old = __hip_atomic_fetch_add(group_arrive(g), 1u, __ATOMIC_RELEASE,
                                                  __HIP_MEMORY_SCOPE_AGENT);
      if (old == count * gsize - 1) {
        // last of its group: global level
        __hip_atomic_fetch_add(ctl, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        ok = fg_wait_geq(ctl, count * ngroups, abort_flag(), 1);
        if (ok)
          __hip_atomic_store(group_release(g), count, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        ok = fg_wait_geq(group_release(g), count, abort_flag(), 1);
      }
      *s_flag = !ok;
    }
    __syncthreads();
    return *s_flag == 0;
  }

  // The same barrier without the L2 write-back (the costly half of sync()
  // when lines are dirty): for phases whose outputs read by other
  // workgroups are atomics or fg_st_shared stores.  Every wave first waits
  // for its own memory operations, the arrivals are relaxed, and each
  // workgroup ends with one agent-scope acquire (fg_wait_geq), so plain
  // loads after the barrier see what the other workgroups wrote.  Plain
  // stores made before it stay unordered with other workgroups.
  __device__ bool sync_acquire(int* s_flag) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
      count++;
      const uint32_t g = blockIdx.x / FG_BAR_GROUP;
      const uint32_t ngroups = (nblocks + FG_BAR_GROUP - 1) / FG_BAR_GROUP;
      const uint32_t gsize = (g + 1 < ngroups) ? FG_BAR_GROUP : nblocks - g * FG_BAR_GROUP;
      int ok = 1;
      const uint32_t old = __hip_atomic_fetch_add(group_arrive(g), 1u, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
      if (old == count * gsize - 1) {
        __hip_atomic_fetch_add(ctl, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = fg_wait_geq(ctl, count * ngroups, abort_flag(), 1);
        if (ok)
          __hip_atomic_store(group_release(g), count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        ok = fg_wait_geq(group_release(g), count, abort_flag(), 1);
      }
      *s_flag = !ok;
    }
    __syncthreads();
    return *s_flag == 0;
  }
};

// Block-wide sum for blocks of BT threads (BT multiple of 64); `scratch`
// needs BT/64 elements of LDS.  Every thread of the block must call it.
template <int BT, class T>
__device__ __forceinline__ T fg_block_sum(T x, T* scratch) {
  x = fg_wave_sum(x);
  const int wid = threadIdx.x / FG_WAVE;
  __syncthreads();
  if (fg_lane() == 0) scratch[wid] = x;
  __syncthreads();
  T s = 0;
#pragma unroll
  for (int i = 0; i < BT / FG_WAVE; ++i) s += scratch[i];
  return s;
}

// Block-wide exclusive scan (BT threads); returns the exclusive prefix and
// the block total in *total.  `scratch` needs BT/64 + 1 elements of LDS.
template <int BT, class T>
__device__ __forceinline__ T fg_block_excl_scan(T x, T* scratch, T* total) {
  const int wid = threadIdx.x / FG_WAVE;
  T inc = fg_wave_incl_scan(x);
  __syncthreads();
  if (fg_lane() == FG_WAVE - 1) scratch[wid] = inc;
  __syncthreads();
  T before = 0, all = 0;
#pragma unroll
  for (int i = 0; i < BT / FG_WAVE; ++i) {
    T v = scratch[i];
    before += (i < wid) ? v : (T)0;
    all += v;
  }
  *total = all;
  return before + inc - x;
}
