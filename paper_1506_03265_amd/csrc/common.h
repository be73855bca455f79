// Shared device and host helpers of libcldiam (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/cldiam.h"

#define CLD_INF64 (~(uint64_t)0)
#define CLD_INF32 (0xffffffffu)
#define CLD_DELTA_MAX ((uint64_t)1 << 31)

// ------------------------------------------------------------ host errors --
namespace cld {

void set_error(const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);

#define CLD_HIP(call)                                                   \
  do {                                                                  \
    hipError_t e_ = (call);                                             \
    if (e_ != hipSuccess) return ::cld::hip_fail(e_, #call);            \
  } while (0)

#define CLD_LAUNCH_CHECK(what)                                          \
  do {                                                                  \
    hipError_t e_ = hipGetLastError();                                  \
    if (e_ != hipSuccess) return ::cld::hip_fail(e_, what);             \
  } while (0)

// Bump allocator over a caller workspace; every piece is 256-byte aligned.
struct Arena {
  char *base;
  size_t cap, used;
  Arena(void *p, size_t c) : base((char *)p), cap(c), used(0) {}
  template <class T>
  T *take(size_t count) {
    size_t bytes = (count * sizeof(T) + 255) & ~(size_t)255;
    size_t at = used;
    used += bytes;
    if (base == nullptr || used > cap) return nullptr;
    return (T *)(base + at);
  }
};

// Sizing twin of Arena (no pointer needed).
struct Sizer {
  size_t used = 0;
  template <class T>
  void take(size_t count) { used += (count * sizeof(T) + 255) & ~(size_t)255; }
};

// Pooled pinned host buffers of kPinnedBytes for readbacks (nullptr when the
// request is larger or the allocation fails); give each one back after use.
constexpr size_t kPinnedBytes = 4096;
void *pinned_acquire(size_t bytes);
void pinned_release(void *p);

// Holds a pooled pinned buffer for the lifetime of a call.
template <class T>
struct Pinned {
  T *p;
  Pinned() : p((T *)pinned_acquire(sizeof(T))) {}
  ~Pinned() { pinned_release(p); }
  Pinned(const Pinned &) = delete;
  Pinned &operator=(const Pinned &) = delete;
};

inline int blocks_for(int64_t items, int threads, int cap = 1 << 20) {
  int64_t b = (items + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

}  // namespace cld

// ---------------------------------------------------------- device helpers --

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds, multipliers
// 0xD2511F53 / 0xCD9E8D57, key increments 0x9E3779B9 / 0xBB67AE85.
__device__ __forceinline__ uint32_t cld_philox_word0(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                     uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
    uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
    uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
  }
  return c0;
}

__device__ __forceinline__ int cld_lane() { return (int)(threadIdx.x & 63); }

// Wave-aggregated reservation of `pred ? 1 : 0` slots on a counter.  Works
// with any subset of active lanes; returns the slot of a predicated lane.
__device__ __forceinline__ uint32_t cld_wave_reserve(bool pred, uint32_t *counter) {
  unsigned long long mask = __ballot(pred);
  uint32_t slot = 0;
  if (mask) {
    int leader = __ffsll((long long)mask) - 1;
    int lane = cld_lane();
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(counter, (uint32_t)__popcll(mask));
    base = __shfl(base, leader);
    slot = base + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
  }
  return slot;
}

// Min / max / sum over the lanes that are active, result broadcast to them.
__device__ __forceinline__ uint64_t cld_wave_min_u64(uint64_t v) {
  unsigned long long mask = __ballot(true);
  while (mask) {
    int src = __ffsll((long long)mask) - 1;
    mask &= mask - 1;
    uint64_t o = __shfl(v, src);
    v = o < v ? o : v;
  }
  return v;
}

// ------------------------------------------------------------ grid barrier --
struct CldBarrier {
  uint32_t count;
  uint32_t gen;
};

// Generation barrier for a cooperative (co-resident) grid.  Device-scope
// release/acquire fences make every write before the barrier visible to
// every workgroup after it.  A wait longer than ~20 s of the 100 MHz wall
// clock sets *timeout and returns false so that every wave can leave.
__device__ inline bool cld_grid_barrier(CldBarrier *bar, uint32_t *timeout, uint32_t nblocks) {
  __shared__ uint32_t ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    ok = 1;
    __threadfence();
    const uint32_t gen = __hip_atomic_load(&bar->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t arrived = atomicAdd(&bar->count, 1u);
    if (arrived == nblocks - 1) {
      __hip_atomic_store(&bar->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&bar->gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      const uint64_t t0 = wall_clock64();
      while (__hip_atomic_load(&bar->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        __builtin_amdgcn_s_sleep(1);
        if (wall_clock64() - t0 > 2000000000ull) {
          __hip_atomic_store(timeout, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
      }
    }
    __threadfence();
  }
  __syncthreads();
  return ok != 0;
}

namespace cld {
// Co-resident grid size for a cooperative launch of `kernel` (0 = none).
int cooperative_blocks(const void *kernel, int threads, int max_per_cu, int *blocks);
}  // namespace cld
