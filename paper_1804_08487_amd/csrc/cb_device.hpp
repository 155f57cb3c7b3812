// Device-side helpers for the gfx950 global Curveball library: the counter
// random numbers, agent-scope atomics and fences, and wavefront primitives.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cbx {

constexpr uint32_t kTagMatch = 0x4D415443u;   // node sort keys
constexpr uint32_t kTagSplit = 0x46595348u;   // split draws
constexpr int32_t kUnmatched = 0x7fffffff;    // trade of the node left out
constexpr int kWave = 64;

// Error bits of the device error word.
constexpr int32_t kErrWatchdog = 1;
constexpr int32_t kErrInbox = 2;       // more arrivals than the row has slots
constexpr int32_t kErrOut = 4;         // more final edges than the row has slots
constexpr int32_t kErrDep = 8;         // dependency counter went below zero
constexpr int32_t kErrGather = 16;     // trade saw a row of the wrong size
constexpr int32_t kErrCapacity = 32;   // size outside what a tier can hold
constexpr int32_t kErrRows = 64;       // rebuilt row count differs from degree
constexpr int32_t kErrInvalid = 128;   // upload validation failed
constexpr int32_t kErrMatch = 256;     // matching bucket beyond capacity

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11); returns (w1 << 32) | w0.
__device__ __forceinline__ uint64_t philox64(uint64_t seed, uint32_t c0, uint32_t c1,
                                             uint32_t c2, uint32_t c3) {
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return ((uint64_t)c1 << 32) | c0;
}

// floor(x * k / 2^64)
__device__ __forceinline__ uint64_t bounded(uint64_t x, uint64_t k) { return __umul64hi(x, k); }

// ---- agent-scope memory operations ---------------------------------------
__device__ __forceinline__ int32_t atomic_add(int32_t* p, int32_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t atomic_or(int32_t* p, int32_t v) {
  return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool atomic_cas(int32_t* p, int32_t expected, int32_t desired) {
  return __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED,
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t load_agent(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_agent(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int64_t load_agent64(const int64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long load_agent_u64(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_agent_u64(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_agent64(int64_t* p, int64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t atomic_and(int32_t* p, int32_t v) {
  return __hip_atomic_fetch_and(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// On failure *expected receives the current value.
__device__ __forceinline__ bool atomic_cas_u64(unsigned long long* p, unsigned long long* expected,
                                               unsigned long long desired) {
  return __hip_atomic_compare_exchange_strong(p, expected, desired, __ATOMIC_RELAXED,
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Ordering between trades. Every datum one trade hands to another inside
// the trade kernel (inbox entries, bitmap words, counters, queue slots) is
// written and read with agent-scope atomic operations, which are coherent
// across the XCDs' L2 caches (agent-scope stores and loads are issued with
// sc1 and go to the coherence point; read-modify-write atomics are
// performed there). So a producer only has to let its writes complete
// before the counter update that publishes them, and a consumer's reads
// depend on the value that handed it the work. Full agent-scope fences
// (an L2 write-back plus an L2 invalidate around every trade) are not
// needed for that data; data read by later kernels is ordered by the kernel
// boundary.
__device__ __forceinline__ void publish_wait() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}
__device__ __forceinline__ void consume_order() { __atomic_signal_fence(__ATOMIC_SEQ_CST); }

// ---- wavefront primitives -------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

// Number of set bits of `mask` below this lane.
__device__ __forceinline__ int rank_below(uint64_t mask) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                        __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }
__device__ __forceinline__ int popc64(uint64_t m) { return __popcll(m); }

// Orders this wavefront's LDS accesses across lanes (no cross-wave effect).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Value of a 32-bit variable in lane src_lane (the same for every lane).
__device__ __forceinline__ int32_t wave_bcast(int32_t v, int src_lane) {
  return __builtin_amdgcn_readlane(v, src_lane);
}

// Inclusive prefix sum across the wavefront (every lane active), in
// registers: shifts by 1, 2, 4 and 8 lanes inside each row of 16, then the
// total of row 0 added to row 1 and of row 2 to row 3 (broadcast of lane 15),
// then the total of rows 0-1 added to rows 2-3 (broadcast of lane 31).
__device__ __forceinline__ int32_t wave_incl_scan(int32_t v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return v;
}

// Sum over the wavefront (every lane active), the same in every lane.
__device__ __forceinline__ int32_t wave_sum(int32_t v) {
  return __builtin_amdgcn_readlane(wave_incl_scan(v), kWave - 1);
}

__device__ __forceinline__ uint32_t next_pow2(uint32_t x) {
  if (x <= 1) return 1;
  return 1u << (32 - __clz(x - 1));
}

// Constant-rate clock (used only by the watchdog).
__device__ __forceinline__ uint64_t now_ticks() { return wall_clock64(); }

}  // namespace cbx
