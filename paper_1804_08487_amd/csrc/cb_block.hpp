// Workgroup-level building blocks: prefix sums, in-LDS bitonic sort, and a
// stable LSD radix sort of one segment in global memory.
#pragma once

#include "cb_device.hpp"

namespace cbx {

// Exclusive prefix sum over a workgroup of `nthreads` (a multiple of 64,
// at most 1024). `scratch` holds nthreads / 64 + 1 ints. Returns the
// exclusive prefix of v; *total receives the sum. Contains barriers.
__device__ __forceinline__ int32_t block_excl_scan(int32_t v, int32_t* scratch, int32_t* total) {
  const int tid = threadIdx.x;
  const int w = tid >> 6;
  const int nw = blockDim.x >> 6;
  const int32_t inc = wave_incl_scan(v);
  if (lane_id() == kWave - 1) scratch[w] = inc;
  __syncthreads();
  if (tid == 0) {
    int32_t acc = 0;
    for (int i = 0; i < nw; ++i) {
      const int32_t t = scratch[i];
      scratch[i] = acc;
      acc += t;
    }
    scratch[nw] = acc;
  }
  __syncthreads();
  const int32_t r = scratch[w] + inc - v;
  *total = scratch[nw];
  __syncthreads();
  return r;
}

// Ascending bitonic sort of a[0..s) with every comparator ascending (the
// first step of each merge compares mirror positions), so entries past s act
// as +infinity and are simply skipped. Workgroup-wide; contains barriers.
template <typename T>
__device__ void block_bitonic_sort(T* a, uint32_t s) {
  if (s <= 1) return;
  const uint32_t P = next_pow2(s);
  const uint32_t half = P >> 1;
  for (uint32_t k2 = 2; k2 <= P; k2 <<= 1) {
    const uint32_t h = k2 >> 1;
    for (uint32_t p = threadIdx.x; p < half; p += blockDim.x) {
      const uint32_t i = (p / h) * k2 + (p % h);
      const uint32_t j = i ^ (k2 - 1);
      if (j < s) {
        const T x = a[i], y = a[j];
        if (y < x) { a[i] = y; a[j] = x; }
      }
    }
    __syncthreads();
    for (uint32_t d = k2 >> 2; d > 0; d >>= 1) {
      for (uint32_t p = threadIdx.x; p < half; p += blockDim.x) {
        const uint32_t i = (p / d) * 2 * d + (p % d);
        const uint32_t j = i + d;
        if (j < s) {
          const T x = a[i], y = a[j];
          if (y < x) { a[i] = y; a[j] = x; }
        }
      }
      __syncthreads();
    }
  }
}

// Same network run by one wavefront on its own LDS region.
template <typename T>
__device__ void wave_bitonic_sort(T* a, uint32_t s) {
  if (s <= 1) return;
  const uint32_t P = next_pow2(s);
  const uint32_t half = P >> 1;
  const uint32_t l = (uint32_t)lane_id();
  for (uint32_t k2 = 2; k2 <= P; k2 <<= 1) {
    const uint32_t h = k2 >> 1;
    for (uint32_t p = l; p < half; p += kWave) {
      const uint32_t i = (p / h) * k2 + (p % h);
      const uint32_t j = i ^ (k2 - 1);
      if (j < s) {
        const T x = a[i], y = a[j];
        if (y < x) { a[i] = y; a[j] = x; }
      }
    }
    wave_sync();
    for (uint32_t d = k2 >> 2; d > 0; d >>= 1) {
      for (uint32_t p = l; p < half; p += kWave) {
        const uint32_t i = (p / d) * 2 * d + (p % d);
        const uint32_t j = i + d;
        if (j < s) {
          const T x = a[i], y = a[j];
          if (y < x) { a[i] = y; a[j] = x; }
        }
      }
      wave_sync();
    }
  }
}

// LDS needed by block_radix_sort.
struct RadixLds {
  int32_t hist[256];
  int32_t offs[256];
  int32_t wcnt[16][257];   // per-wave digit counts of one tile (at most 16 waves)
  int32_t scan[17];
};

template <typename T> __device__ __forceinline__ uint32_t radix_key(T e);
template <> __device__ __forceinline__ uint32_t radix_key<uint64_t>(uint64_t e) { return (uint32_t)(e >> 32); }
template <> __device__ __forceinline__ uint32_t radix_key<int32_t>(int32_t e) { return (uint32_t)e; }

// Stable LSD radix sort (8-bit digits) of s elements by the low `keybits`
// bits of radix_key(), ping-ponging between a and b (both global memory,
// s elements each). Returns the buffer that holds the sorted sequence.
// Workgroup-wide (blockDim a multiple of 64, at most 1024); barriers inside.
template <typename T>
__device__ __forceinline__ T* block_radix_sort(T* a, T* b, int64_t s, int keybits, RadixLds& R) {
  const int tid = threadIdx.x;
  const int w = tid >> 6;
  const int nw = blockDim.x >> 6;
  const uint64_t lt = (1ull << lane_id()) - 1ull;
  T* src = a;
  T* dst = b;
  for (int shift = 0; shift < keybits; shift += 8) {
    for (int d = tid; d < 256; d += blockDim.x) R.hist[d] = 0;
    __syncthreads();
    for (int64_t i = tid; i < s; i += blockDim.x)
      atomicAdd(&R.hist[(radix_key<T>(src[i]) >> shift) & 255u], 1);
    __syncthreads();
    // A digit that holds every element leaves the order unchanged.
    bool single = false;
    for (int d = 0; d < 256; ++d) single |= (R.hist[d] == s);
    if (single) continue;   // uniform across the workgroup
    if (tid == 0) {
      int32_t acc = 0;
      for (int d = 0; d < 256; ++d) { R.offs[d] = acc; acc += R.hist[d]; }
    }
    for (int i = tid; i < nw * 257; i += blockDim.x) R.wcnt[i / 257][i % 257] = 0;
    __syncthreads();
    for (int64_t tile = 0; tile < s; tile += blockDim.x) {
      const int64_t i = tile + tid;
      const bool valid = i < s;
      T e{};
      uint32_t dg = 256;
      if (valid) {
        e = src[i];
        dg = (radix_key<T>(e) >> shift) & 255u;
      }
      uint64_t peers = ballot(valid);
      if (!valid) peers = ~peers;
#pragma unroll
      for (int bit = 0; bit < 8; ++bit) {
        const bool on = (dg >> bit) & 1u;
        const uint64_t bb = ballot(on);
        peers &= on ? bb : ~bb;
      }
      const int rank = popc64(peers & lt);
      if (valid && rank == 0) R.wcnt[w][dg] = popc64(peers);
      __syncthreads();
      if (valid) {
        int32_t pre = 0;
        for (int q = 0; q < w; ++q) pre += R.wcnt[q][dg];
        dst[R.offs[dg] + pre + rank] = e;
      }
      __syncthreads();
      for (int d = tid; d < 256; d += blockDim.x) {
        int32_t t = 0;
        for (int q = 0; q < nw; ++q) { t += R.wcnt[q][d]; R.wcnt[q][d] = 0; }
        R.offs[d] += t;
      }
      __syncthreads();
    }
    T* t = src; src = dst; dst = t;
  }
  return src;
}

// Stable LSD radix sort (8-bit digits) of a[0..s) by the low `keybits` bits
// of (e >> 32), through b[0..s) (each in LDS or global memory; the passes
// alternate between them). Wavefront w ranks the fixed
// segment [w * seg, (w + 1) * seg) in order, so a pass needs three barriers:
// per-wavefront digit counts, offsets in (digit, wavefront) order, scatter.
// cnt: (blockDim / 64) * 256 ints of LDS; scan: blockDim / 64 + 1 ints.
// Returns the buffer that holds the sorted sequence. Workgroup-wide.
__device__ __forceinline__ uint64_t* seg_radix_sort(uint64_t* a, uint64_t* b, int32_t s, int keybits,
                                                    int32_t* cnt, int32_t* scan) {
  const int tid = threadIdx.x;
  const int w = tid >> 6;
  const int l = lane_id();
  const int nw = blockDim.x >> 6;
  const uint64_t lt = (1ull << l) - 1ull;
  const int32_t seg = ((s + nw - 1) / nw + kWave - 1) / kWave * kWave;
  const int32_t lo = w * seg < s ? w * seg : s;
  const int32_t hi = lo + seg < s ? lo + seg : s;
  int32_t* c = cnt + w * 256;
  uint64_t* src = a;
  uint64_t* dst = b;
  for (int shift = 0; shift < keybits; shift += 8) {
    for (int d = l; d < 256; d += kWave) c[d] = 0;
    wave_sync();
    for (int32_t i = lo + l; i < hi; i += kWave) atomicAdd(&c[(uint32_t)(src[i] >> (32 + shift)) & 255u], 1);
    __syncthreads();
    int32_t tot = 0;
    if (tid < 256)
      for (int q = 0; q < nw; ++q) tot += cnt[q * 256 + tid];
    int32_t all;
    const int32_t base = block_excl_scan(tid < 256 ? tot : 0, scan, &all);
    if (tid < 256) {
      int32_t run = base;
      for (int q = 0; q < nw; ++q) {
        const int32_t t = cnt[q * 256 + tid];
        cnt[q * 256 + tid] = run;
        run += t;
      }
    }
    __syncthreads();
    for (int32_t i0 = lo; i0 < hi; i0 += kWave) {
      const int32_t i = i0 + l;
      const bool valid = i < hi;
      uint64_t e = 0;
      uint32_t dg = 256;
      if (valid) {
        e = src[i];
        dg = (uint32_t)(e >> (32 + shift)) & 255u;
      }
      uint64_t peers = ballot(valid);
      if (!valid) peers = ~peers;
#pragma unroll
      for (int bit = 0; bit < 8; ++bit) {
        const bool on = (dg >> bit) & 1u;
        const uint64_t bb = ballot(on);
        peers &= on ? bb : ~bb;
      }
      const int rank = popc64(peers & lt);
      if (valid) dst[c[dg] + rank] = e;
      wave_sync();
      if (valid && rank == 0) c[dg] += popc64(peers);
      wave_sync();
    }
    __syncthreads();
    uint64_t* t = src;
    src = dst;
    dst = t;
  }
  return src;
}

}  // namespace cbx
