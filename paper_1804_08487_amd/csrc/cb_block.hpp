// Workgroup-level building blocks: prefix sums, in-LDS bitonic sort, a
// bucket sort of entries with distinct keys, and stable LSD radix sorts.
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

// Largest bucket the bucket sorts below rank (a fuller one sends the caller
// to another sort); also the margin of the staged sort's LDS windows.
constexpr int32_t kBucketMax = 256;

// Bucket bits for s entries: at most 16 entries per bucket on average, no
// more than maxbits bits and no more bits than the keys have.
__device__ __forceinline__ int bucket_bits(int32_t s, int keybits, int maxbits) {
  int lb = 0;
  while (lb < maxbits && lb < keybits && (16 << lb) < s) ++lb;
  return lb;
}

typedef __attribute__((address_space(3))) uint64_t lds_u64;
typedef __attribute__((address_space(3))) int32_t lds_i32;

// Bucket sort: ascending sort of a[0..s) by the whole 64-bit value into
// out[0..s), where every key (e >> 32) is below 2^keybits. A counting scatter
// by the top lb bits of the key moves the entries from a into buf (cnt: 2^lb
// LDS counters), then an entry's place within its bucket is the number of
// smaller entries in the bucket (equal ones, which distinct keys never give,
// are ordered by their position in buf). a and out may be the same array;
// buf overlaps neither. Workgroup-wide; barriers inside; *flag is LDS.
constexpr int kBucketBatch = 8;   // loads in flight per thread

struct Buckets {
  int32_t nb;
  int sh;
  // the bucket of an entry (clamped, so a stray key cannot leave the arrays)
  __device__ __forceinline__ uint32_t of(uint64_t e) const {
    const uint32_t b = (uint32_t)(e >> 32) >> sh;
    return b < (uint32_t)nb ? b : (uint32_t)nb - 1u;
  }
};

// Counting and scatter passes. False, with a and out untouched, if a bucket
// holds more than kBucketMax entries. Afterwards cnt[b] is the end of bucket
// b in buf and the start of bucket b + 1.
template <typename T, typename U>
__device__ __forceinline__ bool bucket_scatter(const T* a, U* buf, int32_t s, const Buckets& K, lds_i32* cnt,
                                               lds_i32* scan, lds_i32* flag) {
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  for (int32_t b = tid; b < K.nb; b += nt) cnt[b] = 0;
  if (tid == 0) *flag = 0;
  __syncthreads();
  for (int32_t i0 = tid; i0 < s; i0 += kBucketBatch * nt) {
    uint64_t v[kBucketBatch];
#pragma unroll
    for (int r = 0; r < kBucketBatch; ++r) v[r] = i0 + r * nt < s ? a[i0 + r * nt] : 0;
#pragma unroll
    for (int r = 0; r < kBucketBatch; ++r)
      if (i0 + r * nt < s) atomicAdd((int32_t*)&cnt[K.of(v[r])], 1);
  }
  __syncthreads();
  // each thread scans a run of consecutive buckets
  const int32_t per = (K.nb + nt - 1) / nt;
  const int32_t b0 = tid * per < K.nb ? tid * per : K.nb;
  const int32_t b1 = b0 + per < K.nb ? b0 + per : K.nb;
  int32_t sum = 0;
  bool full = false;
  for (int32_t b = b0; b < b1; ++b) {
    const int32_t c = cnt[b];
    sum += c;
    full |= c > kBucketMax;
  }
  if (full) *flag = 1;
  int32_t tot;
  int32_t run = block_excl_scan(sum, (int32_t*)scan, &tot);   // its barriers publish *flag
  if (*flag) return false;                                    // uniform
  for (int32_t b = b0; b < b1; ++b) {
    const int32_t c = cnt[b];
    cnt[b] = run;
    run += c;
  }
  __syncthreads();
  for (int32_t i0 = tid; i0 < s; i0 += kBucketBatch * nt) {
    uint64_t v[kBucketBatch];
#pragma unroll
    for (int r = 0; r < kBucketBatch; ++r) v[r] = i0 + r * nt < s ? a[i0 + r * nt] : 0;
#pragma unroll
    for (int r = 0; r < kBucketBatch; ++r)
      if (i0 + r * nt < s) buf[atomicAdd((int32_t*)&cnt[K.of(v[r])], 1)] = v[r];
  }
  __syncthreads();
  return true;
}

// Place of the entry at position i of src (bucket-ordered, positions offset
// by base) in the sorted order.
template <typename U>
__device__ __forceinline__ int32_t bucket_rank(const U* src, int32_t base, int32_t i, uint64_t e,
                                               const Buckets& K, const lds_i32* cnt) {
  const uint32_t b = K.of(e);
  const int32_t lo = b ? cnt[b - 1] : 0;
  const int32_t hi = cnt[b];
  int32_t r = lo;
  for (int32_t j = lo; j < hi; ++j) {
    const uint64_t x = src[j - base];
    r += (x < e || (x == e && j < i)) ? 1 : 0;
  }
  return r;
}

// All three arrays in LDS. Kept out of line, like the variant below: the
// trade kernel has no registers to spare for them.
// False, with a and out untouched, if a bucket holds more than kBucketMax
// entries.
__device__ __noinline__ bool bucket_sort_lds(lds_u64* a, lds_u64* buf, lds_u64* out, int32_t s, int keybits,
                                             int lb, lds_i32* cnt, lds_i32* scan, lds_i32* flag) {
  const Buckets K{1 << lb, keybits - lb};
  if (!bucket_scatter(a, buf, s, K, cnt, scan, flag)) return false;
  for (int32_t i = threadIdx.x; i < s; i += blockDim.x) {
    const uint64_t e = buf[i];
    out[bucket_rank(buf, 0, i, e, K, cnt)] = e;
  }
  __syncthreads();
  return true;
}

// buf in global memory (a and out anywhere): the ranking reads buf through
// windows staged in LDS (stage: cap entries), each window with a bucket's
// worth of margin on both sides, so every bucket it ranks lies inside.
__device__ __noinline__ bool bucket_sort_staged(uint64_t* a, uint64_t* buf, uint64_t* out, int32_t s,
                                                int keybits, int lb, lds_i32* cnt, lds_i32* scan,
                                                lds_i32* flag, lds_u64* stage, int32_t cap) {
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  const Buckets K{1 << lb, keybits - lb};
  if (!bucket_scatter(a, buf, s, K, cnt, scan, flag)) return false;
  const int32_t W = cap - 2 * kBucketMax;
  for (int32_t p0 = 0; p0 < s; p0 += W) {
    const int32_t p1 = p0 + W < s ? p0 + W : s;
    const int32_t q0 = p0 > kBucketMax ? p0 - kBucketMax : 0;
    const int32_t q1 = p1 + kBucketMax < s ? p1 + kBucketMax : s;
    for (int32_t i0 = q0 + tid; i0 < q1; i0 += kBucketBatch * nt) {
      uint64_t v[kBucketBatch];
#pragma unroll
      for (int r = 0; r < kBucketBatch; ++r) v[r] = i0 + r * nt < q1 ? buf[i0 + r * nt] : 0;
#pragma unroll
      for (int r = 0; r < kBucketBatch; ++r)
        if (i0 + r * nt < q1) stage[i0 + r * nt - q0] = v[r];
    }
    __syncthreads();
    for (int32_t i = p0 + tid; i < p1; i += nt) {
      const uint64_t e = stage[i - q0];
      out[bucket_rank(stage, q0, i, e, K, cnt)] = e;
    }
    __syncthreads();
  }
  return true;
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
