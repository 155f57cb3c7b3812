// Kernels around the trade kernel: per-round reset, the matching (hash keys,
// bucket sort, pairing), the dependency scan, the source list, the row-count
// check, the per-row sort that rebuilds the CSR, and upload validation.
#include "cb_block.hpp"
#include "cb_kernels.hpp"

namespace cbx {

__global__ void k_round_reset(int64_t n, int32_t nb, int32_t* inbox_cur, int32_t* out_cur,
                              int32_t* own_cur, int32_t* bcount, int32_t* bcur, int32_t* ctrl,
                              unsigned long long* stats, int32_t reset_stats) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = t0; i < n; i += stride) {
    inbox_cur[i] = 0;
    out_cur[i] = 0;
    own_cur[i] = 0;
  }
  for (int64_t i = t0; i < nb; i += stride) {
    bcount[i] = 0;
    bcur[i] = 0;
  }
  // Ready-queue slots need no reset: every pushed slot is cleared by its consumer.
  if (t0 < kCwCount && t0 != kCwErr && t0 != kCwAbort && t0 != kCwDbgBits && t0 != kCwDbgA &&
      t0 != kCwDbgB)
    ctrl[cw((int)t0)] = 0;
  if (t0 < kStatCount && reset_stats) stats[t0] = 0;
}

// ---------------------------------------------------------------- single trades
// One phase of uniform single trades: node-disjoint pairs, applied in step
// order as the trades 0..P-1 of a partial global trade (every other node
// sits out). pairs holds u0, v0, u1, v1, ...

__global__ void k_phase_pairs(const int32_t* pairs, int32_t P, int32_t* perm, int32_t* trade_of,
                              int32_t* tinfo, int32_t* dep) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < P; i += gridDim.x * blockDim.x) {
    const int32_t u = pairs[2 * i], v = pairs[2 * i + 1];
    perm[2 * i] = u;
    perm[2 * i + 1] = v;
    trade_of[u] = trade_of[v] = i;
    tinfo[u] = tinfo[v] = i;
    dep[i] = 0;
  }
}

// Edges between two nodes that sit out the phase stay where they are: row x
// of a node without a trade keeps its neighbours without a trade (the other
// edges are written by the trades).
__global__ void k_copy_idle_edges(int64_t n, const int64_t* rp, const int32_t* col, const int32_t* trade_of,
                                  int32_t* col_out, int32_t* out_cur, int32_t* ctrl) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += stride) {
    if (trade_of[x] != kUnmatched) continue;
    const int64_t b = rp[x], e = rp[x + 1];
    for (int64_t i = b; i < e; ++i) {
      const int32_t y = col[i];
      if (trade_of[y] != kUnmatched) continue;
      const int32_t p = atomicAdd(&out_cur[x], 1);
      if (p < e - b) col_out[b + p] = y; else atomic_or(&ctrl[cw(kCwErr)], kErrOut);
    }
  }
}

__global__ void k_set_draws(uint64_t* seed, uint32_t* round, uint32_t* draw_base, uint64_t s, uint32_t r,
                            uint32_t d) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    seed[0] = s;
    round[0] = r;
    draw_base[0] = d;
  }
}

// ---------------------------------------------------------------- chains

__global__ void k_set_chain(uint64_t* seed, uint32_t* round, int32_t c, uint64_t s, uint32_t r) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    seed[c] = s;
    round[c] = r;
  }
}

__global__ void k_advance_rounds(uint32_t* round, int32_t count, uint32_t by) {
  for (int32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < count; c += gridDim.x * blockDim.x)
    round[c] += by;
}

__global__ void k_single_chain(int64_t* node_base, int64_t* trade_base, int32_t* bucket_base,
                               int32_t* left_base, uint64_t* seed, uint32_t* round, uint32_t* draw_base,
                               int64_t n, int32_t nb, uint64_t s, uint32_t r) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    node_base[0] = 0;
    node_base[1] = n;
    trade_base[0] = 0;
    trade_base[1] = n / 2;
    bucket_base[0] = 0;
    bucket_base[1] = nb;
    left_base[0] = 0;
    left_base[1] = (int32_t)(n & 1);
    seed[0] = s;
    round[0] = r;
    draw_base[0] = 0;
  }
}

__global__ void k_fill_i32(int32_t* p, int64_t count, int32_t value) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = value;
}

// ---------------------------------------------------------------- matching
// Node v (local id lv in its chain c) has the key philox64(seed_c; lv,
// round_c, 0, TAG_M). Each chain's nodes are bucketed by the top bits of their
// keys into the chain's own buckets (in key order), each bucket is sorted by
// (key, id) in LDS, and the concatenation, chain by chain, is the pairing
// order: positions 2i and 2i+1 of chain c are its trade i.

__device__ __forceinline__ uint64_t chain_key(const Chains& ch, int32_t c, int64_t v) {
  return philox64(ch.seed[c], (uint32_t)(v - ch.node_base[c]), ch.round[c], 0u, kTagMatch);
}
__device__ __forceinline__ uint32_t node_bucket(const Chains& ch, int64_t v) {
  const int32_t c = chain_of_node(ch, v);
  const uint64_t key = chain_key(ch, c, v);
  const int32_t b0 = ch.bucket_base[c];
  const int32_t lg = 31 - __clz(ch.bucket_base[c + 1] - b0);   // buckets: a power of two
  return (uint32_t)b0 + (lg ? (uint32_t)(key >> (64 - lg)) : 0u);
}

__global__ void k_match_count(int64_t n, Chains ch, int32_t* bcount, const int32_t* ctrl) {
  if (ctrl[cw(kCwErr)]) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
    atomicAdd(&bcount[node_bucket(ch, v)], 1);
}

__global__ void k_match_scan(int32_t nb, const int32_t* bcount, int32_t* bstart,
                             const int32_t* ctrl) {
  __shared__ int32_t scratch[17];
  __shared__ int32_t carry;
  if (ctrl[cw(kCwErr)]) return;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int32_t base = 0; base < nb; base += blockDim.x) {
    const int32_t i = base + threadIdx.x;
    const int32_t v = i < nb ? bcount[i] : 0;
    int32_t total;
    const int32_t ex = block_excl_scan(v, scratch, &total);
    if (i < nb) bstart[i] = carry + ex;
    __syncthreads();
    if (threadIdx.x == 0) carry += total;
    __syncthreads();
  }
  if (threadIdx.x == 0) bstart[nb] = carry;
}

__global__ void k_match_scatter(int64_t n, Chains ch, const int32_t* bstart, int32_t* bcur,
                                int32_t* mtmp, const int32_t* ctrl) {
  if (ctrl[cw(kCwErr)]) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
    const uint32_t b = node_bucket(ch, v);
    mtmp[bstart[b] + atomicAdd(&bcur[b], 1)] = (int32_t)v;
  }
}

struct KeyedNode {
  uint64_t key;
  uint32_t id;
  __device__ bool operator<(const KeyedNode& o) const {
    return key < o.key || (key == o.key && id < o.id);
  }
};

// Node `id` of chain c at global sorted position p (chain c's positions start
// at node_base[c], because its buckets hold exactly its nodes).
__device__ __forceinline__ void write_pair_slot(const Chains& ch, int32_t c, int64_t p, int32_t id,
                                                int32_t* perm, int32_t* trade_of, int32_t* tinfo,
                                                const int32_t* giant_id, int32_t* dep) {
  const int64_t nb0 = ch.node_base[c];
  const int64_t pl = p - nb0;
  const int64_t nc = ch.node_base[c + 1] - nb0;
  if ((nc & 1) && pl == nc - 1) {
    perm[2 * ch.trade_base[ch.count] + ch.left_base[c]] = id;
    trade_of[id] = kUnmatched;
    tinfo[id] = kUnmatched;
    return;
  }
  const int32_t t = (int32_t)(ch.trade_base[c] + (pl >> 1));
  perm[2 * (int64_t)t + (pl & 1)] = id;
  trade_of[id] = t;
  tinfo[id] = giant_id[id] >= 0 ? (t | kGiantBit) : t;
  if (!(pl & 1)) dep[t] = 0;
}

__global__ void __launch_bounds__(kMatchBlock)
k_match_sort(Chains ch, int32_t nb, const int32_t* bstart, int32_t* mtmp, uint64_t* mkey,
             int32_t* perm, int32_t* trade_of, int32_t* tinfo, const int32_t* giant_id, int32_t* dep,
             int32_t* ctrl) {
  __shared__ KeyedNode buf[kMatchCap];
  if (ctrl[cw(kCwErr)]) return;
  for (int32_t b = blockIdx.x; b < nb; b += gridDim.x) {
    const int32_t c = ch.count == 1 ? 0 : chain_search(ch.bucket_base, ch.count, b);
    const int64_t s0 = bstart[b];
    const int64_t cnt = bstart[b + 1] - s0;
    if (cnt <= kMatchCap) {
      for (int64_t i = threadIdx.x; i < cnt; i += blockDim.x) {
        const int32_t id = mtmp[s0 + i];
        buf[i].key = chain_key(ch, c, id);
        buf[i].id = (uint32_t)id;
      }
      __syncthreads();
      block_bitonic_sort(buf, (uint32_t)cnt);
      for (int64_t i = threadIdx.x; i < cnt; i += blockDim.x)
        write_pair_slot(ch, c, s0 + i, (int32_t)buf[i].id, perm, trade_of, tinfo, giant_id, dep);
      __syncthreads();
    } else {
      // A bucket this large has probability far below 2^-500 for hashed
      // keys; it is still sorted exactly, in global memory.
      uint64_t* k = mkey + s0;
      int32_t* ids = mtmp + s0;
      for (int64_t i = threadIdx.x; i < cnt; i += blockDim.x) k[i] = chain_key(ch, c, ids[i]);
      __syncthreads();
      const uint64_t P = (uint64_t)next_pow2((uint32_t)cnt);
      for (uint64_t k2 = 2; k2 <= P; k2 <<= 1) {
        for (uint64_t d = k2 >> 1; d > 0; d >>= 1) {
          for (uint64_t p = threadIdx.x; p < P / 2; p += blockDim.x) {
            uint64_t i, j;
            if (d == (k2 >> 1)) {
              i = (p / d) * k2 + (p % d);
              j = i ^ (k2 - 1);
            } else {
              i = (p / d) * 2 * d + (p % d);
              j = i + d;
            }
            if (j < (uint64_t)cnt) {
              const bool swap = k[j] < k[i] || (k[j] == k[i] && ids[j] < ids[i]);
              if (swap) {
                const uint64_t tk = k[i]; k[i] = k[j]; k[j] = tk;
                const int32_t ti = ids[i]; ids[i] = ids[j]; ids[j] = ti;
              }
            }
          }
          __syncthreads();
        }
      }
      for (int64_t i = threadIdx.x; i < cnt; i += blockDim.x)
        write_pair_slot(ch, c, s0 + i, ids[i], perm, trade_of, tinfo, giant_id, dep);
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------- dep scan
// dep[k] += number of neighbours y of the nodes of trade k with
// trade_of[y] < k; col_t[e] = tinfo[col[e]] for every entry. Rows of giant
// nodes also put their neighbours of later trades (and the partner, and the
// node left out) into the node's bitmap. Work is split into equal chunks of
// CSR entries so hub rows do not serialise.

__device__ __forceinline__ int64_t row_of_entry(const int64_t* rp, int64_t lo, int64_t hi, int64_t e) {
  // largest r in [lo, hi] with rp[r] <= e
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (rp[mid] <= e) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ void __launch_bounds__(256)
k_depscan(int64_t n, int64_t nnz, const int64_t* rp, const int32_t* col,
          const int32_t* trade_of, const int32_t* tinfo, int32_t* col_t, int32_t* dep,
          GiantSets gs, const int32_t* ctrl) {
  __shared__ int64_t lrp[kScanChunk + 1];
  __shared__ int32_t cnt[kScanChunk];
  __shared__ int64_t bounds[2];
  if (ctrl[cw(kCwErr)]) return;
  const int64_t e0 = (int64_t)blockIdx.x * kScanChunk;
  if (e0 >= nnz) return;
  const int64_t e1 = e0 + kScanChunk < nnz ? e0 + kScanChunk : nnz;
  if (threadIdx.x == 0) bounds[0] = row_of_entry(rp, 0, n - 1, e0);
  if (threadIdx.x == 1) bounds[1] = row_of_entry(rp, 0, n - 1, e1 - 1);
  __syncthreads();
  const int64_t r0 = bounds[0], r1 = bounds[1];
  const int64_t nrows = r1 - r0 + 1;
  const bool local = nrows <= kScanChunk;
  if (local) {
    for (int64_t i = threadIdx.x; i <= nrows; i += blockDim.x) lrp[i] = rp[r0 + i];
    for (int64_t i = threadIdx.x; i < nrows; i += blockDim.x) cnt[i] = 0;
  }
  __syncthreads();
  for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    int64_t x;
    if (local) {
      int64_t lo = 0, hi = nrows - 1;
      while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (lrp[mid] <= e) lo = mid; else hi = mid - 1;
      }
      x = r0 + lo;
    } else {
      x = row_of_entry(rp, r0, r1, e);
    }
    const int32_t y = col[e];
    const int32_t ti = tinfo[y];
    col_t[e] = ti;
    const int32_t t = tinfo_trade(ti);
    const int32_t k = trade_of[x];
    if (k == kUnmatched) continue;
    if (t < k) {
      if (local) atomicAdd(&cnt[x - r0], 1);
      else atomicAdd(&dep[k], 1);
    } else {
      const int32_t gi = gs.giant_id[x];
      if (gi >= 0) giant_insert(gs, gi, y);
    }
  }
  __syncthreads();
  if (local) {
    for (int64_t i = threadIdx.x; i < nrows; i += blockDim.x)
      if (cnt[i]) atomicAdd(&dep[trade_of[r0 + i]], cnt[i]);
  }
}

// Debug check: every giant bitmap is empty before the dependency scan.
__global__ void k_check_giants_empty(int64_t total_sb, const int32_t* sc, int32_t* ctrl) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total_sb; i += stride)
    if (sc[i] != 0) {
      if (atomic_cas(&ctrl[cw(kCwDbgBits)], 0, kErrMatch)) {
        store_agent(&ctrl[cw(kCwDbgA)], (int32_t)i + 1);
        store_agent(&ctrl[cw(kCwDbgB)], sc[i]);
      }
      atomic_or(&ctrl[cw(kCwErr)], kErrMatch);
    }
}

// Per trade: its size deg u + deg v, and whether it is a source (no
// dependency). Small sources go to the source list of the wavefront workers;
// large ones straight into the workgroup queues.
// Sources of a round, in two passes around k_sources_scan. Pass 0 records
// every trade's size, queues the large sources, and counts the small ones
// per bucket of the trades that follow them in their chain (most first: a
// source with more later trades can head a longer dependency chain; the
// largest chain's count is the scale, chains being laid out largest first).
// Pass 1 places the small sources in the source list bucket by bucket, and
// they are handed out in that order. A single chain keeps trade order.
__device__ __forceinline__ int32_t source_bucket(const Chains& ch, int32_t k) {
  const int32_t c = chain_of_trade(ch, k);
  const int64_t lmax = ch.trade_base[1] - ch.trade_base[0];
  int64_t rem = ch.trade_base[c + 1] - k;   // this trade and the ones after it
  if (rem > lmax) rem = lmax;
  const int64_t q = lmax > 0 ? ((lmax - rem) * kSrcBuckets) / lmax : 0;
  return q < kSrcBuckets ? (int32_t)q : kSrcBuckets - 1;
}

__global__ void k_sources(int32_t L, const int32_t* dep, const int32_t* perm, const int64_t* rp,
                          int32_t small_max, int32_t* tsz, int32_t* src_list, int32_t* qb,
                          int32_t* ctrl, unsigned long long* stats, Chains ch, int32_t* sb, int pass) {
  if (ctrl[cw(kCwErr)]) return;
  int32_t* cnt = sb;                    // per bucket: small sources (pass 0)
  const int32_t* start = sb + kSrcBuckets;
  int32_t* cur = sb + 2 * kSrcBuckets;  // per bucket: placed so far (pass 1)
  const int32_t stride = gridDim.x * blockDim.x;
  // trip count is uniform across a wavefront (ballots below)
  for (int32_t base = blockIdx.x * blockDim.x; base < L; base += stride) {
    const int32_t k = base + threadIdx.x;
    int32_t s = 0;
    bool src = false;
    if (k < L) {
      if (pass == 0) {
        const int32_t u = perm[2 * k], v = perm[2 * k + 1];
        s = (int32_t)((rp[u + 1] - rp[u]) + (rp[v + 1] - rp[v]));
        tsz[k] = s;
      } else {
        s = tsz[k];
      }
      src = dep[k] == 0;
    }
    const bool big = src && s > small_max;
    const bool small = src && !big;
    const int32_t b = small ? source_bucket(ch, k) : -1;
    // one atomic per wavefront when its small sources share a bucket
    const uint64_t ms = ballot(small);
    const int32_t b0 = wave_bcast(b, ms ? __builtin_ctzll(ms) : 0);
    const bool uniform = ballot(small && b != b0) == 0;
    if (pass == 0) {
      const uint64_t mb = ballot(big);
      if ((ms | mb) == 0) continue;
      int32_t posb = 0;
      const int shard = (int)((uint32_t)base / 64u) % kQbShards;
      if (lane_id() == 0) {
        if (mb) posb = atomic_add(&ctrl[cw(kCwQbTail0 + shard)], popc64(mb));
        atomicAdd(&stats[kStatSources], (unsigned long long)popc64(ms | mb));
        if (ms && uniform) atomicAdd(&cnt[b0], popc64(ms));
      }
      if (small && !uniform) atomicAdd(&cnt[b], 1);
      posb = wave_bcast(posb, 0);
      if (big) qb[(int64_t)shard * L + posb + rank_below(mb)] = k;
    } else {
      if (ms == 0) continue;
      if (uniform) {
        int32_t pos = 0;
        if (lane_id() == 0) pos = start[b0] + atomicAdd(&cur[b0], popc64(ms));
        pos = wave_bcast(pos, 0);
        if (small) src_list[pos + rank_below(ms)] = k;
      } else if (small) {
        src_list[start[b] + atomicAdd(&cur[b], 1)] = k;
      }
    }
  }
}

// Exclusive scan of the per-bucket source counts (one workgroup of
// kSrcBuckets threads); the counts and cursors are left zero for the next
// round, the total goes to the source count.
__global__ void k_sources_scan(int32_t* sb, int32_t* ctrl) {
  if (ctrl[cw(kCwErr)]) return;
  __shared__ int32_t scan[kSrcBuckets / 64 + 1];
  const int t = threadIdx.x;
  const int32_t c = sb[t];
  int32_t tot;
  const int32_t at = block_excl_scan(c, scan, &tot);
  sb[kSrcBuckets + t] = at;
  sb[t] = 0;
  sb[2 * kSrcBuckets + t] = 0;
  if (t == 0) store_agent(&ctrl[cw(kCwSrcCount)], tot);
}

// Row offset, degree and trade information of every node side by side, so
// that a write in the trade kernel finds all three with one 16-byte load
// (offsets fit 32 bits: fewer than 2^31 entries). Rebuilt before every trade
// kernel, after the round's trade information is final.
__global__ void k_node_info(int64_t n, const int64_t* rp, const int32_t* tinfo, uint4* ninfo) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const int64_t b = rp[i];
    ninfo[i] = make_uint4((uint32_t)b, (uint32_t)(rp[i + 1] - b), (uint32_t)tinfo[i], 0u);
  }
}

// Every row received exactly its degree: entries from its front plus the
// own-row entries a workgroup trade wrote from its back.
__global__ void k_check_rows(int64_t n, const int64_t* rp, const int32_t* out_cur,
                             const int32_t* own_cur, int32_t* ctrl) {
  if (ctrl[cw(kCwErr)]) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += stride)
    if ((int64_t)out_cur[x] + own_cur[x] != rp[x + 1] - rp[x]) atomic_or(&ctrl[cw(kCwErr)], kErrRows);
}

// ---------------------------------------------------------------- rebuild
// Row x of src (its entries in any order) is written ascending to row x of
// dst. Size classes are fixed at upload because degrees never change. With a
// NextScan the rebuild also does the next round's dependency scan of every
// entry it writes (the same counts, trade information and bitmap seeds as
// k_depscan), so that scan does not read the adjacency again.

struct RowScan {
  int32_t k = kUnmatched;   // next round's trade of the row's node
  int32_t gi = -1;          // its giant index
};
__device__ __forceinline__ RowScan row_scan(const NextScan& N, int32_t x) {
  RowScan r;
  if (N.tinfo) {
    r.k = N.trade_of[x];
    r.gi = N.gs.bm ? N.gs.giant_id[x] : -1;
  }
  return r;
}
// Entry e (neighbour y) of a row: 1 if it counts towards the row's trade's
// dependencies.
__device__ __forceinline__ int32_t scan_entry(const NextScan& N, const RowScan& r, int64_t e, int32_t y) {
  const int32_t ti = N.tinfo[y];
  N.col_t[e] = ti;
  if (r.k == kUnmatched) return 0;
  if (tinfo_trade(ti) < r.k) return 1;
  if (r.gi >= 0) giant_insert(N.gs, r.gi, y);
  return 0;
}
// Wave-level sum of the counts, added once per wavefront (every lane active).
__device__ __forceinline__ void add_dep(const NextScan& N, const RowScan& r, int32_t cnt) {
  const int32_t tot = wave_sum(cnt);
  if (lane_id() == 0 && tot && r.k != kUnmatched) atomicAdd(&N.dep[r.k], tot);
}

__global__ void __launch_bounds__(256)
k_segsort_small(const int32_t* rows, int64_t nrows, const int64_t* rp, const int32_t* src,
                int32_t* dst, NextScan N, const int32_t* ctrl) {
  if (ctrl[cw(kCwErr)]) return;
  const int l = lane_id();
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t r = wid; r < nrows; r += nwaves) {
    const int32_t x = rows[r];
    const int64_t b = rp[x];
    const int32_t d = (int32_t)(rp[x + 1] - b);
    int32_t v = l < d ? src[b + l] : 0x7fffffff;
    // bitonic network over the 64 lanes (padding sorts to the end)
#pragma unroll
    for (int k2 = 2; k2 <= kWave; k2 <<= 1) {
#pragma unroll
      for (int j = k2 >> 1; j > 0; j >>= 1) {
        const int32_t o = __shfl_xor(v, j, kWave);
        const bool up = (l & k2) == 0;
        const bool lower = (l & j) == 0;
        v = (lower == up) ? min(v, o) : max(v, o);
      }
    }
    if (l < d) dst[b + l] = v;
    if (N.tinfo) {
      const RowScan rs = row_scan(N, x);
      add_dep(N, rs, l < d ? scan_entry(N, rs, b + l, v) : 0);
    }
  }
}

// Rows of 65..4096 entries, one workgroup per row. The ids of a row are
// distinct, so a bucket sort needs no stable pass: a counting scatter by the
// top bits of the id into LDS (about 16 per bucket), then each id's place is
// the number of smaller ids in its bucket. A row whose ids crowd one bucket
// (more than kSegBucketMax) is sorted by the bitonic network instead.
constexpr int kSegMidPer = kSegMidMax / 256;   // ids per thread
constexpr int32_t kSegBucketMax = 256;
__global__ void __launch_bounds__(256)
k_segsort_mid(const int32_t* rows, int64_t nrows, const int64_t* rp, const int32_t* src,
              int32_t* dst, int keybits, NextScan N, const int32_t* ctrl) {
  __shared__ int32_t buf[kSegMidMax];
  __shared__ int32_t cnt[kSegMidMax / 16];
  __shared__ int32_t scan[256 / 64 + 1];
  __shared__ int32_t full;
  if (ctrl[cw(kCwErr)]) return;
  const int tid = threadIdx.x;
  for (int64_t r = blockIdx.x; r < nrows; r += gridDim.x) {
    const int32_t x = rows[r];
    const int64_t b = rp[x];
    const int32_t d = (int32_t)(rp[x + 1] - b);
    int lb = 0;
    while ((16 << lb) < d && lb < keybits) ++lb;   // at most 8: d <= 4096
    const int32_t nb = 1 << lb;
    const int sh = keybits - lb;
    auto bucket = [&](int32_t v) -> int32_t {
      const uint32_t q = (uint32_t)v >> sh;
      return q < (uint32_t)nb ? (int32_t)q : nb - 1;
    };
    int32_t v[kSegMidPer];
#pragma unroll
    for (int q = 0; q < kSegMidPer; ++q) {
      const int32_t i = tid + q * 256;
      v[q] = i < d ? src[b + i] : 0;
    }
    for (int32_t q = tid; q < nb; q += 256) cnt[q] = 0;
    if (tid == 0) full = 0;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kSegMidPer; ++q)
      if (tid + q * 256 < d) atomicAdd(&cnt[bucket(v[q])], 1);
    __syncthreads();
    const int32_t c = tid < nb ? cnt[tid] : 0;   // nb <= 256: one bucket per thread
    if (c > kSegBucketMax) full = 1;
    int32_t tot;
    const int32_t start = block_excl_scan(c, scan, &tot);   // its barriers publish `full`
    if (full) {
#pragma unroll
      for (int q = 0; q < kSegMidPer; ++q)
        if (tid + q * 256 < d) buf[tid + q * 256] = v[q];
      __syncthreads();
      block_bitonic_sort(buf, (uint32_t)d);
      for (int32_t i = tid; i < d; i += blockDim.x) dst[b + i] = buf[i];
      if (N.tinfo) {
        const RowScan rs = row_scan(N, x);
        int32_t cnt = 0;
        for (int32_t i = tid; i < d; i += blockDim.x) cnt += scan_entry(N, rs, b + i, buf[i]);
        add_dep(N, rs, cnt);
      }
      __syncthreads();
      continue;
    }
    if (tid < nb) cnt[tid] = start;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kSegMidPer; ++q)
      if (tid + q * 256 < d) buf[atomicAdd(&cnt[bucket(v[q])], 1)] = v[q];
    __syncthreads();
    // cnt[q] is now the end of bucket q and the start of bucket q + 1
    const RowScan rs = row_scan(N, x);
    int32_t dcnt = 0;
    for (int32_t i = tid; i < d; i += blockDim.x) {
      const int32_t e = buf[i];
      const int32_t q = bucket(e);
      const int32_t lo = q ? cnt[q - 1] : 0;
      const int32_t hi = cnt[q];
      int32_t rk = lo;
      for (int32_t j = lo; j < hi; ++j) {
        const int32_t y = buf[j];
        rk += (y < e || (y == e && j < i)) ? 1 : 0;
      }
      dst[b + rk] = e;
      if (N.tinfo) dcnt += scan_entry(N, rs, b + rk, e);
    }
    if (N.tinfo) add_dep(N, rs, dcnt);
    __syncthreads();
  }
}

// Rows of kSegMidMax < d <= kSegWideMax entries (from the list of big rows;
// larger ones are left to k_segsort_huge), one per workgroup of
// kSegWideThreads, sorted in LDS as k_segsort_mid does it: ids bucketed by
// their top bits (about 16 per bucket), each then placed by its rank within
// its bucket; a bucket of more than kSegBucketMax ids (ids bunched together)
// sends the row to the bitonic network. The row's scan for the next round is
// done by k_scan_big_rows.
__global__ void __launch_bounds__(kSegWideThreads)
k_segsort_wide(const int32_t* rows, int64_t nrows, const int64_t* rp, const int32_t* src, int32_t* dst,
               int keybits, const int32_t* ctrl) {
  constexpr int kPer = kSegWideMax / kSegWideThreads;
  __shared__ int32_t buf[kSegWideMax];
  __shared__ int32_t cnt[kSegWideMax / 16];
  __shared__ int32_t scan[kSegWideThreads / 64 + 1];
  __shared__ int32_t full;
  if (ctrl[cw(kCwErr)]) return;
  const int tid = threadIdx.x;
  for (int64_t r = blockIdx.x; r < nrows; r += gridDim.x) {
    const int32_t x = rows[r];
    const int64_t b = rp[x];
    const int32_t d = (int32_t)(rp[x + 1] - b);
    if (d > kSegWideMax) continue;   // uniform: left to k_segsort_huge
    int lb = 0;
    while ((16 << lb) < d && lb < keybits) ++lb;
    const int32_t nb = 1 << lb;   // at most kSegWideMax / 16
    const int sh = keybits - lb;
    auto bucket = [&](int32_t v) -> int32_t {
      const uint32_t q = (uint32_t)v >> sh;
      return q < (uint32_t)nb ? (int32_t)q : nb - 1;
    };
    int32_t v[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int32_t i = tid + q * kSegWideThreads;
      v[q] = i < d ? src[b + i] : 0;
    }
    for (int32_t q = tid; q < nb; q += kSegWideThreads) cnt[q] = 0;
    if (tid == 0) full = 0;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPer; ++q)
      if (tid + q * kSegWideThreads < d) atomicAdd(&cnt[bucket(v[q])], 1);
    __syncthreads();
    // two buckets per thread (nb <= 2 * kSegWideThreads)
    const int32_t c0 = 2 * tid < nb ? cnt[2 * tid] : 0;
    const int32_t c1 = 2 * tid + 1 < nb ? cnt[2 * tid + 1] : 0;
    if (c0 > kSegBucketMax || c1 > kSegBucketMax) full = 1;
    int32_t tot;
    const int32_t start = block_excl_scan(c0 + c1, scan, &tot);   // its barriers publish `full`
    if (full) {
#pragma unroll
      for (int q = 0; q < kPer; ++q)
        if (tid + q * kSegWideThreads < d) buf[tid + q * kSegWideThreads] = v[q];
      __syncthreads();
      block_bitonic_sort(buf, (uint32_t)d);
      for (int32_t i = tid; i < d; i += kSegWideThreads) dst[b + i] = buf[i];
      __syncthreads();
      continue;
    }
    if (2 * tid < nb) cnt[2 * tid] = start;
    if (2 * tid + 1 < nb) cnt[2 * tid + 1] = start + c0;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPer; ++q)
      if (tid + q * kSegWideThreads < d) buf[atomicAdd(&cnt[bucket(v[q])], 1)] = v[q];
    __syncthreads();
    // cnt[q] is now the end of bucket q and the start of bucket q + 1
    for (int32_t i = tid; i < d; i += kSegWideThreads) {
      const int32_t e = buf[i];
      const int32_t q = bucket(e);
      const int32_t lo = q ? cnt[q - 1] : 0;
      const int32_t hi = cnt[q];
      int32_t rk = lo;
      for (int32_t j = lo; j < hi; ++j) {
        const int32_t y = buf[j];
        rk += (y < e || (y == e && j < i)) ? 1 : 0;
      }
      dst[b + rk] = e;
    }
    __syncthreads();
  }
}

// Sort dst[0, d) in place (d <= kSegWideMax) on the whole workgroup of
// kSegWideThreads, by the low `lo_bits` bits of its ids (the higher ones are
// equal within the run): the bucket-and-rank sort of k_segsort_wide, or the
// bitonic network when a bucket is too full.
__device__ __forceinline__ void lds_sort_run(int32_t* dst, int32_t d, int lo_bits, int32_t* buf, int32_t* cnt,
                                             int32_t* scan, int32_t* full) {
  constexpr int kPer = kSegWideMax / kSegWideThreads;
  const int tid = threadIdx.x;
  int lb = 0;
  while ((16 << lb) < d && lb < lo_bits) ++lb;
  const int32_t nb = 1 << lb;
  const int sh = lo_bits - lb;
  auto bucket = [&](int32_t v) -> int32_t { return (int32_t)(((uint32_t)v >> sh) & (uint32_t)(nb - 1)); };
  int32_t v[kPer];
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int32_t i = tid + q * kSegWideThreads;
    v[q] = i < d ? dst[i] : 0;
  }
  for (int32_t q = tid; q < nb; q += kSegWideThreads) cnt[q] = 0;
  if (tid == 0) *full = 0;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kPer; ++q)
    if (tid + q * kSegWideThreads < d) atomicAdd(&cnt[bucket(v[q])], 1);
  __syncthreads();
  const int32_t c0 = 2 * tid < nb ? cnt[2 * tid] : 0;
  const int32_t c1 = 2 * tid + 1 < nb ? cnt[2 * tid + 1] : 0;
  if (c0 > kSegBucketMax || c1 > kSegBucketMax) *full = 1;
  int32_t tot;
  const int32_t start = block_excl_scan(c0 + c1, scan, &tot);   // its barriers publish `full`
  if (*full) {
#pragma unroll
    for (int q = 0; q < kPer; ++q)
      if (tid + q * kSegWideThreads < d) buf[tid + q * kSegWideThreads] = v[q];
    __syncthreads();
    block_bitonic_sort(buf, (uint32_t)d);
    for (int32_t i = tid; i < d; i += kSegWideThreads) dst[i] = buf[i];
    __syncthreads();
    return;
  }
  if (2 * tid < nb) cnt[2 * tid] = start;
  if (2 * tid + 1 < nb) cnt[2 * tid + 1] = start + c0;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kPer; ++q)
    if (tid + q * kSegWideThreads < d) buf[atomicAdd(&cnt[bucket(v[q])], 1)] = v[q];
  __syncthreads();
  for (int32_t i = tid; i < d; i += kSegWideThreads) {
    const int32_t e = buf[i];
    const int32_t q = bucket(e);
    const int32_t lo = q ? cnt[q - 1] : 0;
    const int32_t hi = cnt[q];
    int32_t rk = lo;
    for (int32_t j = lo; j < hi; ++j) {
      const int32_t y = buf[j];
      rk += (y < e || (y == e && j < i)) ? 1 : 0;
    }
    dst[rk] = e;
  }
  __syncthreads();
}

// Rows of more than kSegWideMax entries, one per workgroup of
// kSegWideThreads: the row is split by the top bits of its ids into runs of
// about kSegWideMax / 2 entries (a count pass and a scatter pass into dst,
// with the runs' cursors in LDS), then each run is sorted in place by
// lds_sort_run (a run above kSegWideMax, ids crowded into one range, by the
// bitonic network in global memory).
__global__ void __launch_bounds__(kSegWideThreads)
k_segsort_huge(const int32_t* rows, int64_t nrows, const int64_t* rp, const int32_t* src, int32_t* dst,
               int keybits, const int32_t* ctrl) {
  constexpr int kPer = kSegWideMax / kSegWideThreads;
  constexpr int32_t kRuns = kSegWideMax / 16;
  __shared__ int32_t buf[kSegWideMax];
  __shared__ int32_t cnt[kSegWideMax / 16];
  __shared__ int32_t run_start[kRuns + 1];
  __shared__ int32_t scan[kSegWideThreads / 64 + 1];
  __shared__ int32_t full;
  if (ctrl[cw(kCwErr)]) return;
  const int tid = threadIdx.x;
  for (int64_t r = blockIdx.x; r < nrows; r += gridDim.x) {
    const int32_t x = rows[r];
    const int64_t b = rp[x];
    const int64_t d = rp[x + 1] - b;
    if (d <= kSegWideMax) continue;   // uniform: sorted by k_segsort_wide
    int lp = 0;
    while ((d >> lp) > kSegWideMax / 2 && lp < keybits && (2 << lp) <= kRuns) ++lp;
    const int32_t np = 1 << lp;
    const int shp = keybits - lp;
    auto part = [&](int32_t v) -> int32_t {
      const uint32_t q = (uint32_t)v >> shp;
      return q < (uint32_t)np ? (int32_t)q : np - 1;
    };
    for (int32_t q = tid; q < np; q += kSegWideThreads) cnt[q] = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < d; c0 += kSegWideMax) {
#pragma unroll
      for (int q = 0; q < kPer; ++q) {
        const int64_t i = c0 + tid + q * kSegWideThreads;
        if (i < d) atomicAdd(&cnt[part(src[b + i])], 1);
      }
    }
    __syncthreads();
    const int32_t c0 = 2 * tid < np ? cnt[2 * tid] : 0;
    const int32_t c1 = 2 * tid + 1 < np ? cnt[2 * tid + 1] : 0;
    int32_t tot;
    const int32_t start = block_excl_scan(c0 + c1, scan, &tot);
    if (2 * tid < np) { cnt[2 * tid] = start; run_start[2 * tid] = start; }
    if (2 * tid + 1 < np) { cnt[2 * tid + 1] = start + c0; run_start[2 * tid + 1] = start + c0; }
    if (tid == 0) run_start[np] = (int32_t)d;
    __syncthreads();
    for (int64_t c = 0; c < d; c += kSegWideMax) {
#pragma unroll
      for (int q = 0; q < kPer; ++q) {
        const int64_t i = c + tid + q * kSegWideThreads;
        if (i < d) {
          const int32_t v = src[b + i];
          dst[b + atomicAdd(&cnt[part(v)], 1)] = v;
        }
      }
    }
    __syncthreads();   // the runs in dst are complete and visible to the workgroup
    for (int32_t p = 0; p < np; ++p) {
      const int32_t lo = run_start[p], len = run_start[p + 1] - lo;
      if (len <= 1) continue;
      if (len <= kSegWideMax) {
        lds_sort_run(dst + b + lo, len, shp, buf, cnt, scan, &full);
      } else {
        block_bitonic_sort(dst + b + lo, (uint32_t)len);
      }
    }
    __syncthreads();
  }
}


// Rows of each rebuild size class, listed once at upload (degrees never
// change): rows of 1..64 entries from rows[0], of 65..4096 from rows[base[1]],
// larger ones from rows[base[2]]; cur[0..3) counts the rows placed so far.
__global__ void k_classify_rows(int64_t n, const int64_t* rp, int32_t* rows, int64_t base1,
                                int64_t base2, unsigned long long* cur) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // trip count is uniform across a wavefront (ballots below)
  for (int64_t b0 = (int64_t)blockIdx.x * blockDim.x; b0 < n; b0 += stride) {
    const int64_t x = b0 + threadIdx.x;
    int cls = -1;
    if (x < n) {
      const int64_t d = rp[x + 1] - rp[x];
      cls = d == 0 ? -1 : (d <= kSegSmallMax ? 0 : (d <= kSegMidMax ? 1 : 2));
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const uint64_t m = ballot(cls == c);
      if (!m) continue;
      unsigned long long pos = 0;
      if (lane_id() == 0) pos = atomicAdd(&cur[c], (unsigned long long)popc64(m));
      pos = __shfl(pos, 0, kWave);
      if (cls == c) rows[(c == 0 ? 0 : (c == 1 ? base1 : base2)) + (int64_t)pos + rank_below(m)] = (int32_t)x;
    }
  }
}

// dst[i] = src[i] + delta (node ids of one chain moved to another id range).
__global__ void k_copy_shift(int32_t* dst, const int32_t* src, int64_t count, int32_t delta) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
    dst[i] = src[i] + delta;
}

// Offsets of the big rows' entries laid end to end: boff[i] = sum of the
// sizes of rows[0..i) (one workgroup; the big rows are few).
__global__ void k_big_offsets(const int32_t* rows, int64_t nrows, const int64_t* rp, int64_t* boff) {
  __shared__ int32_t scratch[17];
  __shared__ int64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < nrows; base += blockDim.x) {
    const int64_t i = base + threadIdx.x;
    const int32_t d = i < nrows ? (int32_t)(rp[rows[i] + 1] - rp[rows[i]]) : 0;
    int32_t total;
    const int32_t ex = block_excl_scan(d, scratch, &total);
    if (i < nrows) boff[i] = carry + ex;
    __syncthreads();
    if (threadIdx.x == 0) carry += total;
    __syncthreads();
  }
  if (threadIdx.x == 0) boff[nrows] = carry;
}

// The next round's scan of the big rows (more than kSegMidMax entries),
// done after their rebuild with their entries split evenly over workgroups
// (a hub row would hold up one workgroup for long otherwise). A chunk of
// kScanChunk entries meets at most two big rows.
__global__ void __launch_bounds__(256)
k_scan_big_rows(const int32_t* rows, int64_t nrows, const int64_t* boff, const int64_t* rp,
                const int32_t* col, NextScan N, const int32_t* ctrl) {
  if (ctrl[cw(kCwErr)]) return;
  const int64_t total = boff[nrows];
  const int64_t v0 = (int64_t)blockIdx.x * kScanChunk;
  if (v0 >= total) return;
  const int64_t v1 = v0 + kScanChunk < total ? v0 + kScanChunk : total;
  const int64_t i0 = row_of_entry(boff, 0, nrows - 1, v0);
  const int64_t i1 = row_of_entry(boff, i0, nrows - 1, v1 - 1);
  const int32_t x0 = rows[i0], x1 = rows[i1];
  const RowScan r0 = row_scan(N, x0), r1 = row_scan(N, x1);
  const int64_t split = boff[i0 + 1];
  const int64_t e0 = rp[x0] - boff[i0], e1 = rp[x1] - boff[i1];
  int32_t c0 = 0, c1 = 0;
  for (int64_t v = v0 + threadIdx.x; v < v1; v += blockDim.x) {
    if (v < split) {
      const int64_t e = e0 + v;
      c0 += scan_entry(N, r0, e, col[e]);
    } else {
      const int64_t e = e1 + v;
      c1 += scan_entry(N, r1, e, col[e]);
    }
  }
  add_dep(N, r0, c0);
  add_dep(N, r1, c1);
}

// ---------------------------------------------------------------- validate
// Every entry: id in range, not the row's own id, strictly above its left
// neighbour in the row, and present in the neighbour's row (symmetry).

__global__ void __launch_bounds__(256)
k_validate(int64_t n, int64_t nnz, const int64_t* rp, const int32_t* col, int32_t* ctrl) {
  __shared__ int64_t bounds[2];
  const int64_t e0 = (int64_t)blockIdx.x * kScanChunk;
  if (e0 >= nnz) return;
  const int64_t e1 = e0 + kScanChunk < nnz ? e0 + kScanChunk : nnz;
  if (threadIdx.x == 0) bounds[0] = row_of_entry(rp, 0, n - 1, e0);
  if (threadIdx.x == 1) bounds[1] = row_of_entry(rp, 0, n - 1, e1 - 1);
  __syncthreads();
  bool bad = false;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const int64_t x = row_of_entry(rp, bounds[0], bounds[1], e);
    const int32_t y = col[e];
    if (y < 0 || (int64_t)y >= n || (int64_t)y == x) { bad = true; continue; }
    if (e > rp[x] && col[e - 1] >= y) bad = true;
    int64_t lo = rp[y], hi = rp[y + 1];
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if ((int64_t)col[mid] < x) lo = mid + 1; else hi = mid;
    }
    if (lo >= rp[y + 1] || (int64_t)col[lo] != x) bad = true;
  }
  if (bad) atomic_or(&ctrl[cw(kCwErr)], kErrInvalid);
}

}  // namespace cbx
