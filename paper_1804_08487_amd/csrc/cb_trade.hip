// Persistent trade kernel: runs every trade of one global trade once all
// edges it shares with earlier trades have been handed to it.
//
// Semantics (Def. "Simple Undirected Trade", Def. "Undirected Global Trade"):
// trade k pairs u = perm[2k] and v = perm[2k+1]; at its turn it sees
//   A_u = {x in the round-start row of u : trade_of[x] >= k}   ("fresh": later
//         nodes, the partner, the node left out - no earlier trade touched
//         these edges)
//       u {p delivered to u's inbox by earlier trades}        (edges to
//         earlier nodes, as the earlier trades left them)
// and the same for v. It keeps C = shared neighbours and the u-v edge, and
// re-splits D = the disjoint neighbours (ascending) by the seeded partial
// Durstenfeld shuffle. Each resulting edge {p, x}:
//   - x in a later trade t: p goes to x's inbox and dep[t] drops by one
//     (IM-CB's push to the endpoint traded next);
//   - otherwise (x earlier, the partner, or left out) the edge is final and
//     is written to both rows of col_out (the partner edge once per side).
// dep[t] starts at the number of edges between trade t's pair and earlier
// pairs at round start, a count no trade changes (a trade only moves an edge
// between its own two nodes), so it reaches zero exactly when trade t has
// every input; the worker whose decrement reaches zero picks it up
// (EM-PGCB's "the processor adding the last missing message runs the
// trade").
//
// Workers: workgroups [0, nbig) run large trades with the whole workgroup
// (in LDS up to kBigCap entries, else in a global scratch slot; lists are
// bucket-sorted, giant nodes' sets read from bitmaps); every other workgroup
// holds eight wavefronts that each run small trades (deg u + deg v <=
// small_max) in LDS.
#include "cb_block.hpp"
#include "cb_kernels.hpp"

namespace cbx {

// Entry = ((node << 1 | side) << 32) | tag; side 0 = u's list, 1 = v's.
// tag 0: final when emitted (earlier node or the node left out),
// tag 1: the partner, tag t + 2: node of the later trade t, with bit 31 set
// when that node keeps its arrivals in a bitmap.
constexpr uint32_t kTagEmit = 0u;
constexpr uint32_t kTagPartner = 1u;
constexpr uint32_t kTagGiant = 0x80000000u;
// Tag of a giant node's member whose trade is looked up only when the edge
// is written (trade indices stay below 2^30, so no real tag takes this value).
constexpr uint32_t kTagUnknown = 0x7FFFFFFFu;

__device__ __forceinline__ uint64_t make_entry(int32_t x, int side, uint32_t tag) {
  return ((uint64_t)(((uint32_t)x << 1) | (uint32_t)side) << 32) | tag;
}
__device__ __forceinline__ int32_t ent_node(uint64_t e) { return (int32_t)(e >> 33); }
__device__ __forceinline__ int ent_side(uint64_t e) { return (int)((e >> 32) & 1u); }
__device__ __forceinline__ uint32_t ent_tag(uint64_t e) { return (uint32_t)e; }
// Tag of neighbour information ti (a tinfo value) seen from trade k.
__device__ __forceinline__ uint32_t tag_of(int32_t ti, int32_t k) {
  const int32_t t = tinfo_trade(ti);
  if (t == k) return kTagPartner;
  if (t == kUnmatched || t < k) return kTagEmit;
  return ((uint32_t)t + 2u) | (tinfo_giant(ti) ? kTagGiant : 0u);
}
__device__ __forceinline__ int32_t tag_trade(uint32_t tag) { return (int32_t)((tag & ~kTagGiant) - 2u); }

struct WaveLds {
  uint64_t E[kSmallCap];
  int32_t D[kSmallCap];
  uint16_t R[kSmallCap / 2];   // swap partners of the split, one per step
  int32_t stack[kStackCap];
};

constexpr int kBucketLdsBits = 10;    // bucket sort of a trade in LDS: counters beside the tile
constexpr int kBucketTileBits = 13;   // ... of a trade in the slot: counters in the (unused) LDS tile
struct BigLds {
  union {
    struct {
      uint64_t E[kBigCap];
      int32_t D[kBigCap];
    } tile;          // trades that fit in LDS
    RadixLds R;      // scratch of the global-memory sort for larger trades
  } u;
  int32_t scan[kWavesPerBlock + 1];
  int32_t next;
  int32_t cnt[4];
  int32_t flag;        // workgroup-wide decision
  uint64_t tick[1];    // trace: end of a giant's bit pass
  int32_t base[2];
  int32_t ndone;
  int32_t bflag;                   // bucket sort: a bucket is too full
  int32_t bkt[1 << kBucketLdsBits];   // bucket sort counters of trades held in LDS
  // giant extraction: output offset and members per superblock; the split
  // reuses both as one buffer of 2 * kTradeBlock swap partners
  int32_t sboff[kTradeBlock];
  int32_t sbcnt[kTradeBlock];
};
static_assert(offsetof(BigLds, sbcnt) == offsetof(BigLds, sboff) + kTradeBlock * sizeof(int32_t),
              "split buffer spans sboff and sbcnt");

// Ready small trades shared by the wavefronts of one workgroup (slot -1:
// empty): a wavefront that makes more trades ready than it keeps leaves the
// rest here, where the workgroup's idle wavefronts find them at LDS cost.
constexpr int kPoolSlots = kWave;
struct SmallLds {
  WaveLds wave[kWavesPerBlock];
  int32_t pool[kPoolSlots];
};

union TradeLds {
  SmallLds small;
  BigLds big;
};

__device__ __forceinline__ void raise_error(const TradeArgs& A, int32_t bits, int32_t trade = -1,
                                            int32_t detail = 0) {
  if (atomic_cas(&A.ctrl[cw(kCwDbgBits)], 0, bits)) {
    store_agent(&A.ctrl[cw(kCwDbgA)], trade + 1);
    store_agent(&A.ctrl[cw(kCwDbgB)], detail);
  }
  atomic_or(&A.ctrl[cw(kCwErr)], bits);
  store_agent(&A.ctrl[cw(kCwAbort)], 1);
}

// Split of the ascending disjoint set D (N indices into the entry array) in
// place; u receives D[0..a), v receives D[a..N). Partial Durstenfeld shuffle
// of the smaller side (Sec. 4, trade procedure): with T = min(a, N - a)
// steps t = 0..T-1 at position j(t) = t (a <= N - a) or N - 1 - t (else),
// swapping D[j] with D[partner(t)], partner drawn from
// philox64(seed; k, round, j, split tag). The draws do not depend on the
// swaps, so they are computed in parallel first; only the swaps run in
// order, on one lane.
__device__ __forceinline__ int32_t split_steps(int32_t N, int32_t a) { return a <= N - a ? a : N - a; }

// Seed, round and draw index of trade k: those of its chain, with the trade's
// index within the chain (plus the chain's draw offset).
struct DrawKey {
  uint64_t seed;
  uint32_t round;
  int32_t idx;
};
__device__ __forceinline__ DrawKey draw_key(const TradeArgs& A, int32_t k) {
  const int32_t c = chain_of_trade(A.ch, k);
  DrawKey d;
  d.seed = A.ch.seed[c];
  d.round = A.ch.round[c];
  d.idx = (int32_t)((uint32_t)(k - A.ch.trade_base[c]) + A.ch.draw_base[c]);
  return d;
}

__device__ __forceinline__ int32_t split_partner(int32_t N, int32_t a, int32_t t, uint64_t seed,
                                                 uint32_t round, int32_t k) {
  const bool fwd = a <= N - a;
  const int32_t j = fwd ? t : N - 1 - t;
  const uint64_t x = philox64(seed, (uint32_t)k, round, (uint32_t)j, kTagSplit);
  return fwd ? j + (int32_t)bounded(x, (uint64_t)(N - j)) : (int32_t)bounded(x, (uint64_t)(j + 1));
}

// Apply steps t0 .. t0+tc-1 given their partners R[0..tc) (single lane).
template <typename Idx, typename RT>
__device__ __forceinline__ void split_apply(Idx* D, int32_t N, int32_t a, int32_t t0, int32_t tc,
                                            const RT* R) {
  const bool fwd = a <= N - a;
  int32_t t = 0;
  for (; t + 4 <= tc; t += 4) {
    int32_t r[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) r[q] = (int32_t)R[t + q];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int32_t j = fwd ? t0 + t + q : N - 1 - (t0 + t + q);
      const Idx x = D[j], y = D[r[q]];
      D[j] = y;
      D[r[q]] = x;
    }
  }
  for (; t < tc; ++t) {
    const int32_t j = fwd ? t0 + t : N - 1 - (t0 + t);
    const int32_t rr = (int32_t)R[t];
    const Idx x = D[j], y = D[rr];
    D[j] = y;
    D[rr] = x;
  }
}

// One wavefront, N <= kSmallCap (so at most kSmallCap / 2 steps).
__device__ __forceinline__ void wave_split(int32_t* D, int32_t N, int32_t a, uint64_t seed, uint32_t round,
                           int32_t k, uint16_t* R) {
  const int32_t T = split_steps(N, a);
  for (int32_t t = lane_id(); t < T; t += kWave) R[t] = (uint16_t)split_partner(N, a, t, seed, round, k);
  wave_sync();
  if (lane_id() == 0) split_apply<int32_t, uint16_t>(D, N, a, 0, T, R);
  wave_sync();
}

// Whole workgroup; the partners go through R (cap entries) in chunks.
__device__ __forceinline__ void block_split(int32_t* D, int32_t N, int32_t a, uint64_t seed, uint32_t round,
                            int32_t k, int32_t* R, int32_t cap) {
  const int32_t T = split_steps(N, a);
  for (int32_t t0 = 0; t0 < T; t0 += cap) {
    const int32_t tc = T - t0 < cap ? T - t0 : cap;
    for (int32_t i = threadIdx.x; i < tc; i += blockDim.x) R[i] = split_partner(N, a, t0 + i, seed, round, k);
    __syncthreads();
    if (threadIdx.x == 0) split_apply<int32_t, int32_t>(D, N, a, t0, tc, R);
    __syncthreads();
  }
}

// The same split for a D in global memory, through LDS: the positions its
// steps touch go into a hash table (with the number of steps touching each),
// their entries are gathered, swapped there and written back. A step whose two
// positions no other step touches commutes with all others, so those steps
// swap in parallel; the others keep their order on one lane (each wavefront
// lists its own in order, and the wavefronts' lists are taken in turn).
// Workgroup-wide; needs 4 * T <= nslots (a power of two). key: position + 1
// (0 = empty), cnt: steps touching it, val: its entry; ST: 2 T slots.
__device__ __forceinline__ void lds_split(int32_t* D, int32_t N, int32_t a, uint64_t seed, uint32_t round,
                                          int32_t k, int32_t* key, int32_t* cnt, int32_t* val, int32_t nslots,
                                          int32_t* ST, int32_t* late, int32_t* nlate) {
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  const int w = tid >> 6;
  const int nw = nt >> 6;
  const int32_t T = split_steps(N, a);
  const bool fwd = a <= N - a;
  const int sh = 31 - __clz(nslots);
  for (int32_t i = tid; i < nslots; i += nt) { key[i] = 0; cnt[i] = 0; }
  __syncthreads();
  for (int32_t i = tid; i < 2 * T; i += nt) {
    const int32_t t = i >> 1;
    const int32_t x = (i & 1) ? split_partner(N, a, t, seed, round, k) : (fwd ? t : N - 1 - t);
    int32_t q = (int32_t)(((uint32_t)x * 2654435761u) >> (32 - sh));
    while (true) {
      const int32_t old = atomicCAS(&key[q], 0, x + 1);
      if (old == 0 || old == x + 1) break;
      q = (q + 1) & (nslots - 1);
    }
    ST[i] = q;
    atomicAdd(&cnt[q], 1);
  }
  __syncthreads();
  for (int32_t i = tid; i < nslots; i += nt)
    if (key[i] != 0) val[i] = D[key[i] - 1];
  // steps of wavefront w: [w * per, (w + 1) * per)
  const int32_t per = (T + nw - 1) / nw;
  const int32_t t_lo = w * per < T ? w * per : T, t_hi = t_lo + per < T ? t_lo + per : T;
  __syncthreads();
  int32_t nl = 0;
  for (int32_t t0 = t_lo; t0 < t_hi; t0 += kWave) {
    const int32_t t = t0 + lane_id();
    bool lt = false;
    if (t < t_hi) {
      const int32_t p = ST[2 * t], q = ST[2 * t + 1];
      if (cnt[p] == 1 && cnt[q] == 1) {
        const int32_t vp = val[p];
        val[p] = val[q];
        val[q] = vp;
      } else {
        lt = p != q;
      }
    }
    const uint64_t lm = ballot(lt);
    if (lt) late[t_lo + nl + rank_below(lm)] = t;
    nl += popc64(lm);
  }
  if (lane_id() == 0) nlate[w] = nl;
  __syncthreads();
  if (tid == 0) {
    for (int v = 0; v < nw; ++v) {
      const int32_t lo = v * per < T ? v * per : T;
      for (int32_t z = 0; z < nlate[v]; ++z) {
        const int32_t t = late[lo + z];
        const int32_t p = ST[2 * t], q = ST[2 * t + 1];
        const int32_t vp = val[p];
        val[p] = val[q];
        val[q] = vp;
      }
    }
  }
  __syncthreads();
  for (int32_t i = tid; i < nslots; i += nt)
    if (key[i] != 0) D[key[i] - 1] = val[i];
  __syncthreads();
}

// The split applied to a trade's published items at disjoint positions
// 0..N-1 (agent-scope array), as lds_split does it to D: the touched
// positions' items are gathered into an LDS hash table, swapped there, and
// written back, each with the side of its new owner (position below a: u). A
// flag bit on a key marks a position that several steps touch. Workgroup-wide;
// needs 4 * T <= nslots (a power of two).
constexpr int32_t kMultiTouch = 0x40000000;
__device__ __forceinline__ void item_split(unsigned long long* I, int32_t N, int32_t a, uint64_t seed,
                                           uint32_t round, int32_t k, int32_t* key, uint64_t* val,
                                           int32_t nslots, int32_t* ST, int32_t* late, int32_t* nlate) {
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  const int w = tid >> 6;
  const int nw = nt >> 6;
  const int32_t T = split_steps(N, a);
  const bool fwd = a <= N - a;
  const int sh = 31 - __clz(nslots);
  for (int32_t i = tid; i < nslots; i += nt) key[i] = 0;
  __syncthreads();
  for (int32_t i = tid; i < 2 * T; i += nt) {
    const int32_t t = i >> 1;
    const int32_t x = (i & 1) ? split_partner(N, a, t, seed, round, k) : (fwd ? t : N - 1 - t);
    int32_t q = (int32_t)(((uint32_t)x * 2654435761u) >> (32 - sh));
    while (true) {
      const int32_t old = atomicCAS(&key[q], 0, x + 1);
      if (old == 0) break;
      if ((old & ~kMultiTouch) == x + 1) {
        atomicOr(&key[q], kMultiTouch);
        break;
      }
      q = (q + 1) & (nslots - 1);
    }
    ST[i] = q;
  }
  __syncthreads();
  for (int32_t i = tid; i < nslots; i += nt)
    if (key[i] != 0) val[i] = load_agent_u64(&I[(key[i] & ~kMultiTouch) - 1]);
  const int32_t per = (T + nw - 1) / nw;
  const int32_t t_lo = w * per < T ? w * per : T, t_hi = t_lo + per < T ? t_lo + per : T;
  __syncthreads();
  int32_t nl = 0;
  for (int32_t t0 = t_lo; t0 < t_hi; t0 += kWave) {
    const int32_t t = t0 + lane_id();
    bool lt = false;
    if (t < t_hi) {
      const int32_t p = ST[2 * t], q = ST[2 * t + 1];
      if (!(key[p] & kMultiTouch) && !(key[q] & kMultiTouch)) {
        const uint64_t vp = val[p];
        val[p] = val[q];
        val[q] = vp;
      } else {
        lt = p != q;
      }
    }
    const uint64_t lm = ballot(lt);
    if (lt) late[t_lo + nl + rank_below(lm)] = t;
    nl += popc64(lm);
  }
  if (lane_id() == 0) nlate[w] = nl;
  __syncthreads();
  if (tid == 0) {
    for (int v = 0; v < nw; ++v) {
      const int32_t lo = v * per < T ? v * per : T;
      for (int32_t z = 0; z < nlate[v]; ++z) {
        const int32_t t = late[lo + z];
        const int32_t p = ST[2 * t], q = ST[2 * t + 1];
        const uint64_t vp = val[p];
        val[p] = val[q];
        val[q] = vp;
      }
    }
  }
  __syncthreads();
  for (int32_t i = tid; i < nslots; i += nt) {
    if (key[i] == 0) continue;
    const int32_t pos = (key[i] & ~kMultiTouch) - 1;
    store_agent_u64(&I[pos], (val[i] & ~(1ull << 32)) | ((pos < a ? 0ull : 1ull) << 32));
  }
  __syncthreads();
}

// Ready queues: `shards` queues of L slots each; q[shard * L + pos]. A pusher
// reserves a slot with its shard's tail counter and fills it; a popper takes
// a slot with a compare-and-swap on the head, waits for the fill, and
// resets the slot to -1 so the queues are clean for the next round.
__device__ __forceinline__ int32_t queue_pop(const TradeArgs& A, int32_t* q, int nscan, int head0, int tail0,
                             int start, int shards) {
  for (int i = 0; i < nscan; ++i) {
    const int sh = (start + i) % shards;
    int32_t* head = &A.ctrl[cw(head0 + sh)];
    const int32_t h = load_agent(head);
    // h >= L only after a push overflowed the shard (an error is raised then)
    if (h >= load_agent(&A.ctrl[cw(tail0 + sh)]) || h >= A.L) continue;
    if (!atomic_cas(head, h, h + 1)) continue;
    int32_t* slot = &q[(int64_t)sh * A.L + h];
    int32_t k;
    // The pusher reserved slot h before filling it; the fill is imminent.
    while ((k = load_agent(slot)) < 0) {
      if (load_agent(&A.ctrl[cw(kCwAbort)])) return -1;
      __builtin_amdgcn_s_sleep(1);
    }
    store_agent(slot, -1);
    return k;
  }
  return -1;
}

// Hand a ready trade to other workers (single lane; caller fenced).
__device__ __forceinline__ void queue_push(const TradeArgs& A, int32_t* q, int tail0, int shard,
                                           int32_t k) {
  const int32_t pos = atomic_add(&A.ctrl[cw(tail0 + shard)], 1);
  if (pos >= A.L) { raise_error(A, kErrCapacity); return; }
  store_agent(&q[(int64_t)shard * A.L + pos], k);
}

__device__ __forceinline__ int32_t source_pop(const TradeArgs& A) {
  const int32_t count = load_agent(&A.ctrl[cw(kCwSrcCount)]);
  if (load_agent(&A.ctrl[cw(kCwSrcHead)]) >= count) return -1;
  const int32_t h = atomic_add(&A.ctrl[cw(kCwSrcHead)], 1);
  return h < count ? A.src_list[h] : -1;
}

// Idle wait that grows with the time spent idle (fewer polls of the shared
// control words while there is nothing to do).
constexpr int32_t kBigMaxBackoff = 1;    // idle workgroup workers: longest back-off level (about 1 us)
__device__ __forceinline__ void idle_backoff(int32_t level) {
  for (int32_t i = 0; i < level; ++i) __builtin_amdgcn_s_sleep(32);
}

// Watchdog bookkeeping of an idle worker: true when no trade has completed
// anywhere for longer than the limit.
struct Watchdog {
  int32_t last_done;
  uint64_t since;
  __device__ __forceinline__ bool stalled(const TradeArgs& A, int32_t done) {
    const uint64_t now = now_ticks();
    if (since == 0 || done != last_done) {
      last_done = done;
      since = now;
      return false;
    }
    return now - since > A.watchdog_ticks;
  }
};

// Emit/forward one output edge {owner, x}. Returns true if it is forwarded.
__device__ __forceinline__ void route_edge(const TradeArgs& A, int32_t owner, int32_t x,
                                           uint32_t tag, int32_t k) {
  if (tag == kTagPartner) return;  // own row only (handled by the caller)
  const uint4 ni = A.ninfo[x];
  const int64_t rx = ni.x;
  const int32_t dx = (int32_t)ni.y;
  if (tag == kTagEmit) {
    const int32_t p = atomic_add(&A.out_cur[x], 1);
    if (p < dx) A.col_out[rx + p] = owner; else raise_error(A, kErrOut, k, x);
  } else {
    const int32_t p = atomic_add(&A.inbox_cur[x], 1);
    if (p >= dx) raise_error(A, kErrInbox, k, x);
    else if (tag & kTagGiant) giant_insert(A.gs, A.gs.giant_id[x], owner);
    else store_agent(&A.inbox[rx + p], owner);
  }
}

// ============================================================ write phase of large trades

constexpr int kBatch = 8;   // items per lane in flight in the write phase

// Output items of a large trade after the split: D[0..nD) are the disjoint
// entries (u receives positions below a), D[nD..s) the kept ones (shared
// neighbours and the partner); item o is entry E[D[o]]. A shared write phase
// reads them from one published array instead (E = items, D unused).
struct ItemSrc {
  const uint64_t* E;
  const int32_t* D;
  int32_t k, u, v, s, nD, a, du, dv;
  int64_t bu, bv;
  int32_t gu, gv;   // giant ids of u and v (-1: none); their bitmaps are cleared here
};

struct WriteCounts {   // per lane
  unsigned long long fwd, emit, push;
  uint32_t moved;
};

// Item o: its entry, with the side bit replaced by the side of its owner
// (0: u, 1: v). Shared: read from the published item array S.E[o].
template <bool kShared>
__device__ __forceinline__ uint64_t item_entry(const ItemSrc& S, int32_t o) {
  if (kShared) return load_agent_u64(reinterpret_cast<const unsigned long long*>(S.E) + o);
  const uint64_t e = S.E[S.D[o]];
  const uint64_t own = o < S.nD ? (o < S.a ? 0ull : 1ull) : (uint64_t)ent_side(e);
  return (e & ~(1ull << 32)) | (own << 32);
}

// Write items first, first + step, ... below end (a wavefront handles kBatch
// * 64 consecutive items per step): own-row entries at positions drawn from
// own_ctr[0] (u) and own_ctr[1] (v), final entries of other rows, inbox
// entries of later trades; each forwarded item then drops its target trade's
// counter once this wave's writes are complete, and a trade that becomes
// ready is queued. kShared: the arrays and own_ctr are in global memory,
// written by another workgroup.
template <bool kShared>
__device__ __forceinline__ void write_range(const TradeArgs& A, const ItemSrc& S, int32_t first, int32_t end,
                            int32_t step, int32_t* own_ctr, WriteCounts& W) {
  const int l = lane_id();
  for (int32_t base = first; base < end; base += step) {
    int32_t tx[kBatch], towner[kBatch], tp[kBatch];
    uint32_t ttag[kBatch];
    uint64_t mu[kBatch], mv[kBatch];
    int32_t nu = 0, nv = 0;
#pragma unroll
    for (int r = 0; r < kBatch; ++r) {
      const int32_t o = base + r * kWave + l;
      tx[r] = -1;
      tp[r] = 0;
      ttag[r] = 0;
      towner[r] = S.u;
      if (o < end) {
        const uint64_t e = item_entry<kShared>(S, o);
        tx[r] = ent_node(e);
        ttag[r] = ent_tag(e);
        towner[r] = ent_side(e) ? S.v : S.u;
        // a disjoint neighbour that changed sides (the published items of a
        // shared phase no longer carry their old side)
        if (!kShared && o < S.nD) W.moved += (uint32_t)(ent_side(S.E[S.D[o]]) != (o < S.a ? 0 : 1));
      }
    }
    // members of a giant node's list learn their tag here, one gather each,
    // and their bitmap words are cleared for the next round (every member of
    // a giant's set is an item of this trade; nothing reads the set again
    // this round)
    // the target rows' offsets and degrees come with the tags (one load)
    int32_t tinf[kBatch];
    int64_t rxa[kBatch];
    int32_t dxa[kBatch];
#pragma unroll
    for (int r = 0; r < kBatch; ++r) {
      const bool unk = tx[r] >= 0 && ttag[r] == kTagUnknown;
      const uint4 ni = tx[r] >= 0 ? A.ninfo[tx[r]] : make_uint4(0u, 0u, 0u, 0u);
      tinf[r] = unk ? (int32_t)ni.z : 0;
      rxa[r] = ni.x;
      dxa[r] = (int32_t)ni.y;
      if (unk) {
        if (S.gu >= 0) A.gs.bm[(int64_t)S.gu * A.gs.gwords + (tx[r] >> 6)] = 0ull;
        if (S.gv >= 0) A.gs.bm[(int64_t)S.gv * A.gs.gwords + (tx[r] >> 6)] = 0ull;
      }
    }
#pragma unroll
    for (int r = 0; r < kBatch; ++r) {
      if (tx[r] >= 0 && ttag[r] == kTagUnknown) ttag[r] = tag_of(tinf[r], S.k);
      const bool own = tx[r] >= 0 && ttag[r] <= kTagPartner;
      mu[r] = ballot(own && towner[r] == S.u);
      mv[r] = ballot(own && towner[r] == S.v);
      nu += popc64(mu[r]);
      nv += popc64(mv[r]);
      if (tx[r] >= 0 && ttag[r] == kTagEmit) tp[r] = atomic_add(&A.out_cur[tx[r]], 1);
      else if (tx[r] >= 0 && ttag[r] >= 2u) tp[r] = atomic_add(&A.inbox_cur[tx[r]], 1);
    }
    int32_t pu = 0, pv = 0;
    if (l == 0) {
      if (kShared) {
        if (nu) pu = atomic_add(&own_ctr[0], nu);
        if (nv) pv = atomic_add(&own_ctr[1], nv);
      } else {
        if (nu) pu = atomicAdd(&own_ctr[0], nu);
        if (nv) pv = atomicAdd(&own_ctr[1], nv);
      }
    }
    pu = wave_bcast(pu, 0);
    pv = wave_bcast(pv, 0);
    bool fwd[kBatch];
#pragma unroll
    for (int r = 0; r < kBatch; ++r) {
      fwd[r] = false;
      const bool ou = (mu[r] >> l) & 1ull, ov = (mv[r] >> l) & 1ull;
      if (ou || ov) {
        const int32_t p = ou ? pu + rank_below(mu[r]) : pv + rank_below(mv[r]);
        const int32_t dd = ou ? S.du : S.dv;
        if (p < dd) A.col_out[(ou ? S.bu : S.bv) + (dd - 1 - p)] = tx[r];
        else raise_error(A, kErrOut, S.k, -2 - towner[r]);
      }
      pu += popc64(mu[r]);
      pv += popc64(mv[r]);
      if (tx[r] < 0 || ttag[r] == kTagPartner) continue;
      const int64_t rx = rxa[r];
      const int32_t dx = dxa[r];
      if (tp[r] >= dx) { raise_error(A, ttag[r] == kTagEmit ? kErrOut : kErrInbox, S.k, tx[r]); continue; }
      if (ttag[r] == kTagEmit) {
        A.col_out[rx + tp[r]] = towner[r];
        W.emit += 1;
      } else {
        if (ttag[r] & kTagGiant) giant_insert(A.gs, A.gs.giant_id[tx[r]], towner[r]);
        else store_agent(&A.inbox[rx + tp[r]], towner[r]);
        fwd[r] = true;
        W.fwd += 1;
      }
    }
    // this wave's inbox and bitmap writes are complete before any counter
    // they unlock
    publish_wait();
    int32_t old[kBatch];
#pragma unroll
    for (int r = 0; r < kBatch; ++r)
      if (fwd[r]) old[r] = atomic_add(&A.dep[tag_trade(ttag[r])], -1);
#pragma unroll
    for (int r = 0; r < kBatch; ++r) {
      if (!fwd[r]) continue;
      const int32_t t = tag_trade(ttag[r]);
      if (old[r] <= 0) raise_error(A, kErrDep, t, S.k);
      if (old[r] == 1) {
        const bool big = A.tsz[t] > A.small_max;
        if (A.trace) {
          A.trace[kTraceFields * (int64_t)t] = (int64_t)now_ticks();
          A.trace[kTraceFields * (int64_t)t + 3] = S.k;
        }
        const int sh = (int)((blockIdx.x * 7 + threadIdx.x) % kQsShards);
        if (big) queue_push(A, A.qb, kCwQbTail0, sh % kQbShards, t);
        else queue_push(A, A.qs, kCwQsTail0, sh, t);
        W.push += 1;
      }
    }
  }
}

// Ticket fields.
constexpr unsigned long long kTicketMask = (1ull << kTicketCountBits) - 1;
__device__ __forceinline__ uint32_t ticket_gen(unsigned long long t) { return (uint32_t)(t >> (2 * kTicketCountBits)); }
__device__ __forceinline__ int32_t ticket_chunks(unsigned long long t) { return (int32_t)((t >> kTicketCountBits) & kTicketMask); }
__device__ __forceinline__ int32_t ticket_next(unsigned long long t) { return (int32_t)(t & kTicketMask); }

// Claim a chunk of a job (single lane): the chunk index, or -1 when the job
// has none left. A job whose chunks are all taken is not incremented again
// except by claims racing with the last one.
__device__ __forceinline__ int32_t claim_chunk(HelpJob* J, uint32_t* gen = nullptr) {
  const unsigned long long seen = load_agent_u64(&J->t.ticket);
  if (ticket_next(seen) >= ticket_chunks(seen)) return -1;
  const unsigned long long t =
      __hip_atomic_fetch_add(&J->t.ticket, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (gen) *gen = ticket_gen(t);
  return ticket_next(t) < ticket_chunks(t) ? ticket_next(t) : -1;
}

// Mask word of owner's jobs: kCwJobMask0/1 (write phases, taken by single
// wavefronts) or kCwJobMask2/3 (parts of a bitmap pass, taken by workgroups).
__device__ __forceinline__ int32_t* job_mask(const TradeArgs& A, int owner, int base = kCwJobMask0) {
  return &A.ctrl[cw(base + (owner < 32 ? 0 : 1))];
}

// Extraction of a giant's neighbour set shared with helper wavefronts is
// switched off: a run with it on (every workgroup trade sharing its phases,
// one giant node) did not finish and its cause is not found yet.
constexpr bool kSharedExtraction = false;

// Offset of the shared list (written only with agent-scope stores, by the
// owner and by helpers) within a slot.
__device__ __forceinline__ int64_t shared_list_off(const TradeArgs& A) { return 2 * A.smax + A.smax / 2 + 1; }

// Open the calling workgroup's job, of nchunks chunks, with its fields
// already stored (thread 0).
__device__ __forceinline__ void open_job(const TradeArgs& A, HelpJob* J, int32_t nchunks,
                                         int mask = kCwJobMask0) {
  store_agent(&J->c.done, 0);
  store_agent(&J->c.own[0], 0);
  store_agent(&J->c.own[1], 0);
  publish_wait();
  const unsigned long long gen = (ticket_gen(load_agent_u64(&J->t.ticket)) + 1u) & 0xFFFFull;
  store_agent_u64(&J->t.ticket, (gen << (2 * kTicketCountBits)) |
                                    ((unsigned long long)nchunks << kTicketCountBits));
  publish_wait();
  atomic_or(job_mask(A, blockIdx.x, mask), (int32_t)(1u << (blockIdx.x & 31)));
}

// Every chunk is claimed: close the job and wait for the helpers (thread 0).
__device__ __forceinline__ void close_job(const TradeArgs& A, HelpJob* J, int32_t nchunks,
                                          int mask = kCwJobMask0) {
  atomic_and(job_mask(A, blockIdx.x, mask), (int32_t)~(1u << (blockIdx.x & 31)));
  while (load_agent(&J->c.done) < nchunks) {
    if (load_agent(&A.ctrl[cw(kCwAbort)])) break;
    __builtin_amdgcn_s_sleep(2);
  }
}

// Phase 1 chunk c (one wavefront): the members of giant gi in superblocks
// [c * kSbChunk, ...), as entries of `side` of trade k, at their positions
// pre[j] + rank in X; their bitmap words and counts are cleared.
__device__ __forceinline__ void extract_chunk(const TradeArgs& A, int32_t k, int32_t gi, int side,
                                              int32_t nsb, const int32_t* pre, unsigned long long* X,
                                              int32_t c) {
  constexpr int kStep = 4;
  const int l = lane_id();
  unsigned long long* bm = A.gs.bm + (int64_t)gi * A.gs.gwords;
  int32_t* sc = A.gs.sc + (int64_t)gi * nsb;
  const int32_t sb0 = c * kSbChunk;
  const int32_t sb1 = sb0 + kSbChunk < nsb ? sb0 + kSbChunk : nsb;
  bool bad = false;
  for (int32_t j0 = sb0; j0 < sb1; j0 += kStep) {
    unsigned long long word[kStep];
    int32_t lo[kStep], hi[kStep];
#pragma unroll
    for (int t = 0; t < kStep; ++t) {
      const int32_t jj = j0 + t;
      const bool valid = jj < sb1;
      word[t] = valid ? load_agent_u64(&bm[(int64_t)jj * kWave + l]) : 0ull;
      lo[t] = valid ? load_agent(&pre[jj]) : 0;
      hi[t] = valid ? load_agent(&pre[jj + 1]) : 0;
    }
#pragma unroll
    for (int t = 0; t < kStep; ++t) {
      const int32_t jj = j0 + t;
      if (jj >= sb1) break;
      unsigned long long bits = word[t];
      const int32_t pc = __popcll(bits);
      const int32_t at = lo[t] + wave_incl_scan(pc) - pc;
      if (wave_sum(pc) != hi[t] - lo[t]) bad = true;
      const int64_t wi = (int64_t)jj * kWave + l;
      int32_t idx = 0;
      while (bits) {
        const int bit = __builtin_ctzll(bits);
        bits &= bits - 1;
        const int32_t x = (int32_t)(wi * 64 + bit);
        if (at + idx < hi[t]) store_agent_u64(&X[at + idx], make_entry(x, side, kTagUnknown));
        ++idx;
      }
      if (l == 0) store_agent(&sc[jj], 0);
    }
  }
  if (ballot(bad) && l == 0) raise_error(A, kErrGather, k, 4000000 + c);
}

// Giant gi's neighbour set (d members) as ascending entries of `side` of
// trade k in the shared list of this workgroup's slot, extracted by this
// workgroup and idle helper wavefronts. Workgroup-wide; false on an error.
__device__ __forceinline__ bool extract_giant_shared(const TradeArgs& A, int32_t k, int32_t gi, int side,
                                                     int32_t d, BigLds& B) {
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  const int32_t nsb = (int32_t)(A.gs.gwords >> 6);
  const int32_t* sc = A.gs.sc + (int64_t)gi * nsb;
  int32_t* pre = A.sbpre + (int64_t)blockIdx.x * A.sbpre_stride;
  int32_t carry = 0;
  for (int32_t j0 = 0; j0 < nsb; j0 += nt) {
    const int32_t j = j0 + tid;
    const int32_t cnt = j < nsb ? load_agent(&sc[j]) : 0;
    int32_t tot;
    const int32_t p = block_excl_scan(cnt, B.scan, &tot);
    if (j < nsb) store_agent(&pre[j], carry + p);
    carry += tot;
  }
  if (carry != d) {
    if (tid == 0) raise_error(A, kErrGather, k, 3000000 + carry - d);
    return false;
  }
  if (tid == 0) store_agent(&pre[nsb], carry);
  HelpJob* J = A.jobs + blockIdx.x;
  const int32_t nchunks = (nsb + kSbChunk - 1) / kSbChunk;
  publish_wait();
  __syncthreads();
  if (tid == 0) {
    store_agent(&J->f.phase, 1);
    store_agent(&J->f.k, k);
    store_agent(&J->f.gi, gi);
    store_agent(&J->f.side, side);
    store_agent(&J->f.d, d);
    store_agent64(&J->f.e_off, shared_list_off(A));
    open_job(A, J, nchunks);
  }
  __syncthreads();
  unsigned long long* X =
      reinterpret_cast<unsigned long long*>(A.slots + (int64_t)blockIdx.x * A.slot_elems + shared_list_off(A));
  for (;;) {
    int32_t c = -1;
    if (lane_id() == 0) c = claim_chunk(J);
    c = wave_bcast(c, 0);
    if (c < 0) break;
    extract_chunk(A, k, gi, side, nsb, pre, X, c);
    publish_wait();
    if (lane_id() == 0) atomic_add(&J->c.done, 1);
  }
  __syncthreads();
  // one decision for the whole workgroup: the abort word may change meanwhile
  if (tid == 0) {
    close_job(A, J, nchunks);
    B.flag = load_agent(&A.ctrl[cw(kCwAbort)]);
  }
  __syncthreads();
  return B.flag == 0;
}

// Helper groups: workgroup b helps only the jobs of owners j with
// j % G == b % G (G = help_groups, a divisor of 64), so a job is shared by a
// bounded set of workgroups and claims of different jobs do not meet on one
// word.
__device__ __forceinline__ uint64_t help_group_mask(int32_t b, int32_t groups) {
  uint64_t m = 0;
  for (int j = b % groups; j < kMaxJobs; j += groups) m |= 1ull << j;
  return m;
}

// An idle wavefront of workgroup b writes chunks of an open write job of its
// group, if there is one: up to `runs` chunks of that job in a row, so the
// fields are read once per generation, not once per chunk.
constexpr int kHelpRun = 8;   // chunks in a row for a wavefront worker (a workgroup worker takes one)
__device__ __forceinline__ bool try_help(const TradeArgs& A, int32_t b, WriteCounts& W, int runs) {
  const int l = lane_id();
  int32_t j = -1, c = -1;
  uint32_t gen = 0;
  if (l == 0) {
    const uint64_t group = help_group_mask(b, A.help_groups);
    const uint64_t m = ((uint64_t)(uint32_t)load_agent(&A.ctrl[cw(kCwJobMask0)]) |
                        ((uint64_t)(uint32_t)load_agent(&A.ctrl[cw(kCwJobMask1)]) << 32)) & group;
    if (m) {
      // spread the waves of one workgroup over the open jobs of its group
      const int rot = (int)((threadIdx.x >> 6) * A.help_groups) & 63;
      const uint64_t rm = rot ? ((m >> rot) | (m << (64 - rot))) : m;
      j = (int32_t)((__builtin_ctzll(rm) + rot) & 63);
      c = claim_chunk(A.jobs + j, &gen);
    }
  }
  c = wave_bcast(c, 0);
  if (c < 0) return false;
  j = wave_bcast(j, 0);
  HelpJob* J = A.jobs + j;
  const uint64_t* slot = A.slots + (int64_t)j * A.slot_elems;
  ItemSrc S;
  uint32_t have = 0;   // generation whose fields S holds (0: none yet)
  int32_t phase = 0;
  for (int run = 0;;) {
    consume_order();
    // the fields of the claimed generation stay put until this chunk is reported
    gen = (uint32_t)wave_bcast((int32_t)gen, 0) | 0x10000u;
    if (have != gen) phase = load_agent(&J->f.phase);
    if (phase == 1) {
      extract_chunk(A, load_agent(&J->f.k), load_agent(&J->f.gi), load_agent(&J->f.side),
                    (int32_t)(A.gs.gwords >> 6), A.sbpre + (int64_t)j * A.sbpre_stride,
                    reinterpret_cast<unsigned long long*>(const_cast<uint64_t*>(slot) + load_agent64(&J->f.e_off)),
                    c);
      have = gen;
    } else {
      if (have != gen) {
        S.E = slot + load_agent64(&J->f.e_off);
        S.D = nullptr;
        S.k = load_agent(&J->f.k);
        S.u = load_agent(&J->f.u);
        S.v = load_agent(&J->f.v);
        S.s = load_agent(&J->f.s);
        S.nD = load_agent(&J->f.nD);
        S.a = load_agent(&J->f.a);
        S.du = load_agent(&J->f.du);
        S.dv = load_agent(&J->f.dv);
        S.bu = load_agent64(&J->f.bu);
        S.bv = load_agent64(&J->f.bv);
        S.gu = load_agent(&J->f.gu);
        S.gv = load_agent(&J->f.gv);
        have = gen;
      }
      const int32_t first = c * A.help_chunk;
      const int32_t end = first + A.help_chunk < S.s ? first + A.help_chunk : S.s;
      write_range<true>(A, S, first, end, kWave * kBatch, J->c.own, W);
    }
    publish_wait();
    if (l == 0) atomic_add(&J->c.done, 1);
    if (++run >= runs) break;
    // the next chunk of the same job; a new generation brings new fields
    c = -1;
    if (l == 0) c = claim_chunk(J, &gen);
    c = wave_bcast(c, 0);
    if (c < 0) break;
  }
  return true;
}

// ============================================================ small trades

struct WaveState {
  int32_t top;        // ready trades kept locally (uniform)
  int32_t head;       // ... the oldest of them, in a ring of kStackCap slots
  int32_t ndone;
  int32_t shard;      // home shard of the small-trade queues
  int32_t* pool;      // the workgroup's pool of ready trades (LDS; null: none)
  unsigned long long n_small, n_push, work, fwd, emit, ticks, moved;
};

// Put trade t into a free pool slot (wave-wide, t uniform): false if the pool
// stays full after a few tries.
__device__ __forceinline__ bool pool_put(int32_t* pool, int32_t t) {
  for (int tries = 0; tries < 4; ++tries) {
    const uint64_t freem = ballot(pool[lane_id()] < 0);
    if (!freem) return false;
    int32_t ok = 0;
    if (lane_id() == 0) ok = atomicCAS(&pool[__builtin_ctzll(freem)], -1, t) == -1;
    if (wave_bcast(ok, 0)) return true;
  }
  return false;
}

// Take a trade from the pool (wave-wide): -1 if it is empty.
__device__ __forceinline__ int32_t pool_take(int32_t* pool) {
  for (int tries = 0; tries < 4; ++tries) {
    const uint64_t full = ballot(pool[lane_id()] >= 0);
    if (!full) return -1;
    int32_t k = -1;
    if (lane_id() == 0) k = atomicExch(&pool[__builtin_ctzll(full)], -1);
    k = wave_bcast(k, 0);
    if (k >= 0) return k;
  }
  return -1;
}

// Drops the dependency counters of later trades reached by trade k's
// output; a ready small trade goes to the local stack or the global queue,
// a ready large one to the workgroup queues.
__device__ __forceinline__ void wave_release_ready(const TradeArgs& A, WaveLds& W, WaveState& S,
                                                   bool ready, int32_t t, int32_t k) {
  if (ballot(ready) == 0) return;
  bool big = false;
  if (ready) {
    big = A.tsz[t] > A.small_max;
    if (A.trace) {
      A.trace[kTraceFields * (int64_t)t] = (int64_t)now_ticks();
      A.trace[kTraceFields * (int64_t)t + 3] = k;
    }
  }
  const bool keep = ready && !big;
  const uint64_t m = ballot(keep);
  const int cnt = popc64(m);
  const int room = A.stack_cap - S.top;
  const int r = rank_below(m);
  // beyond the local stack: the workgroup's pool, else the global queues
  uint64_t rest = ballot(keep && r >= room);
  if (rest && S.pool) {
    uint64_t pooled = 0;
    for (uint64_t left = rest; left; left &= left - 1) {
      const int ln = __builtin_ctzll(left);
      if (pool_put(S.pool, wave_bcast(t, ln))) pooled |= 1ull << ln;
      else break;
    }
    rest &= ~pooled;
  }
  const uint64_t spill = rest | ballot(big);
  if (spill) publish_wait();
  if (keep && r < room) W.stack[(S.head + S.top + r) & (kStackCap - 1)] = t;
  else if (keep && ((rest >> lane_id()) & 1ull)) queue_push(A, A.qs, kCwQsTail0, S.shard, t);
  else if (big) queue_push(A, A.qb, kCwQbTail0, S.shard % kQbShards, t);
  wave_sync();
  S.top += cnt < room ? cnt : (room > 0 ? room : 0);
  S.n_push += (unsigned long long)popc64(spill);
}

__device__ __forceinline__ void small_trade(const TradeArgs& A, int32_t k, int32_t u, int32_t v, WaveLds& W,
                            WaveState& S) {
  const int l = lane_id();
  const int64_t bu = A.rp[u], bv = A.rp[v];
  const int32_t du = (int32_t)(A.rp[u + 1] - bu), dv = (int32_t)(A.rp[v + 1] - bv);
  const int32_t s = du + dv;
  const int32_t niu = load_agent(&A.inbox_cur[u]);
  const int32_t niv = load_agent(&A.inbox_cur[v]);

  // ---- gather both lists into E (u's at [0, du), v's at [du, s)): row
  // entries of later nodes from the front of each side's range, arrivals
  // from its back. A row's inbox has as many slots as the row, so slot e is
  // read with row entry e (kept if e is below the arrival count): every
  // load of both rows in one round trip.
  constexpr int kGatherIt = kSmallCap / kWave;
  int32_t gx[kGatherIt], gt[kGatherIt], gy[kGatherIt];
#pragma unroll
  for (int it = 0; it < kGatherIt; ++it) {
    const int32_t i = it * kWave + l;
    gx[it] = 0;
    gt[it] = -1;
    gy[it] = 0;
    if (i < s) {
      const int64_t at = i < du ? bu + i : bv + (i - du);
      gx[it] = A.col[at];
      gt[it] = A.col_t[at];
      gy[it] = load_agent(&A.inbox[at]);
    }
  }
  int32_t cnt0 = 0, cnt1 = 0;
#pragma unroll
  for (int it = 0; it < kGatherIt; ++it) {
    if (it * kWave >= s) break;   // uniform across the wavefront
    const int32_t i = it * kWave + l;
    const int side = i < du ? 0 : 1;
    const bool fresh = i < s && tinfo_trade(gt[it]) >= k;
    const uint64_t m0 = ballot(fresh && side == 0);
    const uint64_t m1 = ballot(fresh && side == 1);
    if (fresh)
      W.E[side ? du + cnt1 + rank_below(m1) : cnt0 + rank_below(m0)] = make_entry(gx[it], side, tag_of(gt[it], k));
    cnt0 += popc64(m0);
    cnt1 += popc64(m1);
    if (i < du) {
      if (i < niu && niu <= du) W.E[du - 1 - i] = make_entry(gy[it], 0, kTagEmit);
    } else if (i < s) {
      if (i - du < niv && niv <= dv) W.E[s - 1 - (i - du)] = make_entry(gy[it], 1, kTagEmit);
    }
  }
  if (cnt0 + niu != du) { raise_error(A, kErrGather, k, (cnt0 + niu) - du); return; }
  if (cnt1 + niv != dv) { raise_error(A, kErrGather, k, (cnt1 + niv) - dv); return; }
  wave_sync();
  wave_bitonic_sort(W.E, (uint32_t)s);

  // ---- classify: shared (C), partner (P), disjoint (D[0..nD), ascending);
  // the kept ones (C, P) fill D[nD..s) from the back
  int32_t nD = 0, a = 0, nk = 0;
  for (int32_t c = 0; c < s; c += kWave) {
    const int32_t i = c + l;
    bool isD = false;
    int side = 0;
    if (i < s) {
      const uint64_t e = W.E[i];
      const int32_t x = ent_node(e);
      side = ent_side(e);
      const bool isP = ent_tag(e) == kTagPartner;
      const bool isC = !isP && ((i > 0 && ent_node(W.E[i - 1]) == x) ||
                                (i + 1 < s && ent_node(W.E[i + 1]) == x));
      isD = !isP && !isC;
    }
    const uint64_t m = ballot(isD);
    if (isD) W.D[nD + rank_below(m)] = i;
    nD += popc64(m);
    a += popc64(ballot(isD && side == 0));
    const uint64_t mk = ballot(i < s && !isD);
    if (i < s && !isD) W.D[s - 1 - (nk + rank_below(mk))] = i;
    nk += popc64(mk);
  }
  wave_sync();
  const DrawKey dk = draw_key(A, k);
  wave_split(W.D, nD, a, dk.seed, dk.round, dk.idx, W.R);

  // ---- write: kWriteIt * 64 items at a time (all of most trades). Item o is
  // entry E[D[o]]; a disjoint one (o < nD) goes to u below position a, a
  // kept one stays with its side. Own-row finals take their positions with
  // one out_cur atomic per row; other-row finals and forwards reserve a slot
  // of their target row; once this wavefront's writes are complete, every
  // forward drops its target trade's counter (one round trip for all).
  constexpr int kWriteIt = 8;
  int32_t nmoved = 0, nfwd = 0, nemit = 0;
  for (int32_t o0 = 0; o0 < s; o0 += kWriteIt * kWave) {
  int32_t ix[kWriteIt], ip[kWriteIt], isd[kWriteIt];
  uint32_t itag[kWriteIt];
  int64_t irx[kWriteIt];
  int32_t idd[kWriteIt];
  int32_t nu = 0, nv = 0;
#pragma unroll
  for (int it = 0; it < kWriteIt; ++it) {
    const int32_t o = o0 + it * kWave + l;
    ix[it] = -1;
    itag[it] = kTagPartner;
    isd[it] = 0;
    ip[it] = 0;
    irx[it] = 0;
    idd[it] = 0;
    if (o < s) {
      const uint64_t e = W.E[W.D[o]];
      ix[it] = ent_node(e);
      itag[it] = ent_tag(e);
      isd[it] = o < nD ? (o < a ? 0 : 1) : ent_side(e);
      if (o < nD) nmoved += ent_side(e) != isd[it] ? 1 : 0;
      if (itag[it] != kTagPartner) {
        const uint4 ni = A.ninfo[ix[it]];
        irx[it] = ni.x;
        idd[it] = (int32_t)ni.y;
        ip[it] = atomic_add(itag[it] == kTagEmit ? &A.out_cur[ix[it]] : &A.inbox_cur[ix[it]], 1);
      }
    }
    const bool own = ix[it] >= 0 && itag[it] <= kTagPartner;
    nu += popc64(ballot(own && isd[it] == 0));
    nv += popc64(ballot(own && isd[it] == 1));
  }
  int32_t baseu = 0, basev = 0;
  if (l == 0) {
    if (nu) baseu = atomic_add(&A.out_cur[u], nu);
    if (nv) basev = atomic_add(&A.out_cur[v], nv);
  }
  baseu = wave_bcast(baseu, 0);
  basev = wave_bcast(basev, 0);
  int32_t cfwd = 0, cemit = 0;
  bool fwd[kWriteIt];
#pragma unroll
  for (int it = 0; it < kWriteIt; ++it) {
    const bool own = ix[it] >= 0 && itag[it] <= kTagPartner;
    const uint64_t mu = ballot(own && isd[it] == 0);
    const uint64_t mv = ballot(own && isd[it] == 1);
    const int32_t owner = isd[it] ? v : u;
    if (own) {
      const int32_t p = isd[it] ? basev + rank_below(mv) : baseu + rank_below(mu);
      const int32_t dd = isd[it] ? dv : du;
      if (p < dd) A.col_out[(isd[it] ? bv : bu) + p] = ix[it]; else raise_error(A, kErrOut, k, -2 - owner);
    }
    baseu += popc64(mu);
    basev += popc64(mv);
    fwd[it] = false;
    if (ix[it] >= 0 && itag[it] != kTagPartner) {
      if (ip[it] >= idd[it]) {
        raise_error(A, itag[it] == kTagEmit ? kErrOut : kErrInbox, k, ix[it]);
      } else if (itag[it] == kTagEmit) {
        A.col_out[irx[it] + ip[it]] = owner;
        cemit += 1;
      } else {
        if (itag[it] & kTagGiant) giant_insert(A.gs, A.gs.giant_id[ix[it]], owner);
        else store_agent(&A.inbox[irx[it] + ip[it]], owner);
        fwd[it] = true;
        cfwd += 1;
      }
    }
  }
  cfwd = wave_sum(cfwd);
  nfwd += cfwd;
  nemit += wave_sum(cemit);
  if (cfwd) {
    // the inbox entries and bitmap bits are written before the counters
    // they unlock
    publish_wait();
    int32_t old[kWriteIt];
#pragma unroll
    for (int it = 0; it < kWriteIt; ++it) old[it] = fwd[it] ? atomic_add(&A.dep[tag_trade(itag[it])], -1) : 2;
#pragma unroll
    for (int it = 0; it < kWriteIt; ++it) {
      if (o0 + it * kWave >= s) break;   // uniform across the wavefront
      const int32_t t = fwd[it] ? tag_trade(itag[it]) : -1;
      if (fwd[it] && old[it] <= 0) raise_error(A, kErrDep, t, -1 - old[it]);
      wave_release_ready(A, W, S, fwd[it] && old[it] == 1, t, k);
    }
  }
  }
  S.n_small += 1;
  S.work += (unsigned long long)s;
  S.fwd += (unsigned long long)nfwd;
  S.moved += (unsigned long long)wave_sum(nmoved);
  S.emit += (unsigned long long)nemit;
}

__device__ __forceinline__ void wave_flush(const TradeArgs& A, WaveState& S) {
  if (lane_id() == 0) {
    if (S.ndone) atomic_add(&A.ctrl[cw(kCwDone)], S.ndone);
    if (S.n_small) atomicAdd(&A.stats[kStatSmall], S.n_small);
    if (S.n_push) atomicAdd(&A.stats[kStatPush], S.n_push);
    if (S.work) atomicAdd(&A.stats[kStatWork], S.work);
    if (S.fwd) atomicAdd(&A.stats[kStatForward], S.fwd);
    if (S.emit) atomicAdd(&A.stats[kStatEmit], S.emit);
    if (S.ticks) atomicAdd(&A.stats[kStatSmallTicks], S.ticks);
    if (S.moved) atomicAdd(&A.stats[kStatMoved], S.moved);
    if (S.n_small) atomicAdd(&A.stats[kStatCounted], S.n_small);
  }
  S.ndone = 0;
  S.n_small = S.n_push = S.work = S.fwd = S.emit = S.ticks = S.moved = 0;
}

constexpr int32_t kFlushEvery = 32;   // trades between progress flushes
// An idle wavefront worker scans this many ready-queue shards per poll
// (rotating; the many idle wavefronts cover every shard between them) and
// sleeps up to A.idle_backoff * 32 * 64 cycles (about 110 us at the default
// 128) between polls, which keeps the polls of the shared control words from
// crowding the memory side on large graphs; small graphs, where ready trades
// would wait for a sleeping poller, want a short back-off.
constexpr int kQsScan = 1;
constexpr int32_t kLocalRun = 4;   // local trades between two polls of a queue shard

__device__ __forceinline__ void small_worker(const TradeArgs& A, WaveLds& W, int32_t* pool) {
  const int l = lane_id();
  const int32_t wid = (int32_t)(blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6));
  WaveState S{};
  S.shard = wid % kQsShards;
  S.pool = A.cu_pool ? pool : nullptr;
  Watchdog wd{0, 0};
  int32_t backoff = 1;
  bool sources_left = true;   // no trade becomes a source during the kernel
  int32_t scan = S.shard;
  int32_t local_run = 0;   // trades taken from the ring and pool since the last queue poll
  for (;;) {
    int32_t k = -1;
    // every kLocalRun local trades, one poll of a queue shard first: trades
    // released by workgroup trades (and overflow) wait there, and wavefronts
    // that keep finding local work would leave them waiting
    if (local_run >= kLocalRun) {
      local_run = 0;
      if (l == 0) {
        k = queue_pop(A, A.qs, kQsScan, kCwQsHead0, kCwQsTail0, scan, kQsShards);
        scan = (scan + kQsScan) % kQsShards;
      }
      k = wave_bcast(k, 0);
    }
    if (k >= 0) {
      // taken from a queue shard
    } else if (S.top > 0) {
      // oldest first: a trade that waits here may be on the critical path,
      // and newer ones would keep it at the bottom of a stack
      S.top -= 1;
      k = W.stack[S.head];
      S.head = (S.head + 1) & (kStackCap - 1);
      ++local_run;
    } else if (S.pool && (k = pool_take(S.pool)) >= 0) {
      ++local_run;
      // a ready trade left by a wavefront of this workgroup
    } else {
      if (l == 0) {
        // released trades before sources: a released trade may be on the
        // round's critical path, a source has waited for nothing
        k = queue_pop(A, A.qs, kQsScan, kCwQsHead0, kCwQsTail0, scan, kQsShards);
        scan = (scan + kQsScan) % kQsShards;
        if (k < 0 && sources_left) {
          k = source_pop(A);
          sources_left = k >= 0;
        }
      }
      k = wave_bcast(k, 0);
    }
    if (k < 0) {
      wave_flush(A, S);
      int32_t stop = 0;
      if (l == 0) {
        const int32_t done = load_agent(&A.ctrl[cw(kCwDone)]);
        stop = load_agent(&A.ctrl[cw(kCwAbort)]) || done >= A.L;
        if (!stop && wd.stalled(A, done)) { raise_error(A, kErrWatchdog); stop = 1; }
      }
      if (wave_bcast(stop, 0)) break;
      // an idle wavefront also writes chunks of the large trades' write jobs
      WriteCounts H{0, 0, 0, 0};
      if (try_help(A, (int32_t)blockIdx.x, H, kHelpRun)) {
        S.fwd += (unsigned long long)wave_sum((int32_t)H.fwd);
        S.emit += (unsigned long long)wave_sum((int32_t)H.emit);
        S.n_push += (unsigned long long)wave_sum((int32_t)H.push);
        backoff = 1;
        continue;
      }
      // sleep, but look at the workgroup's pool between short naps
      for (int32_t i = 0; i < backoff; ++i) {
        __builtin_amdgcn_s_sleep(32);
        if (S.pool && ballot(S.pool[l] >= 0)) break;
      }
      backoff = backoff < A.idle_backoff ? backoff * 2 : A.idle_backoff;
      continue;
    }
    backoff = 1;
    const int32_t u = A.perm[2 * k], v = A.perm[2 * k + 1];
    const int64_t s = (A.rp[u + 1] - A.rp[u]) + (A.rp[v + 1] - A.rp[v]);
    if (s > A.small_max) {
      // large trade: hand it to a workgroup worker
      if (l == 0) {
        publish_wait();
        queue_push(A, A.qb, kCwQbTail0, wid % kQbShards, k);
      }
      continue;
    }
    consume_order();
    const uint64_t t_start = now_ticks();
    small_trade(A, k, u, v, W, S);
    const uint64_t t_end = now_ticks();
    S.ticks += t_end - t_start;
    if (A.trace && l == 0) {
      A.trace[kTraceFields * (int64_t)k + 1] = (int64_t)t_start;
      A.trace[kTraceFields * (int64_t)k + 2] = (int64_t)t_end;
    }
    S.ndone += 1;
    if (S.ndone >= kFlushEvery) wave_flush(A, S);
    int32_t ab = 0;
    if (l == 0) ab = load_agent(&A.ctrl[cw(kCwAbort)]);
    if (wave_bcast(ab, 0)) break;
  }
  wave_flush(A, S);
}

// ============================================================ large trades
// One workgroup per trade. Entries live in LDS when deg u + deg v <= kBigCap,
// otherwise in this workgroup's global scratch slot (bucket sort, with LSD
// radix sort for node ids bunched together).

// Collect one list of trade k (in any order): the round-start neighbours of
// later trades (plus partner and left-out node) from the CSR row, then the
// arrivals from the inbox. Workgroup-wide; false (error raised) on a size
// mismatch.
constexpr int kGatherBatch = 4;   // loads in flight per thread while collecting a list
__device__ __forceinline__ bool gather_list(const TradeArgs& A, int32_t k, int64_t b, int32_t d, int32_t ni,
                            int side, uint64_t* out, BigLds& B) {
  const int tid = threadIdx.x;
  if (tid == 0) B.cnt[0] = 0;
  __syncthreads();
  // one LDS counter update per wavefront and chunk (trip count is uniform
  // across a wavefront: the bound is rounded up to whole wavefronts)
  // kGatherBatch strides of loads are issued before the first is used. The
  // row's inbox slot e is read with row entry e and kept if e < ni; arrivals
  // fill out[] from the back (the j-th at d-1-j).
  const int32_t dr = (d + kWave - 1) / kWave * kWave;
  const int32_t nt = blockDim.x;
  for (int32_t e0 = tid; e0 < dr; e0 += kGatherBatch * nt) {
    int32_t t[kGatherBatch], x[kGatherBatch], y[kGatherBatch];
#pragma unroll
    for (int r = 0; r < kGatherBatch; ++r) {
      const int32_t e = e0 + r * nt;
      t[r] = e < d ? A.col_t[b + e] : 0;
      x[r] = e < d ? A.col[b + e] : 0;
      y[r] = e < d ? load_agent(&A.inbox[b + e]) : 0;
    }
#pragma unroll
    for (int r = 0; r < kGatherBatch; ++r) {
      const int32_t e = e0 + r * nt;
      if (e >= dr) break;   // uniform across a wavefront
      const bool fresh = e < d && tinfo_trade(t[r]) >= k;
      const uint64_t m = ballot(fresh);
      int32_t base = 0;
      if (lane_id() == 0 && m) base = atomicAdd(&B.cnt[0], popc64(m));
      base = wave_bcast(base, 0);
      if (fresh) out[base + rank_below(m)] = make_entry(x[r], side, tag_of(t[r], k));
      if (e < ni && ni <= d) out[d - 1 - e] = make_entry(y[r], side, kTagEmit);
    }
  }
  __syncthreads();
  const int32_t nf = B.cnt[0];
  __syncthreads();
  if (nf + ni != d) {
    if (tid == 0) raise_error(A, kErrGather, k, 1000000 + nf + ni - d);
    return false;
  }
  return true;
}

// Both lists of trade k into out[0..du + dv) in no particular order (the
// caller sorts them): u's and v's row entries whose other end has not traded
// yet, then the arrivals in their inboxes, each as an entry of its side.
// Workgroup-wide; false (error raised) if a row's count does not match.
__device__ __forceinline__ bool gather_both(const TradeArgs& A, int32_t k, int64_t bu, int32_t du, int32_t niu,
                                            int64_t bv, int32_t dv, int32_t niv, uint64_t* out, BigLds& B) {
  const int tid = threadIdx.x;
  const int32_t nt = blockDim.x;
  if (tid == 0) { B.cnt[0] = 0; B.cnt[1] = 0; }
  __syncthreads();
  const int32_t s = du + dv;
  const int32_t sr = (s + kWave - 1) / kWave * kWave;
  // A row's inbox has as many slots as the row; slot e is read with row
  // entry e (one round trip for both) and kept if e is below the row's
  // arrival count. Arrivals fill out[] from the back: u's j-th at s-1-j, v's
  // at s-1-niu-j; row entries of later nodes fill it from the front.
  for (int32_t e0 = tid; e0 < sr; e0 += kGatherBatch * nt) {
    int32_t t[kGatherBatch], x[kGatherBatch], y[kGatherBatch];
#pragma unroll
    for (int r = 0; r < kGatherBatch; ++r) {
      const int32_t e = e0 + r * nt;
      const int64_t at = e < du ? bu + e : bv + (e - du);
      t[r] = e < s ? A.col_t[at] : 0;
      x[r] = e < s ? A.col[at] : 0;
      y[r] = e < s ? load_agent(&A.inbox[at]) : 0;
    }
#pragma unroll
    for (int r = 0; r < kGatherBatch; ++r) {
      const int32_t e = e0 + r * nt;
      if (e >= sr) break;   // uniform across a wavefront
      const int side = e < du ? 0 : 1;
      const bool fresh = e < s && tinfo_trade(t[r]) >= k;
      const uint64_t m = ballot(fresh);
      const uint64_t mu = ballot(fresh && side == 0);
      int32_t base = 0;
      if (lane_id() == 0 && m) {
        base = atomicAdd(&B.cnt[0], popc64(m));
        if (mu) atomicAdd(&B.cnt[1], popc64(mu));
      }
      base = wave_bcast(base, 0);
      if (fresh) out[base + rank_below(m)] = make_entry(x[r], side, tag_of(t[r], k));
      if (e < du) {
        if (e < niu && niu <= du) out[s - 1 - e] = make_entry(y[r], 0, kTagEmit);
      } else if (e < s) {
        if (e - du < niv && niv <= dv) out[s - 1 - niu - (e - du)] = make_entry(y[r], 1, kTagEmit);
      }
    }
  }
  __syncthreads();
  const int32_t nf = B.cnt[0];
  const int32_t nfu = B.cnt[1];
  __syncthreads();
  if (nfu + niu != du || nf - nfu + niv != dv) {
    if (tid == 0) raise_error(A, kErrGather, k, 1000000 + nf + niu + niv - s);
    return false;
  }
  return true;
}

// Write giant gi's neighbour set, ascending, as entries of `side` of trade k
// into out[0..d), and clear its counts for the next round (the write phase
// clears its words).
// Workgroup-wide; false (error raised) if the set does not hold d members.
// Wave w takes 64 superblocks of each block of superblocks, 32 loaded at a
// time, a lane covering 8 words. The members' tags are left unknown: the
// write phase looks each one up when it routes the edge, in parallel.
__device__ __forceinline__ bool extract_giant(const TradeArgs& A, int32_t k, int32_t gi, int side, int32_t d,
                              uint64_t* out, BigLds& B) {
  constexpr int kGroups = 4;   // groups of 8 superblocks loaded per wavefront step
  const int tid = threadIdx.x;
  const int w = tid >> 6;
  const int l = lane_id();
  const int64_t nsb = A.gs.gwords >> 6;
  unsigned long long* bm = A.gs.bm + (int64_t)gi * A.gs.gwords;
  int32_t* sc = A.gs.sc + (int64_t)gi * nsb;
  int32_t carry = 0;
  bool bad = false;
  for (int64_t j0 = 0; j0 < nsb; j0 += blockDim.x) {
    const int64_t j = j0 + tid;
    const int32_t c = j < nsb ? load_agent(&sc[j]) : 0;
    int32_t tot;
    const int32_t pre = block_excl_scan(c, B.scan, &tot);
    B.sboff[tid] = carry + pre;
    B.sbcnt[tid] = c;
    __syncthreads();
    // Lane l covers words 8 * (l % 8) .. + 7 of superblock l / 8 of its
    // group, so one wavefront instruction covers 8 superblocks; a wavefront
    // takes the 64 superblocks w * 64 .. of this block in kGroups groups of 8
    // per step.
    const int seg = l >> 3;           // superblock of this lane within a group
    const int part = l & 7;           // its 8-word part of the superblock
    const int seg0 = l & ~7;          // first lane of the segment
    for (int q = 0; q < kWave; q += 8 * kGroups) {
      unsigned long long word[kGroups][8];
#pragma unroll
      for (int g = 0; g < kGroups; ++g) {
        const int sbi = w * kWave + q + g * 8 + seg;
        const int64_t jj = j0 + sbi;
        const bool valid = jj < nsb && B.sbcnt[sbi] > 0;
#pragma unroll
        for (int i = 0; i < 8; ++i)
          word[g][i] = valid ? load_agent_u64(&bm[jj * kWave + part * 8 + i]) : 0ull;
      }
#pragma unroll
      for (int g = 0; g < kGroups; ++g) {
        const int sbi = w * kWave + q + g * 8 + seg;
        const int64_t jj = j0 + sbi;
        const bool valid = jj < nsb;
        int32_t pc = 0;
#pragma unroll
        for (int i = 0; i < 8; ++i) pc += __popcll(word[g][i]);
        // exclusive prefix of pc inside the 8-lane segment, and its total
        const int32_t incl = wave_incl_scan(pc);
        const int32_t before = __shfl(incl, seg0 > 0 ? seg0 - 1 : 0, kWave);
        const int32_t seg_end = __shfl(incl, seg0 + 7, kWave);
        const int32_t base = seg0 > 0 ? before : 0;
        if (valid && seg_end - base != B.sbcnt[sbi]) bad = true;
        const int32_t at = (valid ? B.sboff[sbi] : 0) + incl - pc - base;
        int32_t idx = 0;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          unsigned long long bits = word[g][i];
          if (!bits) continue;
          const int64_t wi = jj * kWave + part * 8 + i;
          while (bits) {
            const int bit = __builtin_ctzll(bits);
            bits &= bits - 1;
            if (at + idx < d) out[at + idx] = make_entry((int32_t)(wi * 64 + bit), side, kTagUnknown);
            ++idx;
          }
        }
        if (valid && part == 0 && B.sbcnt[sbi] > 0) sc[jj] = 0;
      }
    }
    carry += tot;
    __syncthreads();
  }
  if (tid == 0) B.cnt[1] = 0;
  __syncthreads();
  if (bad) B.cnt[1] = 1;
  __syncthreads();
  const bool ok = B.cnt[1] == 0 && carry == d;
  __syncthreads();
  if (!ok) {
    if (tid == 0) raise_error(A, kErrGather, k, 2000000 + carry - d);
    return false;
  }
  if (tid == 0) B.tick[0] = now_ticks();
  __syncthreads();
  return true;
}

   // items per thread whose atomics are in flight together

constexpr int kPer = 8;     // consecutive entries per thread in the classification scan
// hash slots of the split through LDS (key, count, value, then 2 T + T step
// slots): 3 * 8192 + 6144 ints of the tile's 36864
constexpr int32_t kSplitSlots = 8192;
static_assert(3 * kSplitSlots + 3 * (kSplitSlots / 4) <= kBigCap * 3, "split slots fit the tile");

constexpr int32_t kFastOther = 2048;   // other-side sizes of the one-pass giant classification
// the split of a fused giant pass's items has at most kFastOther steps (the
// small side's disjoint entries), which its hash table must hold four times
static_assert(4 * kFastOther <= kSplitSlots, "item split slots cover the fused pass");
constexpr int kRing = 512;             // nonzero bitmap words buffered per producer / consumer pair
constexpr int kPairs = kWavesPerBlock / 2;
constexpr int kChunkBatch = 8;         // 1 KiB bitmap chunks a producer keeps in flight (twice)
static_assert(kFastOther + 3 * kPairs * kRing + 2 * kPairs <= kBigCap, "fused pass LDS fits the tile");
constexpr int32_t kSlowWord = 0x40000000;   // ring word holding a node of the other side (or its node)
constexpr int kSbRegs = 8;   // superblock counts per thread kept in registers by the fused pass
constexpr int32_t kFusedShareMin = 512;     // members per offered part of a giant's bitmap pass
constexpr int32_t kFusedParts = 16;         // at most this many parts
constexpr int kBufDword3 = 0x00020000; // raw buffer resource: 32-bit format, bounds-checked by bytes
constexpr int kCpolSc1 = 16;           // cache policy: agent-coherent load

// LDS hand-over between two wavefronts of a workgroup: this wavefront's LDS
// writes (and reads) complete before the counter changes; global memory
// operations in flight are not waited for.
__device__ __forceinline__ void lds_publish(int32_t* p, int32_t v) {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0) only
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ int32_t lds_observe(const int32_t* p) {
  const int32_t v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  return v;
}

// Item of the shared write phase for the entry at D position p: the entry
// with the side of its owner (by position among the disjoint ones, by its own
// side among the kept ones).
__device__ __forceinline__ void put_item(unsigned long long* I, int32_t p, uint64_t e, int32_t nD, int32_t a) {
  const uint64_t own = p < nD ? (p < a ? 0ull : 1ull) : (uint64_t)ent_side(e);
  store_agent_u64(&I[p], (e & ~(1ull << 32)) | (own << 32));
}

// Bits of the two words w0 (ids b .. b + 63) and w1 (ids b + 64 ..) below id x.
__device__ __forceinline__ int32_t bits_below(uint64_t w0, uint64_t w1, int32_t b, int32_t x) {
  int32_t c = 0;
  if (x >= b + 64) c += popc64(w0);
  else if (x > b) c += popc64(w0 & ((1ull << (x - b)) - 1ull));
  if (x >= b + 128) c += popc64(w1);
  else if (x > b + 64) c += popc64(w1 & ((1ull << (x - b - 64)) - 1ull));
  return c;
}

// Parameters of the producer / consumer phase of a fused giant pass, the
// same for the owner and for a helper workgroup that takes part of the
// bitmap; O, kc and Kk are in the workgroup's LDS at the fixed places.
struct FusedCtx {
  const unsigned long long* bm;   // the giant's bitmap
  const int32_t* pre;             // prefix of its superblock counts (agent-scope)
  unsigned long long* I;          // items, or null: E and D
  uint64_t* E;
  int32_t* D;
  int64_t gwords;
  int32_t k, sh, d_g, d_o, nK1, s, nD, a, o;
  bool edge;
  bool trace;                     // record trade k's trace fields of the phase
};

// The producer / consumer phase of a fused giant pass over the superblocks
// [sb_from, sb_to) (sb_from even). Workgroup-wide; false if the members
// found do not match the superblock counts.
__device__ __forceinline__ bool fused_roles(const TradeArgs& A, BigLds& B, const FusedCtx& C, int64_t sb_from,
                                            int64_t sb_to) {
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  const int w = tid >> 6;
  const int l = lane_id();
  const int np = (nt >> 6) >> 1;               // producer wavefronts; as many consume
  const int32_t k = C.k, sh = C.sh, so = 1 - C.sh, d_g = C.d_g, d_o = C.d_o, nK1 = C.nK1, s = C.s;
  const int32_t nD = C.nD, a = C.a, o = C.o;
  const bool edge = C.edge;
  const uint64_t kgp = ((uint64_t)o << 1) | (uint64_t)sh;   // key of the giant's partner entry
  const unsigned long long* bm = C.bm;
  const int64_t gwords = C.gwords;
  unsigned long long* I = C.I;
  uint64_t* E = C.E;
  int32_t* D = C.D;
  const bool items_only = I != nullptr;
  const uint64_t* O = B.u.tile.E;
  const int32_t* kc = B.u.tile.D + kFastOther;
  const uint64_t* Kk = reinterpret_cast<const uint64_t*>(B.u.tile.D + 2 * kFastOther);
  const int pair = w < np ? w : w - np;
  uint64_t* ringW = B.u.tile.E + kFastOther + pair * kRing;
  int4* ringM = reinterpret_cast<int4*>(B.u.tile.E + kFastOther + kPairs * kRing) + pair * kRing;
  auto ring_ctr = [&](int q) {
    return reinterpret_cast<int32_t*>(B.u.tile.E + kFastOther + 3 * kPairs * kRing) + 4 * q;
  };
  int32_t* rc = ring_ctr(pair);
  if (tid == 0) B.cnt[2] = 0;
  if (w < np && l < 4) rc[l] = 0;   // fill, head, done, finished wavefronts (trace)
  __syncthreads();
  const int64_t span = sb_to - sb_from;
  const int64_t R = (((span + np - 1) / np) + 1) & ~(int64_t)1;
  const int64_t sb_lo = sb_from + ((int64_t)pair * R < span ? (int64_t)pair * R : span);
  const int64_t sb_hi = sb_lo + R < sb_to ? sb_lo + R : sb_to;
  int32_t run = load_agent(&C.pre[sb_lo]);
  // trace: the last producer and the last consumer to finish record the time
  auto trace_finish = [&](int q, int field) {
    int32_t* f = ring_ctr(q) + 3;
    if (C.trace && A.trace && l == 0 && atomicAdd(f, 1) == np - 1)
      A.trace[kTraceFields * (int64_t)k + field] = (int64_t)now_ticks();
  };
  if (w < np) {
    // ---- producer
    const int32_t run0 = run;
    const int32_t nchunks = (int32_t)((sb_hi - sb_lo + 1) >> 1);
    const int32_t wbase = (int32_t)(sb_lo * 64);   // first word of the range
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void*)bm, (short)0, (int)(gwords * 8), kBufDword3);
    // O and kept entries below the current chunk, next node of O or o at or
    // after it (all uniform across the wavefront)
    const uint32_t id_lo = (uint32_t)wbase * 64u;
    int32_t ro = 0, rk = 0;
    {
      int32_t lo = 0, hi = d_o;
      while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if ((uint32_t)ent_node(O[mid]) < id_lo) lo = mid + 1; else hi = mid;
      }
      ro = lo;
      lo = 0;
      hi = nK1;
      while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (Kk[mid] < ((uint64_t)id_lo << 1)) lo = mid + 1; else hi = mid;
      }
      rk = lo;
    }
    auto next_special = [&](uint32_t from) -> uint32_t {
      uint32_t sp = ro < d_o ? (uint32_t)ent_node(O[ro]) : 0xFFFFFFFFu;
      if ((uint32_t)o >= from && (uint32_t)o < sp) sp = (uint32_t)o;
      return sp;
    };
    uint32_t sp = next_special(id_lo);
    int32_t fill = 0, head_seen = 0;
    int32_t spins = 0;   // trace: waits for ring space
    // lane l holds words 2 l and 2 l + 1 of a chunk (sc1 loads: the words
    // were set by other workgroups' atomics; past the bitmap they read 0)
    auto load_batch = [&](uint4* v, int32_t c0) {
#pragma unroll
      for (int b = 0; b < kChunkBatch; ++b)
        v[b] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(
                                             rs, (wbase + 128 * (c0 + b) + 2 * l) * 8, 0, kCpolSc1));
    };
    // two register sets in turn, each batch loaded a batch ahead; the loads
    // are unconditional (one batch past the range is read and dropped)
    auto process = [&](const uint4* v, int32_t c0) {
#pragma unroll
      for (int b = 0; b < kChunkBatch; ++b) {
        const int32_t ch = c0 + b;
        if (ch >= nchunks) break;
        const int32_t wb = wbase + 128 * ch;
        const uint32_t id0 = (uint32_t)wb * 64u;
        const uint32_t id_end = id0 + 128u * 64u;
        const bool slow = sp < id_end;
        const uint64_t w0 = ((uint64_t)v[b].y << 32) | v[b].x;
        const uint64_t w1 = ((uint64_t)v[b].w << 32) | v[b].z;
        const int32_t pc = popc64(w0) + popc64(w1);
        const int32_t nzc = (w0 != 0ull ? 1 : 0) + (w1 != 0ull ? 1 : 0);
        const int32_t pk = pc | (nzc << 16);
        const int32_t incl = wave_incl_scan(pk);
        const int32_t tot = wave_bcast(incl, kWave - 1);
        const int32_t ex = incl - pk;
        // per word: O entries and kept keys below its first id; a word that
        // holds a node of O or o itself is expanded with a short scan
        const uint32_t b0 = id0 + 128u * (uint32_t)l, b1 = b0 + 64u;
        const int32_t e0 = (edge && (uint32_t)o < b0) ? 1 : 0;
        const int32_t e1 = (edge && (uint32_t)o < b1) ? 1 : 0;
        int32_t ro0 = ro, ro1 = ro, rk0 = rk, rk1 = rk;
        bool s0 = false, s1 = false;
        if (slow) {
          // ranks of the O nodes in this chunk among the giant's members
          while (ro < d_o && (uint32_t)ent_node(O[ro]) < id_end) {
            const int32_t x = ent_node(O[ro]);
            const int32_t kx = kc[ro];
            if ((uint32_t)x < b0) { ++ro0; rk0 += kx; }
            if ((uint32_t)x < b1) { ++ro1; rk1 += kx; }
            s0 |= (uint32_t)x >= b0 && (uint32_t)x < b1;
            s1 |= (uint32_t)x >= b1 && (uint32_t)x < b1 + 64u;
            ++ro;
          }
          s0 |= (uint32_t)o >= b0 && (uint32_t)o < b1;
          s1 |= (uint32_t)o >= b1 && (uint32_t)o < b1 + 64u;
        }
        const int32_t add = tot >> 16;
        if (add != 0) {
          if (fill + add - head_seen > kRing) {
            lds_publish(&rc[0], fill);   // all written entries visible before waiting
            while (true) {
              head_seen = lds_observe(&rc[1]);
              if (fill + add - head_seen <= kRing) break;
              __builtin_amdgcn_s_sleep(1);
              ++spins;
            }
          }
          int32_t at = fill + (ex >> 16);
          const int32_t r0 = run + (ex & 0xFFFF);
          if (w0) {
            ringW[at & (kRing - 1)] = w0;
            ringM[at & (kRing - 1)] =
                make_int4(r0, wb + 2 * l, s0 ? (ro0 | kSlowWord) : ro0, s0 ? rk0 : rk0 + e0);
            ++at;
          }
          if (w1) {
            ringW[at & (kRing - 1)] = w1;
            ringM[at & (kRing - 1)] = make_int4(r0 + popc64(w0), wb + 2 * l + 1,
                                                s1 ? (ro1 | kSlowWord) : ro1, s1 ? rk1 : rk1 + e1);
          }
          fill += add;
        }
        run += tot & 0xFFFF;
        if (slow) {
          while (rk < nK1 && Kk[rk] < ((uint64_t)id_end << 1)) ++rk;
          sp = next_special(id_end);
        }
      }
      lds_publish(&rc[0], fill);
    };
    uint4 va[kChunkBatch], vb[kChunkBatch];
    load_batch(va, 0);
    for (int32_t c0 = 0;;) {
      load_batch(vb, c0 + kChunkBatch);
      process(va, c0);
      c0 += kChunkBatch;
      if (c0 >= nchunks) break;
      load_batch(va, c0 + kChunkBatch);
      process(vb, c0);
      c0 += kChunkBatch;
      if (c0 >= nchunks) break;
    }
    lds_publish(&rc[0], fill);
    lds_publish(&rc[2], 1);
    // the members found must match the superblock counts of the range
    if (l == 0 && run - run0 != load_agent(&C.pre[sb_hi]) - load_agent(&C.pre[sb_lo])) B.cnt[2] = 1;
    trace_finish(0, 20);
    if (A.trace && l == 0) atomicAdd(ring_ctr(2) + 3, spins);
  } else {
    // ---- consumer: members of one ring word: rank of its lowest bit, word
    // index, O entries below the word (with kSlowWord: the word holds one of
    // the special nodes), kept entries below it
    int32_t head = 0, fill_seen = 0;
    int32_t spins = 0;   // trace: waits for ring entries
    while (true) {
      if (fill_seen - head < kWave) {
        const int32_t dn = lds_observe(&rc[2]);
        fill_seen = lds_observe(&rc[0]);
        if (fill_seen - head < kWave && dn == 0) {
          __builtin_amdgcn_s_sleep(1);
          ++spins;
          continue;
        }
      }
      int32_t cnt = fill_seen - head;
      if (cnt == 0) break;
      if (cnt > kWave) cnt = kWave;
      if (l < cnt) {
        const int32_t p = (head + l) & (kRing - 1);
        uint64_t bits = ringW[p];
        const int4 m = ringM[p];
        int32_t r = m.x;
        while (bits) {
          const int bit = __builtin_ctzll(bits);
          bits &= bits - 1ull;
          const int32_t x = m.y * 64 + bit;
          const int32_t i = r++;
          if (i >= d_g) continue;
          const uint64_t e = make_entry(x, sh, kTagUnknown);
          int32_t pe, pd;
          if (!(m.z & kSlowWord)) {
            pe = i + m.z;
            pd = pe - m.w;
          } else {
            // from the word's counts past the few O entries and kept keys below this member
            const uint64_t key = e >> 32;
            int32_t rO = m.z & ~kSlowWord;
            while (rO < d_o && (O[rO] >> 32) < key) ++rO;
            int32_t rK = m.w;
            while (rK < nK1 && Kk[rK] < key) ++rK;
            const bool common =
                sh < so ? (rO < d_o && ent_node(O[rO]) == x) : (rO > 0 && ent_node(O[rO - 1]) == x);
            pe = i + rO;
            const int32_t rkt = rK + ((edge && kgp < key) ? 1 : 0);
            pd = (common || x == o) ? s - 1 - rkt : pe - rkt;
          }
          if (items_only) {
            put_item(I, pd, e, nD, a);
          } else {
            E[pe] = e;
            D[pd] = pe;
          }
        }
      }
      head += cnt;
      lds_publish(&rc[1], head);
    }
    trace_finish(1, 21);
    if (A.trace && l == 0) atomicAdd(ring_ctr(3) + 3, spins);
  }
  __syncthreads();
  if (C.trace && A.trace && tid == 0) {
    A.trace[kTraceFields * (int64_t)k + 22] = *(ring_ctr(2) + 3);
    A.trace[kTraceFields * (int64_t)k + 23] = *(ring_ctr(3) + 3);
  }
  const bool ok = B.cnt[2] == 0;
  __syncthreads();
  return ok;
}

// One giant side (node h, side sh, d_g members in giant gi's bitmap) and a
// small other side O (ascending in LDS, d_o <= kFastOther entries, node o):
// the merged list E and the disjoint / kept index array D in one pass over
// the bitmap, without materialising the giant's sorted list.
//
// A member's merged position is its rank among the giant's members plus the
// O entries below it; its disjoint position is that minus the kept entries
// below it (kept ones fill D from the back by the same count). The kept
// entries follow from O alone: a shared neighbour x gives the keys (x, 0) and
// (x, 1), the partner edge gives O's entry for h and the giant's for o. So
// within a bitmap word that holds no node of O and not o both counts are
// constant; the producer works them out per word (per chunk of 128 words
// (8192 ids) when the chunk holds none of those nodes), and only the members
// of the few words that do hold one scan on from the word's counts.
//
// Half of the wavefronts produce, half consume, in pairs (fused_roles). A
// producer streams a contiguous range of superblocks (starting at the prefix
// of the superblock counts before it) with wide loads kept in flight a batch
// ahead, and compacts the nonzero words into its pair's LDS ring; it never
// stores to global memory, so its waits for loads never wait for stores. Its
// consumer expands the ring one word per lane and writes the entries. The
// two synchronise through LDS counters only. The ranks of O's nodes among
// the members (the prefix of their superblock plus the members below them in
// it) are worked out first, so O's entries are written before the members.
//
// If I is not null (a shared write phase), only the items are written, at the
// positions before the split (the caller applies the split to them), and a
// large giant offers all but the first of its superblock parts to idle
// workgroups (fused_help), taking back any part nobody claimed. Otherwise E
// and D are written. Clears the superblock counts of the bitmap; its words
// are cleared when the edges are written. Workgroup-wide; sets *nD and *a in
// every thread, and *split_done when only the items were written. False
// (error raised) if the bitmap does not hold d_g members.
__device__ __forceinline__ bool giant_fused(const TradeArgs& A, int32_t k, int32_t gi, int sh, int32_t d_g,
                                            int32_t h, int32_t o, int32_t d_o, BigLds& B, uint64_t* E,
                                            int32_t* D, int32_t s, int32_t* nD_out, int32_t* a_out,
                                            unsigned long long* I, bool* split_done) {
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  const int w = tid >> 6;
  const int l = lane_id();
  const int np = (nt >> 6) >> 1;               // producer wavefronts; as many consume
  const int so = 1 - sh;
  const uint64_t* O = B.u.tile.E;
  int32_t* posO = B.u.tile.D;                  // merged position of O[j]
  int32_t* kc = B.u.tile.D + kFastOther;       // kept entries O[j] stands for (0, 1 or 2)
  uint64_t* Kk = reinterpret_cast<uint64_t*>(B.u.tile.D + 2 * kFastOther);   // kept keys from O
  const int64_t gwords = A.gs.gwords;
  const int64_t nsb = gwords >> 6;
  const unsigned long long* bm = A.gs.bm + (int64_t)gi * gwords;
  int32_t* sc = A.gs.sc + (int64_t)gi * nsb;
  // superblock counts: a contiguous run per thread, loaded now (their
  // latency overlaps the probes of O below) and kept in registers when the
  // run is short enough
  const int64_t per = (nsb + nt - 1) / nt;
  const int64_t j0s = (int64_t)tid * per < nsb ? (int64_t)tid * per : nsb;
  const int64_t j1s = j0s + per < nsb ? j0s + per : nsb;
  const bool inreg = per <= kSbRegs;   // uniform
  int32_t cv[kSbRegs];
#pragma unroll
  for (int i = 0; i < kSbRegs; ++i) cv[i] = inreg && j0s + i < j1s ? load_agent(&sc[j0s + i]) : 0;
  if (tid == 0) { B.cnt[0] = 0; B.cnt[1] = 0; B.cnt[2] = 0; }
  __syncthreads();
  // O entries, from the words of their superblock up to their own (8 lanes,
  // 8 words each; these loads overlap those of the counts above): the
  // giant's members below them (posO, the prefix of the superblock is added
  // below) and whether they are shared neighbours (their bit set in the
  // giant's set) or the partner
  for (int32_t j0 = w * 8; j0 < d_o; j0 += (nt >> 6) * 8) {
    const int32_t j = j0 + (l >> 3);
    int32_t c = 0, mem = 0;
    if (j < d_o) {
      const int32_t x = ent_node(O[j]);
      const int64_t wb = (int64_t)(x >> 12) * 64 + (l & 7) * 8;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int64_t wi = wb + i;
        const int32_t below = x - (int32_t)(wi * 64);   // bits of word wi below x
        if (below >= 0) {
          const uint64_t word = load_agent_u64(&bm[wi]);
          c += below >= 64 ? popc64(word) : popc64(word & ((1ull << below) - 1ull));
          if (below < 64) mem = (int32_t)((word >> below) & 1ull);
        }
      }
    }
    c += __shfl_xor(c, 1, kWave);
    c += __shfl_xor(c, 2, kWave);
    c += __shfl_xor(c, 4, kWave);
    mem |= __shfl_xor(mem, 1, kWave);
    mem |= __shfl_xor(mem, 2, kWave);
    mem |= __shfl_xor(mem, 4, kWave);
    if (j < d_o && (l & 7) == 0) {
      const bool partner = ent_node(O[j]) == h;
      posO[j] = c;
      kc[j] = mem ? 2 : (partner ? 1 : 0);
      if (mem) atomicAdd(&B.cnt[0], 1);
      if (partner) B.cnt[1] = 1;
    }
  }
  __syncthreads();
  int32_t nK1 = 0;
  for (int32_t j0 = 0; j0 < d_o; j0 += nt) {
    const int32_t j = j0 + tid;
    const int32_t c = j < d_o ? kc[j] : 0;
    int32_t tot;
    const int32_t p = nK1 + block_excl_scan(c, B.scan, &tot);
    if (c == 2) {
      const uint64_t kx0 = (uint64_t)ent_node(O[j]) << 1;
      Kk[p] = kx0;
      Kk[p + 1] = kx0 | 1ull;
    } else if (c == 1) {
      Kk[p] = O[j] >> 32;
    }
    nK1 += tot;
  }
  // prefix of the superblock counts (cleared as they are read); each
  // producer takes an even number of superblocks (whole chunks)
  int32_t* pre = A.sbpre + (int64_t)blockIdx.x * A.sbpre_stride;
  // a copy in LDS, for the ranks of O's nodes below, in the ring space (not
  // in use until the roles start) when it fits
  int32_t* preL = reinterpret_cast<int32_t*>(B.u.tile.E + kFastOther);
  const bool pre_lds = nsb <= 2 * (int64_t)(kBigCap - kFastOther);
  int32_t total;
  {
    int32_t sum = 0;
    if (inreg) {
#pragma unroll
      for (int i = 0; i < kSbRegs; ++i) sum += cv[i];
    } else {
      for (int64_t j = j0s; j < j1s; ++j) sum += load_agent(&sc[j]);
    }
    int32_t at = block_excl_scan(sum, B.scan, &total);
    if (inreg) {
#pragma unroll
      for (int i = 0; i < kSbRegs; ++i) {
        if (j0s + i < j1s) {
          store_agent(&pre[j0s + i], at);
          if (pre_lds) preL[j0s + i] = at;
          at += cv[i];
          if (cv[i] != 0) sc[j0s + i] = 0;
        }
      }
    } else {
      for (int64_t j = j0s; j < j1s; ++j) {
        const int32_t c = load_agent(&sc[j]);
        store_agent(&pre[j], at);
        if (pre_lds) preL[j] = at;
        at += c;
        if (c != 0) sc[j] = 0;
      }
    }
    if (tid == 0) store_agent(&pre[nsb], total);
  }
  __syncthreads();
  // ranks of O's nodes among the giant's members: the prefix of their
  // superblock plus the members below them in it (counted above)
  for (int32_t j = tid; j < d_o; j += nt) {
    const int32_t x = ent_node(O[j]);
    posO[j] = j + (pre_lds ? preL[x >> 12] : load_agent(&pre[x >> 12])) + posO[j] +
              ((kc[j] == 2 && sh < so) ? 1 : 0);
  }
  __syncthreads();   // posO is read by other wavefronts below
  const int32_t n_common = B.cnt[0];
  const bool edge = B.cnt[1] != 0;
  const uint64_t kgp = ((uint64_t)o << 1) | (uint64_t)sh;   // key of the giant's partner entry
  const int32_t nD = s - nK1 - (edge ? 1 : 0);
  const int32_t a = (sh == 0 ? d_g : d_o) - n_common - (edge ? 1 : 0);
  if (total != d_g) {
    __syncthreads();
    if (tid == 0) raise_error(A, kErrGather, k, 2000000 + total - d_g);
    return false;
  }
  // with items (a shared write phase), only the items are written: the
  // split is applied to them afterwards; the other side's entries first
  const bool items_only = I != nullptr;
  for (int32_t j = tid; j < d_o; j += nt) {
    const uint64_t e = O[j];
    const uint64_t key = e >> 32;
    int32_t lo = 0, hi = nK1;
    while (lo < hi) {
      const int32_t mid = (lo + hi) >> 1;
      if (Kk[mid] < key) lo = mid + 1; else hi = mid;
    }
    const int32_t rkt = lo + ((edge && kgp < key) ? 1 : 0);
    const int32_t pe = posO[j];
    const int32_t pd = kc[j] ? s - 1 - rkt : pe - rkt;
    if (items_only) {
      put_item(I, pd, e, nD, a);
    } else {
      E[pe] = e;
      D[pd] = pe;
    }
  }
  if (A.trace && tid == 0) A.trace[kTraceFields * (int64_t)k + 15] = (int64_t)now_ticks();
  FusedCtx C{bm, pre, I, E, D, gwords, k, sh, d_g, d_o, nK1, s, nD, a, o, edge, true};
  // a large giant with a shared write phase offers all but the first of
  // its parts (one per kFusedShareMin members, at most kFusedParts) to idle
  // workgroups: the other side's entries, flags and kept keys go to the
  // (otherwise unused) entry region of the slot
  const int32_t parts = d_g / kFusedShareMin < kFusedParts ? d_g / kFusedShareMin : kFusedParts;
  const bool offer = items_only && parts >= 2 && nsb >= 2 * parts && (int)blockIdx.x < kMaxJobs;
  const int64_t step = offer ? (((nsb / parts) + 1) & ~(int64_t)1) : nsb;   // superblocks per part
  const int32_t noff = offer ? (int32_t)((nsb + step - 1) / step) - 1 : 0;   // parts offered
  HelpJob* Jf = A.jobs + kMaxJobs + blockIdx.x;
  if (offer) {
    unsigned long long* Pub = reinterpret_cast<unsigned long long*>(E);
    for (int32_t j = tid; j < d_o; j += nt) {
      store_agent_u64(&Pub[j], O[j]);
      store_agent(reinterpret_cast<int32_t*>(Pub + d_o + nK1) + j, kc[j]);
    }
    for (int32_t j = tid; j < nK1; j += nt) store_agent_u64(&Pub[d_o + j], Kk[j]);
    if (tid == 0) {
      store_agent(&Jf->f.k, k);
      store_agent(&Jf->f.gi, gi);
      store_agent(&Jf->f.side, sh);
      store_agent(&Jf->f.d, d_g);
      store_agent(&Jf->f.d_o, d_o);
      store_agent(&Jf->f.nK1, nK1);
      store_agent(&Jf->f.s, s);
      store_agent(&Jf->f.nD, nD);
      store_agent(&Jf->f.a, a);
      store_agent(&Jf->f.o, o);
      store_agent(&Jf->f.edge, edge ? 1 : 0);
      store_agent64(&Jf->f.sb_from, step);
      store_agent64(&Jf->f.sb_to, nsb);
      store_agent(&Jf->f.phase, 3);
    }
    publish_wait();
    __syncthreads();
    if (tid == 0) open_job(A, Jf, noff, kCwJobMask2);
  }
  bool ok = fused_roles(A, B, C, 0, step < nsb ? step : nsb);
  if (offer) {
    // parts nobody took yet are done here
    C.trace = false;
    while (true) {
      if (tid == 0) B.next = claim_chunk(Jf);
      __syncthreads();
      const int32_t c = B.next;
      __syncthreads();
      if (c < 0) break;
      const int64_t from = (c + 1) * step;
      ok = fused_roles(A, B, C, from, from + step < nsb ? from + step : nsb) && ok;
      publish_wait();
      __syncthreads();
      if (tid == 0) atomic_add(&Jf->c.done, 1);
    }
    if (tid == 0) close_job(A, Jf, noff, kCwJobMask2);
    __syncthreads();
  }
  if (!ok) {
    if (tid == 0) raise_error(A, kErrGather, k, 3000000);
    return false;
  }
  if (tid == 0) B.tick[0] = now_ticks();
  if (items_only) publish_wait();   // the items are gathered by other wavefronts next
  __syncthreads();
  *nD_out = nD;
  *a_out = a;
  *split_done = items_only;
  return true;
}

// An idle workgroup's part of owner j's giant bitmap pass (phase 3 of the
// second set of jobs, chunk c claimed: part c + 1): the other side, its flags and
// kept keys from j's slot into this workgroup's LDS, then the producer /
// consumer phase over the offered superblocks, writing into j's items.
__device__ __forceinline__ void fused_help(const TradeArgs& A, BigLds& B, int32_t j, int32_t c) {
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  HelpJob* J = A.jobs + kMaxJobs + j;
  consume_order();
  const int32_t k = load_agent(&J->f.k), gi = load_agent(&J->f.gi), sh = load_agent(&J->f.side);
  const int32_t d_g = load_agent(&J->f.d), d_o = load_agent(&J->f.d_o), nK1 = load_agent(&J->f.nK1);
  const int32_t s = load_agent(&J->f.s), nD = load_agent(&J->f.nD), a = load_agent(&J->f.a);
  const int32_t o = load_agent(&J->f.o), edge = load_agent(&J->f.edge);
  const int64_t step = load_agent64(&J->f.sb_from), nsb = load_agent64(&J->f.sb_to);
  const int64_t sb_from = (c + 1) * step, sb_to = sb_from + step < nsb ? sb_from + step : nsb;
  uint64_t* slot = A.slots + (int64_t)j * A.slot_elems;
  const unsigned long long* Pub = reinterpret_cast<const unsigned long long*>(slot);
  int32_t* kc = B.u.tile.D + kFastOther;
  uint64_t* Kk = reinterpret_cast<uint64_t*>(B.u.tile.D + 2 * kFastOther);
  for (int32_t i = tid; i < d_o; i += nt) {
    B.u.tile.E[i] = load_agent_u64(&Pub[i]);
    kc[i] = load_agent(reinterpret_cast<const int32_t*>(Pub + d_o + nK1) + i);
  }
  for (int32_t i = tid; i < nK1; i += nt) Kk[i] = load_agent_u64(&Pub[d_o + i]);
  __syncthreads();
  const int64_t gwords = A.gs.gwords;
  FusedCtx C{A.gs.bm + (int64_t)gi * gwords, A.sbpre + (int64_t)j * A.sbpre_stride,
             reinterpret_cast<unsigned long long*>(slot + shared_list_off(A)), nullptr, nullptr, gwords,
             k, sh, d_g, d_o, nK1, s, nD, a, o, edge != 0, false};
  const bool ok = fused_roles(A, B, C, sb_from, sb_to);
  publish_wait();   // the items are complete before the owner hears of it
  __syncthreads();
  if (tid == 0) {
    if (!ok) raise_error(A, kErrGather, k, 5000000);
    atomic_add(&J->c.done, 1);
  }
}

// Items at the positions the split touched (its windows and its partners),
// rewritten from the split disjoint array. Workgroup-wide.
__device__ __forceinline__ void split_fix_items(const uint64_t* E, const int32_t* D, int32_t nD, int32_t a,
                                                uint64_t seed, uint32_t round, int32_t k,
                                                unsigned long long* I) {
  const int32_t T = split_steps(nD, a);
  const bool fwd = a <= nD - a;
  for (int32_t t = threadIdx.x; t < T; t += blockDim.x) {
    const int32_t j = fwd ? t : nD - 1 - t;
    const int32_t r = split_partner(nD, a, t, seed, round, k);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int32_t p = q ? r : j;
      const uint64_t e = E[D[p]];
      store_agent_u64(&I[p], (e & ~(1ull << 32)) | ((p < a ? 0ull : 1ull) << 32));
    }
  }
}

__device__ __forceinline__ void big_trade(const TradeArgs& A, int32_t k, BigLds& B, uint64_t* slot,
                          unsigned long long* counters) {
  const uint64_t t_begin = now_ticks();
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  const int32_t u = A.perm[2 * k], v = A.perm[2 * k + 1];
  const int64_t bu = A.rp[u], bv = A.rp[v];
  const int32_t du = (int32_t)(A.rp[u + 1] - bu), dv = (int32_t)(A.rp[v + 1] - bv);
  const int32_t s = du + dv;
  if ((int64_t)s > A.smax) {
    if (tid == 0) raise_error(A, kErrCapacity);
    return;
  }
  const int32_t gu = A.gs.giant_id[u], gv = A.gs.giant_id[v];
  const bool giant = gu >= 0 || gv >= 0;
  const bool in_lds = !giant && s <= A.big_lds_max;
  uint64_t* E = in_lds ? B.u.tile.E : slot;
  int32_t* D = in_lds ? B.u.tile.D : (int32_t*)(slot + 2 * A.smax);
  const int32_t niu = load_agent(&A.inbox_cur[u]);
  const int32_t niv = load_agent(&A.inbox_cur[v]);
  uint64_t t_lists = 0;
  int32_t nD = 0, a = 0;
  bool classified = false;   // E and D already built by the one-pass giant path
  bool items_ready = false;  // ... and the shared write phase's items too
  bool items_only = false;   // ... only those (the split is applied to them)
  const bool share = A.help_min > 0 && s >= A.help_min && (int)blockIdx.x < kMaxJobs;
  unsigned long long* Ig = reinterpret_cast<unsigned long long*>(slot + shared_list_off(A));
  if (tid == 0) B.tick[0] = 0;

  if (giant) {
    // Both lists sorted separately (a giant's straight from its bitmap, a
    // small other side in LDS), then merged into the slot. The larger giant
    // side is extracted together with idle helper wavefronts into the shared
    // list of the slot.
    uint64_t* L2 = slot + A.smax;   // lists kept by this workgroup: u's at [0, du), v's at [du, s)
    const unsigned long long* X = reinterpret_cast<const unsigned long long*>(slot + shared_list_off(A));
    int xside = -1, lds_side = -1;
    if (kSharedExtraction && A.help_min > 0 && (int)blockIdx.x < kMaxJobs) {
      if (gu >= 0 && (gv < 0 || du >= dv)) xside = 0;
      else if (gv >= 0) xside = 1;
      if (xside >= 0 && (xside ? dv : du) < A.help_min) xside = -1;
    }
    // exactly one giant side and a small other side: one fused pass
    const int gside = gu >= 0 ? 0 : 1;
    const bool fused = (gu >= 0) != (gv >= 0) && xside < 0 && (gside ? du : dv) <= kFastOther;
    for (int side = 0; side < 2; ++side) {
      const int32_t gi = side ? gv : gu;
      const int32_t d = side ? dv : du;
      const int32_t off = side ? du : 0;
      if (fused && side == gside) continue;
      if (side == xside) {
        if (!extract_giant_shared(A, k, gi, side, d, B)) return;
      } else if (gi >= 0) {
        if (!extract_giant(A, k, gi, side, d, L2 + off, B)) return;
      } else if (d <= kBigCap) {
        if (!gather_list(A, k, side ? bv : bu, d, side ? niv : niu, side, B.u.tile.E, B)) return;
        lds_u64* le = (lds_u64*)B.u.tile.E;
        if (2 * d > kBigCap + kBigCap / 2 ||
            !bucket_sort_lds(le, le + d, le, d, A.keybits, bucket_bits(d, A.keybits, kBucketLdsBits),
                             (lds_i32*)B.bkt, (lds_i32*)B.scan, (lds_i32*)&B.bflag))
          block_bitonic_sort(B.u.tile.E, (uint32_t)d);
        lds_side = side;
      } else {
        // the other node is too large for LDS (giant degree set above kBigCap)
        if (!gather_list(A, k, side ? bv : bu, d, side ? niv : niu, side, L2 + off, B)) return;
        __syncthreads();
        const uint64_t* sorted = block_radix_sort<uint64_t>(L2 + off, E, d, A.keybits, B.u.R);
        if (sorted != L2 + off)
          for (int32_t i = tid; i < d; i += nt) L2[off + i] = sorted[i];
      }
      __syncthreads();
    }
    t_lists = now_ticks();
    if (fused) {
      if (!giant_fused(A, k, gside ? gv : gu, gside, gside ? dv : du, gside ? v : u, gside ? u : v,
                       gside ? du : dv, B, E, D, s, &nD, &a, share ? Ig : nullptr, &items_only))
        return;
      classified = true;
      items_ready = share;
    }
    auto list_at = [&](int sd, int32_t i) -> uint64_t {
      if (sd == lds_side) return B.u.tile.E[i];
      if (sd == xside) return load_agent_u64(&X[i]);
      return L2[(sd ? du : 0) + i];
    };
    // position in the merged list = own index + members of the other list below
    for (int32_t i = tid; i < (classified ? 0 : s); i += nt) {
      const int sd = i < du ? 0 : 1;
      const int32_t idx = sd ? i - du : i;
      const uint64_t e = list_at(sd, idx);
      int32_t lo = 0, hi = sd ? du : dv;
      while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (list_at(1 - sd, mid) < e) lo = mid + 1; else hi = mid;
      }
      E[idx + lo] = e;
    }
    __syncthreads();
  } else {
    if (!gather_both(A, k, bu, du, niu, bv, dv, niv, E, B)) return;
    t_lists = now_ticks();
    // Bucket sort: its buffer follows the entries in LDS while both fit in
    // the tile (the index array is not used yet), else it is in the slot and
    // read back through LDS windows.
    // If a bucket is too full (node ids bunched together), LSD radix sort:
    // LDS ping-pong when both halves fit, else through the slot; the digit
    // counters live in the (not yet used) LDS index array.
    const int lb = bucket_bits(s, A.keybits, in_lds ? kBucketLdsBits : kBucketTileBits);
    lds_i32* bscan = (lds_i32*)B.scan;
    lds_i32* bflag = (lds_i32*)&B.bflag;
    bool bsorted;
    if (in_lds && 2 * s <= kBigCap + kBigCap / 2) {
      lds_u64* le = (lds_u64*)B.u.tile.E;
      bsorted = bucket_sort_lds(le, le + s, le, s, A.keybits, lb, (lds_i32*)B.bkt, bscan, bflag);
    } else if (in_lds) {
      // staged through the index array (kBigCap / 2 entries)
      bsorted = bucket_sort_staged(E, slot, E, s, A.keybits, lb, (lds_i32*)B.bkt, bscan, bflag,
                                   (lds_u64*)B.u.tile.D, kBigCap / 2);
    } else {
      // counters in the index array, staged through the entry array
      bsorted = bucket_sort_staged(E, slot + A.smax, E, s, A.keybits, lb, (lds_i32*)B.u.tile.D, bscan,
                                   bflag, (lds_u64*)B.u.tile.E, kBigCap);
    }
    if (bsorted) {
      // sorted in place
    } else if (in_lds && s <= kBigCap / 2)
      E = seg_radix_sort(E, E + kBigCap / 2, s, A.keybits, B.u.tile.D, B.scan);
    else if (in_lds)
      E = seg_radix_sort(E, slot, s, A.keybits, B.u.tile.D, B.scan);
    else
      E = seg_radix_sort(E, slot + A.smax, s, A.keybits, B.u.tile.D, B.scan);
    __syncthreads();
  }

  const uint64_t t_gathered = now_ticks();
  // ---- classify: disjoint entries go to D[0..nD) in ascending order, kept
  // ones (shared neighbours, partner) to D[nD..s) from the back; a = entries
  // of u among the disjoint ones. Each thread takes kPer consecutive
  // entries, so one workgroup scan covers kPer * blockDim entries.
  for (int32_t c = 0; c < (classified ? 0 : s); c += nt * kPer) {
    const int32_t i0 = c + tid * kPer;
    int32_t nodes[kPer + 2];
    uint32_t meta[kPer];   // bit 0: the partner, bit 1: side
#pragma unroll
    for (int r = 0; r < kPer + 2; ++r) {
      const int32_t i = i0 - 1 + r;
      nodes[r] = (i >= 0 && i < s) ? ent_node(E[i]) : -1;
    }
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
      const int32_t i = i0 + r;
      meta[r] = 0;
      if (i < s) {
        const uint64_t e = E[i];
        const int sd = ent_side(e);
        meta[r] = (ent_node(e) == (sd ? u : v) ? 1u : 0u) | ((uint32_t)sd << 1);
      }
    }
    int32_t cnt = 0, cntu = 0;
    uint32_t dmask = 0;
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
      const int32_t i = i0 + r;
      if (i >= s) continue;
      const bool isP = meta[r] & 1u;
      const bool isC = !isP && (nodes[r] == nodes[r + 1] || nodes[r + 2] == nodes[r + 1]);
      if (!isP && !isC) {
        dmask |= 1u << r;
        ++cnt;
        if (!(meta[r] & 2u)) ++cntu;
      }
    }
    int32_t tot;
    const int32_t pre = block_excl_scan(cnt | (cntu << 16), B.scan, &tot);
    int32_t pos = nD + (pre & 0xFFFF);
    // entries before this thread's first: i0 (all earlier ones are placed)
    int32_t kpos = (i0 < s ? i0 : s) - pos;
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
      if (i0 + r >= s) break;
      if (dmask & (1u << r)) D[pos++] = i0 + r;
      else D[s - 1 - kpos++] = i0 + r;
    }
    nD += tot & 0xFFFF;
    a += tot >> 16;
  }
  __syncthreads();
  const uint64_t t_classified = now_ticks();
  const DrawKey dk = draw_key(A, k);
  {
    // D in global memory: the touched positions through LDS (the tile is
    // free by now); D in LDS, or a long split: in place, in order
    const int32_t T = split_steps(nD, a);
    int32_t* Lt = reinterpret_cast<int32_t*>(B.u.tile.E);
    // hash slots in use: a power of two of at least 4 T (the arrays are laid
    // out for kSplitSlots); fewer slots are fewer to clear and scan
    int32_t nslots = 512;
    while (nslots < 4 * T && nslots < kSplitSlots) nslots <<= 1;
    if (items_only) {
      if (T > 0)
        item_split(Ig, nD, a, dk.seed, dk.round, dk.idx, Lt, B.u.tile.E + kSplitSlots / 2, nslots,
                   Lt + 3 * kSplitSlots, Lt + 3 * kSplitSlots + 2 * (kSplitSlots / 4), B.sboff);
    } else if (!in_lds && T > 0 && 4 * T <= kSplitSlots) {
      lds_split(D, nD, a, dk.seed, dk.round, dk.idx, Lt, Lt + kSplitSlots, Lt + 2 * kSplitSlots, nslots,
                Lt + 3 * kSplitSlots, Lt + 3 * kSplitSlots + 2 * (kSplitSlots / 4), B.sboff);
    } else {
      block_split(D, nD, a, dk.seed, dk.round, dk.idx, B.sboff, 2 * kTradeBlock);
    }
  }
  if (items_ready && !items_only) split_fix_items(E, D, nD, a, dk.seed, dk.round, dk.idx, Ig);
  if (tid == 0) {
    B.cnt[1] = 0;
    B.cnt[2] = 0;
    B.cnt[3] = 0;
  }
  __syncthreads();

  const uint64_t t_split = now_ticks();
  // ---- write and release (s items). Own-row entries fill the two rows from
  // their back (own_cur), so later trades released here may emit into them
  // from the front at once. Large trades open this phase to idle workgroups
  // through their write job.
  WriteCounts W{0, 0, 0, 0};
  const int w = tid >> 6;
  ItemSrc S{E, D, k, u, v, s, nD, a, du, dv, bu, bv, gu, gv};
  if (!share) {
    write_range<false>(A, S, w * kWave * kBatch, s, kWavesPerBlock * kWave * kBatch, B.cnt + 1, W);
  } else {
    // publish the items where other workgroups can read them, in the slot
    // region that is only ever written with agent-scope stores
    if (!items_ready)
      for (int32_t o = tid; o < s; o += nt) store_agent_u64(&Ig[o], item_entry<false>(S, o));
    publish_wait();
    __syncthreads();
    if (A.trace && tid == 0) A.trace[kTraceFields * (int64_t)k + 16] = (int64_t)now_ticks();
    HelpJob* J = A.jobs + blockIdx.x;
    const int32_t nchunks = (s + A.help_chunk - 1) / A.help_chunk;
    if (tid == 0) {
      store_agent64(&J->f.bu, bu);
      store_agent64(&J->f.bv, bv);
      store_agent64(&J->f.e_off, shared_list_off(A));
      store_agent(&J->f.k, k);
      store_agent(&J->f.u, u);
      store_agent(&J->f.v, v);
      store_agent(&J->f.s, s);
      store_agent(&J->f.nD, nD);
      store_agent(&J->f.a, a);
      store_agent(&J->f.du, du);
      store_agent(&J->f.dv, dv);
      store_agent(&J->f.gu, gu);
      store_agent(&J->f.gv, gv);
      store_agent(&J->f.phase, 2);
      open_job(A, J, nchunks);
    }
    __syncthreads();
    S.E = reinterpret_cast<const uint64_t*>(Ig);
    S.D = nullptr;
    for (;;) {
      int32_t c = -1;
      if (lane_id() == 0) c = claim_chunk(J);
      c = wave_bcast(c, 0);
      if (c < 0) break;
      const int32_t first = c * A.help_chunk;
      write_range<true>(A, S, first, first + A.help_chunk < s ? first + A.help_chunk : s, kWave * kBatch,
                        J->c.own, W);
      publish_wait();
      if (lane_id() == 0) {
        atomic_add(&J->c.done, 1);
        if (A.trace) atomicAdd(&B.cnt[3], 1);
      }
    }
    __syncthreads();
    if (tid == 0) {
      if (A.trace) A.trace[kTraceFields * (int64_t)k + 17] = (int64_t)now_ticks();
      close_job(A, J, nchunks);
      if (A.trace) {
        A.trace[kTraceFields * (int64_t)k + 18] = (int64_t)now_ticks();
        A.trace[kTraceFields * (int64_t)k + 19] = B.cnt[3];
      }
      B.cnt[1] = load_agent(&J->c.own[0]);
      B.cnt[2] = load_agent(&J->c.own[1]);
    }
  }
  __syncthreads();
  if (tid == 0) {
    // the back parts of the own rows, for the row check after the kernel
    if (B.cnt[1]) atomic_add(&A.own_cur[u], B.cnt[1]);
    if (B.cnt[2]) atomic_add(&A.own_cur[v], B.cnt[2]);
    counters[0] += (unsigned long long)s;
    counters[4] += t_gathered - t_begin;
    counters[5] += t_split - t_gathered;
    counters[6] += now_ticks() - t_split;
    if (A.trace) {
      int64_t* T = A.trace + kTraceFields * (int64_t)k;
      T[4] = (int64_t)t_lists;
      T[5] = (int64_t)t_gathered;
      T[6] = (int64_t)t_classified;
      T[7] = (int64_t)t_split;
      T[8] = s;
      T[9] = giant ? 1 : (in_lds ? 2 : 3);
      T[10] = du;
      T[11] = dv;
      T[12] = nD;
      T[13] = a;
      T[14] = B.tick[0] ? (int64_t)B.tick[0] : -1;
    }
  }
  counters[1] += W.fwd;
  counters[2] += W.push;
  counters[3] += W.emit;
  const int32_t moved = wave_sum((int32_t)W.moved);
  if (lane_id() == 0 && moved) atomicAdd(&A.stats[kStatMoved], (unsigned long long)moved);
  if (tid == 0 && !share) atomicAdd(&A.stats[kStatCounted], 1ull);
  __syncthreads();
}

__device__ __forceinline__ void big_worker(const TradeArgs& A, BigLds& B) {
  const int tid = threadIdx.x;
  uint64_t* slot = A.slots + (int64_t)blockIdx.x * A.slot_elems;
  // per-thread partial counters: work, forwarded, pushes, emitted, then
  // (thread 0) ticks of gather, split, write, release
  unsigned long long counters[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  unsigned long long max_ticks = 0;
  unsigned long long n_big = 0;
  Watchdog wd{0, 0};
  int32_t backoff = 1;
  for (;;) {
    if (tid == 0) {
      int32_t k;
      if (load_agent(&A.ctrl[cw(kCwAbort)])) {
        k = -2;
      } else {
        k = queue_pop(A, A.qb, kQbShards, kCwQbHead0, kCwQbTail0, (int)(blockIdx.x % kQbShards), kQbShards);
        if (k < 0) {
          const int32_t done = load_agent(&A.ctrl[cw(kCwDone)]);
          if (done >= A.L) k = -2;
          else if (wd.stalled(A, done)) { raise_error(A, kErrWatchdog); k = -2; }
        }
      }
      B.next = k;
    }
    __syncthreads();
    const int32_t k = B.next;
    __syncthreads();
    if (k == -2) break;
    if (k < 0) {
      // the whole workgroup may take part of a giant's bitmap pass
      if (tid == 0) {
        int32_t jj = -1;
        const uint64_t m = (uint64_t)(uint32_t)load_agent(&A.ctrl[cw(kCwJobMask2)]) |
                           ((uint64_t)(uint32_t)load_agent(&A.ctrl[cw(kCwJobMask3)]) << 32);
        if (m) {
          const int rot = (int)(blockIdx.x & 63);
          const uint64_t rm = rot ? ((m >> rot) | (m << (64 - rot))) : m;
          const int32_t j = (int32_t)((__builtin_ctzll(rm) + rot) & 63);
          const int32_t c = claim_chunk(A.jobs + kMaxJobs + j);
          if (c >= 0) jj = j | (c << 8);
        }
        B.next = jj;
      }
      __syncthreads();
      const int32_t fj = B.next;
      __syncthreads();
      if (fj >= 0) {
        fused_help(A, B, fj & 255, fj >> 8);
        backoff = 1;
        continue;
      }
      WriteCounts H{0, 0, 0, 0};
      const bool helped = try_help(A, (int32_t)blockIdx.x, H, 1);
      counters[1] += H.fwd;
      counters[2] += H.push;
      counters[3] += H.emit;
      if (helped) {
        backoff = 1;
      } else {
        idle_backoff(backoff);
        backoff = backoff < kBigMaxBackoff ? backoff * 2 : kBigMaxBackoff;
      }
      continue;
    }
    backoff = 1;
    consume_order();
    const uint64_t t0 = now_ticks();
    big_trade(A, k, B, slot, counters);
    const uint64_t t1 = now_ticks();
    const uint64_t dt = t1 - t0;
    if (dt > max_ticks) max_ticks = dt;
    if (A.trace && tid == 0) {
      A.trace[kTraceFields * (int64_t)k + 1] = (int64_t)t0;
      A.trace[kTraceFields * (int64_t)k + 2] = (int64_t)t1;
    }
    if (tid == 0) {
      atomic_add(&A.ctrl[cw(kCwDone)], 1);
      n_big += 1;
    }
  }
  __syncthreads();
  if (counters[0]) atomicAdd(&A.stats[kStatWork], counters[0]);
  if (counters[1]) atomicAdd(&A.stats[kStatForward], counters[1]);
  if (counters[2]) atomicAdd(&A.stats[kStatPush], counters[2]);
  if (counters[3]) atomicAdd(&A.stats[kStatEmit], counters[3]);
  if (tid == 0 && n_big) atomicAdd(&A.stats[kStatBig], n_big);
  if (tid == 0) {
    const unsigned long long busy = counters[4] + counters[5] + counters[6] + counters[7];
    if (busy) atomicAdd(&A.stats[kStatBigTicks], busy);
    if (counters[4]) atomicAdd(&A.stats[kStatBigGather], counters[4]);
    if (counters[5]) atomicAdd(&A.stats[kStatBigSplit], counters[5]);
    if (counters[6]) atomicAdd(&A.stats[kStatBigWrite], counters[6]);
    if (counters[7]) atomicAdd(&A.stats[kStatBigRelease], counters[7]);
    if (max_ticks) atomicMax(&A.stats[kStatBigMaxTicks], max_ticks);
  }
}

__global__ void __launch_bounds__(kTradeBlock) k_trade(TradeArgs A) {
  __shared__ TradeLds lds;
  if (load_agent(&A.ctrl[cw(kCwErr)])) return;
  if ((int32_t)blockIdx.x < A.nbig) {
    big_worker(A, lds.big);
  } else {
    for (int i = threadIdx.x; i < kPoolSlots; i += blockDim.x) lds.small.pool[i] = -1;
    __syncthreads();
    small_worker(A, lds.small.wave[threadIdx.x >> 6], lds.small.pool);
  }
}

}  // namespace cbx
