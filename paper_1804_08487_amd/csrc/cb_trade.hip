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
// (global scratch, radix sort); every other workgroup holds four wavefronts
// that each run small trades (deg u + deg v <= small_max) in LDS.
#include "cb_block.hpp"
#include "cb_kernels.hpp"

namespace cbx {

// Entry = ((node << 1 | side) << 32) | tag; side 0 = u's list, 1 = v's.
// tag 0: final when emitted (earlier node or the node left out),
// tag 1: the partner, tag t + 2: node of the later trade t.
constexpr uint32_t kTagEmit = 0u;
constexpr uint32_t kTagPartner = 1u;

__device__ __forceinline__ uint64_t make_entry(int32_t x, int side, uint32_t tag) {
  return ((uint64_t)(((uint32_t)x << 1) | (uint32_t)side) << 32) | tag;
}
__device__ __forceinline__ int32_t ent_node(uint64_t e) { return (int32_t)(e >> 33); }
__device__ __forceinline__ int ent_side(uint64_t e) { return (int)((e >> 32) & 1u); }
__device__ __forceinline__ uint32_t ent_tag(uint64_t e) { return (uint32_t)e; }
__device__ __forceinline__ uint32_t tag_of(int32_t t, int32_t k) {
  return t == k ? kTagPartner : (t == kUnmatched ? kTagEmit : (uint32_t)t + 2u);
}

struct WaveLds {
  uint64_t E[kSmallCap];
  int32_t D[kSmallCap];
  int32_t stack[kStackCap];
};

struct BigLds {
  RadixLds R;
  int32_t scan[kWavesPerBlock + 1];
  int32_t next;
  int32_t cnt[4];
  int32_t base[2];
  int32_t ndone;
};

union TradeLds {
  WaveLds wave[kWavesPerBlock];
  BigLds big;
};

__device__ __forceinline__ void raise_error(const TradeArgs& A, int32_t bits) {
  atomic_or(&A.ctrl[kCtrlErr], bits);
  store_agent(&A.ctrl[kCtrlAbort], 1);
}

// Split of the ascending disjoint set (indices into the entry array) in
// place; u receives D[0..a), v receives D[a..N).
template <typename Idx>
__device__ __forceinline__ void split_serial(Idx* D, int64_t N, int64_t a, uint64_t seed,
                                             uint32_t round, int32_t k) {
  if (a <= N - a) {
    for (int64_t j = 0; j < a; ++j) {
      const uint64_t x = philox64(seed, (uint32_t)k, round, (uint32_t)j, kTagSplit);
      const int64_t r = j + (int64_t)bounded(x, (uint64_t)(N - j));
      const Idx t = D[j]; D[j] = D[r]; D[r] = t;
    }
  } else {
    for (int64_t j = N - 1; j >= a; --j) {
      const uint64_t x = philox64(seed, (uint32_t)k, round, (uint32_t)j, kTagSplit);
      const int64_t r = (int64_t)bounded(x, (uint64_t)(j + 1));
      const Idx t = D[j]; D[j] = D[r]; D[r] = t;
    }
  }
}

// Pop one item of a ready queue (single thread). -1: empty or lost a race.
__device__ int32_t queue_pop(const TradeArgs& A, int32_t* q, int head_slot, int tail_slot) {
  int32_t* head = &A.ctrl[head_slot];
  const int32_t h = load_agent(head);
  const int32_t t = load_agent(&A.ctrl[tail_slot]);
  if (h >= t) return -1;
  if (!atomic_cas(head, h, h + 1)) return -1;
  int32_t k;
  // The pusher reserved slot h before filling it; the fill is imminent.
  while ((k = load_agent(&q[h])) < 0) {
    if (load_agent(&A.ctrl[kCtrlAbort])) return -1;
    __builtin_amdgcn_s_sleep(1);
  }
  return k;
}

// Hand a ready trade to other workers (single lane; caller fenced).
__device__ __forceinline__ void queue_push(const TradeArgs& A, int32_t* q, int tail_slot, int32_t k) {
  const int32_t pos = atomic_add(&A.ctrl[tail_slot], 1);
  if (pos >= A.L) { raise_error(A, kErrCapacity); return; }
  store_agent(&q[pos], k);
}

__device__ __forceinline__ int32_t source_pop(const TradeArgs& A) {
  if (load_agent(&A.ctrl[kCtrlSrcHead]) >= load_agent(&A.ctrl[kCtrlSrcCount])) return -1;
  const int32_t h = atomic_add(&A.ctrl[kCtrlSrcHead], 1);
  if (h < load_agent(&A.ctrl[kCtrlSrcCount])) return A.src_list[h];
  return -1;
}

// Emit/forward one output edge {owner, x}. Returns true if it is forwarded.
__device__ __forceinline__ void route_edge(const TradeArgs& A, int32_t owner, int32_t x,
                                           uint32_t tag) {
  if (tag == kTagPartner) return;  // own row only (handled by the caller)
  const int64_t rx = A.rp[x];
  const int32_t dx = (int32_t)(A.rp[x + 1] - rx);
  if (tag == kTagEmit) {
    const int32_t p = atomic_add(&A.out_cur[x], 1);
    if (p < dx) A.col_out[rx + p] = owner; else raise_error(A, kErrOut);
  } else {
    const int32_t p = atomic_add(&A.inbox_cur[x], 1);
    if (p < dx) A.inbox[rx + p] = owner; else raise_error(A, kErrInbox);
  }
}

// ============================================================ small trades

struct WaveState {
  int32_t top;        // local stack depth (uniform)
  int32_t ndone;
  unsigned long long n_small, n_push, work, fwd, emit;
};

// Drops the dependency counters of later trades reached by this trade's
// output; ready trades go to the local stack or the global queue.
__device__ __forceinline__ void wave_release_item(const TradeArgs& A, WaveLds& W, WaveState& S,
                                                  bool fwd, uint32_t tag) {
  bool ready = false;
  int32_t t = -1;
  if (fwd) {
    t = (int32_t)(tag - 2u);
    const int32_t old = atomic_add(&A.dep[t], -1);
    if (old <= 0) raise_error(A, kErrDep);
    ready = old == 1;
  }
  const uint64_t m = ballot(ready);
  if (m == 0) return;
  const int cnt = popc64(m);
  const int room = A.stack_cap - S.top;
  const int r = rank_below(m);
  const uint64_t spill = ballot(ready && r >= room);
  if (spill) fence_acq_rel();
  if (ready) {
    if (r < room) W.stack[S.top + r] = t;
    else queue_push(A, A.qs, kCtrlQsTail, t);
  }
  wave_sync();
  S.top += cnt < room ? cnt : (room > 0 ? room : 0);
  S.n_push += (unsigned long long)popc64(spill);
}

__device__ void small_trade(const TradeArgs& A, int32_t k, int32_t u, int32_t v, WaveLds& W,
                            WaveState& S) {
  const int l = lane_id();
  const int64_t bu = A.rp[u], bv = A.rp[v];
  const int32_t du = (int32_t)(A.rp[u + 1] - bu), dv = (int32_t)(A.rp[v + 1] - bv);
  const int32_t s = du + dv;
  const int32_t niu = load_agent(&A.inbox_cur[u]);
  const int32_t niv = load_agent(&A.inbox_cur[v]);

  // ---- gather both lists into E (u's at [0, du), v's at [du, s))
  int32_t nf[2] = {0, 0};
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const int64_t b = side ? bv : bu;
    const int32_t d = side ? dv : du;
    const int32_t off = side ? du : 0;
    int32_t cnt = 0;
    for (int32_t c = 0; c < d; c += kWave) {
      const int32_t e = c + l;
      int32_t x = 0, t = -1;
      if (e < d) { x = A.col[b + e]; t = A.col_t[b + e]; }
      const bool fresh = e < d && t >= k;
      const uint64_t m = ballot(fresh);
      if (fresh) W.E[off + cnt + rank_below(m)] = make_entry(x, side, tag_of(t, k));
      cnt += popc64(m);
    }
    nf[side] = cnt;
    const int32_t ni = side ? niv : niu;
    if (cnt + ni != d) { raise_error(A, kErrGather); return; }
    for (int32_t j = l; j < ni; j += kWave) W.E[off + cnt + j] = make_entry(A.inbox[b + j], side, kTagEmit);
  }
  wave_sync();
  wave_bitonic_sort(W.E, (uint32_t)s);

  // ---- classify: shared (C), partner (P), disjoint (D, kept ascending)
  int32_t nD = 0, a = 0;
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
  }
  wave_sync();
  if (l == 0) split_serial<int32_t>(W.D, nD, a, A.seed, A.round, k);
  wave_sync();

  // ---- write: own-row finals, other-row finals, forwards
  int32_t nfwd = 0, nemit = 0;
#pragma unroll
  for (int pass = 0; pass < 2; ++pass) {
    const int32_t count = pass ? nD : s;
    for (int32_t c = 0; c < count; c += kWave) {
      const int32_t o = c + l;
      bool valid = o < count;
      int32_t owner = u, x = 0;
      uint32_t tag = 0;
      if (valid) {
        if (pass == 0) {
          const uint64_t e = W.E[o];
          x = ent_node(e);
          tag = ent_tag(e);
          const bool isP = tag == kTagPartner;
          const bool isC = !isP && ((o > 0 && ent_node(W.E[o - 1]) == x) ||
                                    (o + 1 < s && ent_node(W.E[o + 1]) == x));
          valid = isP || isC;
          owner = ent_side(e) ? v : u;
        } else {
          const uint64_t e = W.E[W.D[o]];
          x = ent_node(e);
          tag = ent_tag(e);
          owner = o < a ? u : v;
        }
      }
      const bool own = valid && tag <= kTagPartner;
      const uint64_t mu = ballot(own && owner == u);
      const uint64_t mv = ballot(own && owner == v);
      int32_t baseu = 0, basev = 0;
      if (l == 0) {
        if (mu) baseu = atomic_add(&A.out_cur[u], popc64(mu));
        if (mv) basev = atomic_add(&A.out_cur[v], popc64(mv));
      }
      baseu = wave_bcast(baseu, 0);
      basev = wave_bcast(basev, 0);
      if (own) {
        const int32_t p = owner == u ? baseu + rank_below(mu) : basev + rank_below(mv);
        const int32_t dd = owner == u ? du : dv;
        if (p < dd) A.col_out[(owner == u ? bu : bv) + p] = x; else raise_error(A, kErrOut);
      }
      if (valid) route_edge(A, owner, x, tag);
      nfwd += popc64(ballot(valid && tag >= 2u));
      nemit += popc64(ballot(valid && tag == kTagEmit));
    }
  }
  // every write above is visible before any counter it unlocks
  fence_release();
#pragma unroll
  for (int pass = 0; pass < 2; ++pass) {
    const int32_t count = pass ? nD : s;
    for (int32_t c = 0; c < count; c += kWave) {
      const int32_t o = c + l;
      bool fwd = false;
      uint32_t tag = 0;
      if (o < count) {
        if (pass == 0) {
          const uint64_t e = W.E[o];
          const int32_t x = ent_node(e);
          tag = ent_tag(e);
          const bool isC = tag != kTagPartner && ((o > 0 && ent_node(W.E[o - 1]) == x) ||
                                                  (o + 1 < s && ent_node(W.E[o + 1]) == x));
          fwd = isC && tag >= 2u;
        } else {
          tag = ent_tag(W.E[W.D[o]]);
          fwd = tag >= 2u;
        }
      }
      wave_release_item(A, W, S, fwd, tag);
    }
  }
  S.n_small += 1;
  S.work += (unsigned long long)s;
  S.fwd += (unsigned long long)nfwd;
  S.emit += (unsigned long long)nemit;
}

__device__ void wave_flush(const TradeArgs& A, WaveState& S) {
  if (lane_id() == 0) {
    if (S.ndone) atomic_add(&A.ctrl[kCtrlDone], S.ndone);
    if (S.n_small) atomicAdd(&A.stats[kStatSmall], S.n_small);
    if (S.n_push) atomicAdd(&A.stats[kStatPush], S.n_push);
    if (S.work) atomicAdd(&A.stats[kStatWork], S.work);
    if (S.fwd) atomicAdd(&A.stats[kStatForward], S.fwd);
    if (S.emit) atomicAdd(&A.stats[kStatEmit], S.emit);
  }
  S.ndone = 0;
  S.n_small = S.n_push = S.work = S.fwd = S.emit = 0;
}

__device__ void small_worker(const TradeArgs& A, WaveLds& W) {
  const int l = lane_id();
  WaveState S{};
  uint64_t idle_since = 0;
  for (;;) {
    int32_t k = -1;
    if (S.top > 0) {
      S.top -= 1;
      k = W.stack[S.top];
    } else {
      if (l == 0) {
        k = source_pop(A);
        if (k < 0) k = queue_pop(A, A.qs, kCtrlQsHead, kCtrlQsTail);
      }
      k = wave_bcast(k, 0);
    }
    if (k < 0) {
      wave_flush(A, S);
      int32_t stop = 0;
      if (l == 0) {
        stop = load_agent(&A.ctrl[kCtrlAbort]) ||
               load_agent(&A.ctrl[kCtrlDone]) >= A.L;
        if (!stop) {
          const uint64_t now = now_ticks();
          if (idle_since == 0) idle_since = now;
          else if (now - idle_since > A.watchdog_ticks) { raise_error(A, kErrWatchdog); stop = 1; }
        }
      }
      if (wave_bcast(stop, 0)) break;
      __builtin_amdgcn_s_sleep(2);
      continue;
    }
    idle_since = 0;
    const int32_t u = A.perm[2 * k], v = A.perm[2 * k + 1];
    const int64_t s = (A.rp[u + 1] - A.rp[u]) + (A.rp[v + 1] - A.rp[v]);
    if (s > A.small_max) {
      // large trade: hand it to a workgroup worker
      if (l == 0) {
        fence_acq_rel();
        queue_push(A, A.qb, kCtrlQbTail, k);
      }
      continue;
    }
    fence_acquire();
    small_trade(A, k, u, v, W, S);
    S.ndone += 1;
    int32_t ab = 0;
    if (l == 0) ab = load_agent(&A.ctrl[kCtrlAbort]);
    if (wave_bcast(ab, 0)) break;
  }
  wave_flush(A, S);
}

// ============================================================ large trades

__device__ void big_trade(const TradeArgs& A, int32_t k, BigLds& B, uint64_t* slot,
                          unsigned long long* counters) {
  const int tid = threadIdx.x;
  const int32_t u = A.perm[2 * k], v = A.perm[2 * k + 1];
  const int64_t bu = A.rp[u], bv = A.rp[v];
  const int32_t du = (int32_t)(A.rp[u + 1] - bu), dv = (int32_t)(A.rp[v + 1] - bv);
  const int64_t s = (int64_t)du + dv;
  if (s > A.smax) {
    if (tid == 0) raise_error(A, kErrCapacity);
    return;
  }
  uint64_t* E0 = slot;
  uint64_t* E1 = slot + A.smax;
  int32_t* D = (int32_t*)(slot + 2 * A.smax);
  const int32_t niu = load_agent(&A.inbox_cur[u]);
  const int32_t niv = load_agent(&A.inbox_cur[v]);

  // ---- gather (order is irrelevant: the list is sorted next)
  for (int side = 0; side < 2; ++side) {
    const int64_t b = side ? bv : bu;
    const int32_t d = side ? dv : du;
    const int32_t off = side ? du : 0;
    const int32_t ni = side ? niv : niu;
    if (tid == 0) B.cnt[0] = 0;
    __syncthreads();
    for (int32_t e = tid; e < d; e += blockDim.x) {
      const int32_t t = A.col_t[b + e];
      if (t >= k) {
        const int32_t p = atomicAdd(&B.cnt[0], 1);
        E0[off + p] = make_entry(A.col[b + e], side, tag_of(t, k));
      }
    }
    __syncthreads();
    const int32_t nf = B.cnt[0];
    __syncthreads();
    if (nf + ni != d) {
      if (tid == 0) raise_error(A, kErrGather);
      return;
    }
    for (int32_t j = tid; j < ni; j += blockDim.x)
      E0[off + nf + j] = make_entry(A.inbox[b + j], side, kTagEmit);
  }
  __syncthreads();
  uint64_t* E = block_radix_sort<uint64_t>(E0, E1, s, A.keybits, B.R);

  // ---- classify and compact the disjoint set in ascending order
  int32_t nD = 0, a = 0;
  for (int64_t c = 0; c < s; c += blockDim.x) {
    const int64_t i = c + tid;
    int32_t isD = 0, isU = 0;
    if (i < s) {
      const uint64_t e = E[i];
      const int32_t x = ent_node(e);
      const bool isP = ent_tag(e) == kTagPartner;
      const bool isC = !isP && ((i > 0 && ent_node(E[i - 1]) == x) ||
                                (i + 1 < s && ent_node(E[i + 1]) == x));
      isD = (!isP && !isC) ? 1 : 0;
      isU = (isD && ent_side(e) == 0) ? 1 : 0;
    }
    int32_t tot;
    const int32_t pos = block_excl_scan(isD, B.scan, &tot);
    if (isD) D[nD + pos] = (int32_t)i;
    nD += tot;
    int32_t totu;
    (void)block_excl_scan(isU, B.scan, &totu);
    a += totu;
  }
  __syncthreads();
  if (tid == 0) split_serial<int32_t>(D, nD, a, A.seed, A.round, k);
  __syncthreads();

  // ---- write
  int32_t nfwd = 0, nemit = 0;
  for (int pass = 0; pass < 2; ++pass) {
    const int64_t count = pass ? nD : s;
    for (int64_t c = 0; c < count; c += blockDim.x) {
      const int64_t o = c + tid;
      bool valid = o < count;
      int32_t owner = u, x = 0;
      uint32_t tag = 0;
      if (valid) {
        if (pass == 0) {
          const uint64_t e = E[o];
          x = ent_node(e);
          tag = ent_tag(e);
          const bool isP = tag == kTagPartner;
          const bool isC = !isP && ((o > 0 && ent_node(E[o - 1]) == x) ||
                                    (o + 1 < s && ent_node(E[o + 1]) == x));
          valid = isP || isC;
          owner = ent_side(e) ? v : u;
        } else {
          const uint64_t e = E[D[o]];
          x = ent_node(e);
          tag = ent_tag(e);
          owner = o < a ? u : v;
        }
      }
      const bool own = valid && tag <= kTagPartner;
      if (tid == 0) { B.cnt[1] = 0; B.cnt[2] = 0; }
      __syncthreads();
      int32_t slot_pos = -1;
      if (own) slot_pos = atomicAdd(&B.cnt[owner == u ? 1 : 2], 1);
      __syncthreads();
      if (tid == 0) {
        B.base[0] = B.cnt[1] ? atomic_add(&A.out_cur[u], B.cnt[1]) : 0;
        B.base[1] = B.cnt[2] ? atomic_add(&A.out_cur[v], B.cnt[2]) : 0;
      }
      __syncthreads();
      if (own) {
        const int32_t p = B.base[owner == u ? 0 : 1] + slot_pos;
        const int32_t dd = owner == u ? du : dv;
        if (p < dd) A.col_out[(owner == u ? bu : bv) + p] = x; else raise_error(A, kErrOut);
      }
      if (valid) {
        route_edge(A, owner, x, tag);
        if (tag >= 2u) ++nfwd;
        if (tag == kTagEmit) ++nemit;
      }
    }
  }
  __syncthreads();
  fence_release();
  for (int pass = 0; pass < 2; ++pass) {
    const int64_t count = pass ? nD : s;
    for (int64_t o = tid; o < count; o += blockDim.x) {
      uint32_t tag;
      bool fwd;
      if (pass == 0) {
        const uint64_t e = E[o];
        const int32_t x = ent_node(e);
        tag = ent_tag(e);
        const bool isC = tag != kTagPartner && ((o > 0 && ent_node(E[o - 1]) == x) ||
                                                (o + 1 < s && ent_node(E[o + 1]) == x));
        fwd = isC && tag >= 2u;
      } else {
        tag = ent_tag(E[D[o]]);
        fwd = tag >= 2u;
      }
      if (fwd) {
        const int32_t t = (int32_t)(tag - 2u);
        const int32_t old = atomic_add(&A.dep[t], -1);
        if (old <= 0) raise_error(A, kErrDep);
        if (old == 1) {
          fence_acq_rel();
          queue_push(A, A.qs, kCtrlQsTail, t);
          counters[2] += 1;
        }
      }
    }
  }
  if (tid == 0) counters[0] += (unsigned long long)s;
  counters[1] += (unsigned long long)(nfwd);
  counters[3] += (unsigned long long)(nemit);
  __syncthreads();
}

__device__ void big_worker(const TradeArgs& A, BigLds& B) {
  const int tid = threadIdx.x;
  uint64_t* slot = A.slots + (int64_t)blockIdx.x * A.slot_elems;
  // per-thread partial counters: work, forwarded, pushes, emitted
  unsigned long long counters[4] = {0, 0, 0, 0};
  unsigned long long n_big = 0;
  uint64_t idle_since = 0;
  if (tid == 0) B.ndone = 0;
  __syncthreads();
  for (;;) {
    if (tid == 0) {
      int32_t k = -1;
      if (load_agent(&A.ctrl[kCtrlAbort])) {
        k = -2;
      } else {
        k = queue_pop(A, A.qb, kCtrlQbHead, kCtrlQbTail);
        if (k < 0) k = source_pop(A);
        if (k < 0) k = queue_pop(A, A.qs, kCtrlQsHead, kCtrlQsTail);
        if (k < 0) {
          if (B.ndone) { atomic_add(&A.ctrl[kCtrlDone], B.ndone); B.ndone = 0; }
          if (load_agent(&A.ctrl[kCtrlDone]) >= A.L) {
            k = -2;
          } else {
            const uint64_t now = now_ticks();
            if (idle_since == 0) idle_since = now;
            else if (now - idle_since > A.watchdog_ticks) { raise_error(A, kErrWatchdog); k = -2; }
          }
        } else {
          idle_since = 0;
        }
      }
      B.next = k;
    }
    __syncthreads();
    const int32_t k = B.next;
    __syncthreads();
    if (k == -2) break;
    if (k < 0) {
      __builtin_amdgcn_s_sleep(2);
      continue;
    }
    fence_acquire();
    big_trade(A, k, B, slot, counters);
    if (tid == 0) { B.ndone += 1; n_big += 1; }
  }
  __syncthreads();
  if (tid == 0 && B.ndone) atomic_add(&A.ctrl[kCtrlDone], B.ndone);
  if (counters[0]) atomicAdd(&A.stats[kStatWork], counters[0]);
  if (counters[1]) atomicAdd(&A.stats[kStatForward], counters[1]);
  if (counters[2]) atomicAdd(&A.stats[kStatPush], counters[2]);
  if (counters[3]) atomicAdd(&A.stats[kStatEmit], counters[3]);
  if (tid == 0 && n_big) atomicAdd(&A.stats[kStatBig], n_big);
}

__global__ void __launch_bounds__(kTradeBlock) k_trade(TradeArgs A) {
  __shared__ TradeLds lds;
  if (load_agent(&A.ctrl[kCtrlErr])) return;
  if ((int32_t)blockIdx.x < A.nbig) {
    big_worker(A, lds.big);
  } else {
    small_worker(A, lds.wave[threadIdx.x >> 6]);
  }
}

}  // namespace cbx
