// Kernel entry points and argument blocks shared by the host orchestration
// (cb_host.hip) and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cb_device.hpp"

namespace cbx {

// Control words of one graph (int32, device memory), each on its own
// 128-byte line so that polling and pushing do not share a cache line.
constexpr int kCtrlStride = 32;
constexpr int kQsShards = 16;   // ready queues of small trades
constexpr int kQbShards = 4;    // ready queues of large trades
enum CtrlWord : int {
  kCwSrcCount = 0,   // trades with no dependency (written by k_sources)
  kCwSrcHead,        // next source to hand out
  kCwDone,           // completed trades (flushed by workers in batches)
  kCwErr,            // error bits (sticky across rounds)
  kCwAbort,          // set with an error: every worker leaves
  kCwDbgBits,        // error bits of the first recorded error
  kCwDbgA,           // first recorded error: trade (+1)
  kCwDbgB,           // first recorded error: detail
  kCwQsHead0,
  kCwQsTail0 = kCwQsHead0 + kQsShards,
  kCwQbHead0 = kCwQsTail0 + kQsShards,
  kCwQbTail0 = kCwQbHead0 + kQbShards,
  kCwJobMask0 = kCwQbTail0 + kQbShards,   // write jobs open to helpers: workgroups 0..31
  kCwJobMask1,                            // ... and 32..63
  kCwJobMask2,                            // giant bitmap passes open to a helper workgroup: 0..31
  kCwJobMask3,                            // ... and 32..63
  kCwCount
};
__host__ __device__ constexpr int cw(int word) { return word * kCtrlStride; }
constexpr int kCtrlInts = kCwCount * kCtrlStride;

// 64-bit round counters (device memory).
enum Stat : int {
  kStatSmall = 0, kStatBig, kStatPush, kStatWork, kStatForward, kStatEmit, kStatSources,
  kStatSmallTicks,   // wall-clock ticks inside small trades (all wavefronts)
  kStatBigTicks,     // wall-clock ticks inside large trades (all workgroups)
  kStatBigGather,    // ... of which collecting and sorting the lists
  kStatBigSplit,     // ... classification and split
  kStatBigWrite,     // ... writing and forwarding
  kStatBigRelease,   // ... unlocking later trades
  kStatBigMaxTicks,  // longest single large trade
  kStatMoved,        // disjoint neighbours that changed sides (counted trades only)
  kStatCounted,      // trades whose moved neighbours were counted (all but shared write phases)
  kStatCount = 16
};

constexpr int kSmallCap = 512;        // largest deg u + deg v on one wavefront
constexpr int kBigCap = 12288;        // largest deg u + deg v held in LDS by one workgroup
constexpr int kGiantMinDeg = kBigCap / 2;   // default giant degree: any other pair fits LDS
constexpr int kTradeBlock = 512;      // threads per trade-kernel workgroup (one per CU: 256 VGPRs each)
constexpr int kWavesPerBlock = kTradeBlock / 64;
constexpr int kStackCap = 16;         // ready trades a wavefront may keep
constexpr int kTraceFields = 24;      // int64 per trade of the optional trace
constexpr int kMaxJobs = 64;          // workgroups that can open their write phase to helpers
                                      // (and, in a second set of jobs, part of a giant's bitmap pass)
constexpr int32_t kHelpChunk = 128;   // default output items per claimed chunk
constexpr int32_t kHelpMinItems = 4096;   // default: smaller trades work alone
constexpr int32_t kSbChunk = 16;      // bitmap superblocks per claimed extraction chunk

// A phase of one large trade open to helper wavefronts (one job per
// workgroup worker, reused phase after phase): phase 1 extracts a giant
// node's neighbour set from its bitmap, phase 2 writes the trade's output.
// The owner publishes the fields, then the ticket of a new generation g with
// n chunks; a wavefront claims chunk c by moving the ticket's counter from c
// to c + 1, and the value it gets back alone says whether it holds a chunk
// (c < n). The fields of g stay unchanged until every chunk of it is
// reported in `done`, so a wavefront holding a chunk reads g's fields.
constexpr int kTicketCountBits = 24;   // chunk counter and chunk count per ticket
struct HelpJob {
  struct alignas(128) {
    unsigned long long ticket;   // generation (16 bits) | chunks (24) | next chunk (24)
  } t;
  struct alignas(128) {
    int32_t done;                // chunks written
    int32_t own[2];              // own-row positions handed out for u and v
  } c;
  struct alignas(128) {
    int64_t bu, bv;              // row offsets of u and v
    int64_t e_off;               // phase 2: items at owner's slot + e_off;
                                 // phase 1: output list there
    int32_t k, u, v, s, nD, a, du, dv;
    int32_t phase, gi, side, d;  // phase 1: giant id, side and size of the list
    int32_t gu, gv;              // phase 2: giant ids of u and v (-1: none)
    int32_t d_o, nK1, o, edge;   // phase 3 (part of a giant's bitmap pass): the other side
    int64_t sb_from, sb_to;      // phase 3: the helper's superblocks
  } f;
};
constexpr int kMatchCap = 2048;       // bucket size sorted in LDS by k_match_sort
constexpr int kMatchBlock = 256;
constexpr int kScanChunk = 2048;      // CSR entries per workgroup in k_depscan/k_validate
constexpr int kSrcBuckets = 256;     // buckets of relative position that order a round's sources
constexpr int kSegMidMax = 4096;      // rows sorted in LDS by one workgroup
constexpr int kSegWideMax = 32768;    // bigger rows up to this are sorted in LDS by one wide workgroup
constexpr int kSegWideThreads = 1024;
constexpr int kSegSmallMax = 64;      // rows sorted in registers by one wavefront

// Trade information of a node as stored per CSR entry (col_t) and per node
// (tinfo): its trade index, with bit 30 set when the node keeps its arrivals
// in a bitmap (a "giant" node); kUnmatched for the node left out.
constexpr int32_t kGiantBit = 0x40000000;
__host__ __device__ constexpr bool tinfo_giant(int32_t ti) { return ti != kUnmatched && (ti & kGiantBit); }
__host__ __device__ constexpr int32_t tinfo_trade(int32_t ti) { return ti == kUnmatched ? ti : (ti & ~kGiantBit); }

// Bitmap neighbour sets of giant nodes: per giant, words of 64 bits over all
// node ids (gwords per giant, a multiple of 64) and one count per superblock
// of 64 words (4096 ids).
struct GiantSets {
  const int32_t* giant_id;  // index among giant nodes, or -1
  unsigned long long* bm;   // ngiant * gwords
  int32_t* sc;              // ngiant * (gwords / 64)
  int64_t gwords;
};

// Add node y to giant gi's bitmap set.
__device__ __forceinline__ void giant_insert(const GiantSets& gs, int32_t gi, int32_t y) {
  atomicOr(&gs.bm[(int64_t)gi * gs.gwords + (y >> 6)], 1ull << (y & 63));
  atomicAdd(&gs.sc[(int64_t)gi * (gs.gwords >> 6) + (y >> 12)], 1);
}

// Independent chains run as one graph. Chain c owns the nodes
// [node_base[c], node_base[c+1]) (its CSR entries hold these global ids, and
// no edge joins two chains), the trades [trade_base[c], trade_base[c+1])
// (floor(n_c / 2) of them) and the matching buckets
// [bucket_base[c], bucket_base[c+1]) (a power of two per chain). Its node keys
// and split draws use its own seed and round, with local node ids and local
// trade indices (plus draw_base[c]); so each chain's result is the one it
// would have alone. The pair list `perm` holds the pairs of trade t at
// 2t, 2t+1; the left-out node of an odd chain c sits at
// 2 * trade_base[count] + left_base[c].
struct Chains {
  int32_t count;
  const int64_t* node_base;    // count + 1
  const int64_t* trade_base;   // count + 1
  const int32_t* bucket_base;  // count + 1
  const int32_t* left_base;    // count + 1 (odd chains before c)
  const uint64_t* seed;        // count
  const uint32_t* round;       // count
  const uint32_t* draw_base;   // count
};

// Largest c in [0, count) with base[c] <= x (base ascending, base[0] <= x).
template <typename T>
__device__ __forceinline__ int32_t chain_search(const T* base, int32_t count, T x) {
  int32_t lo = 0, hi = count - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (base[mid] <= x) lo = mid; else hi = mid - 1;
  }
  return lo;
}
__device__ __forceinline__ int32_t chain_of_node(const Chains& ch, int64_t v) {
  return ch.count == 1 ? 0 : chain_search(ch.node_base, ch.count, v);
}
__device__ __forceinline__ int32_t chain_of_trade(const Chains& ch, int64_t k) {
  return ch.count == 1 ? 0 : chain_search(ch.trade_base, ch.count, k);
}

struct TradeArgs {
  const int64_t* rp;
  const int32_t* col;
  const int32_t* col_t;     // trade information of every neighbour, from k_depscan
  const int32_t* tinfo;     // trade information per node
  const int32_t* perm;
  int32_t* inbox;           // CSR-shaped: arrivals for each node's row
  int32_t* inbox_cur;
  int32_t* col_out;         // CSR-shaped: final edges of the round
  int32_t* out_cur;         // final entries written into a row from its front
  int32_t* own_cur;         // entries a workgroup trade wrote into its own rows, from the back
  int32_t* dep;
  const int32_t* src_list;
  const int32_t* tsz;       // deg u + deg v per trade, from k_sources
  const uint4* ninfo;       // per node: row offset, degree, trade information (one load)
  int64_t* trace;           // optional: per trade ready, start, end tick and releasing trade
  HelpJob* jobs;            // kMaxJobs write jobs
  int32_t* qs;              // kQsShards ready queues of L slots (-1 = empty)
  int32_t* qb;              // kQbShards ready queues of large trades
  int32_t* ctrl;
  unsigned long long* stats;
  GiantSets gs;
  uint64_t* slots;          // large-trade scratch, slot_elems u64 per workgroup
  int64_t slot_elems;       // = 3 * smax + smax / 2 + 1: entries, lists, D, shared list
  int32_t* sbpre;           // per workgroup: prefix of a giant's superblock counts
  int64_t sbpre_stride;     // = superblocks + 1
  int64_t smax;             // largest possible deg u + deg v
  int64_t n;
  int32_t L;
  int32_t small_max;
  int32_t help_min;         // trades of at least this many items open their write phase (0: none)
  int32_t help_groups;      // workgroup b helps owners j with j % help_groups == b % help_groups
  int32_t help_chunk;       // items per claimed chunk of a shared write phase (a multiple of 64)
  int32_t idle_backoff;     // longest sleep of an idle wavefront worker, in units of 2048 cycles
  int32_t cu_pool;          // 1: ready small trades beyond the local stack go to the workgroup's LDS pool
  int32_t big_lds_max;
  int32_t nbig;
  int32_t stack_cap;
  int32_t keybits;          // bits of (node << 1 | side)
  Chains ch;                // seed, round and trade range of each chain
  uint64_t watchdog_ticks;
};

// ---- kernels ---------------------------------------------------------------
__global__ void k_round_reset(int64_t n, int32_t nb, int32_t* inbox_cur, int32_t* out_cur,
                              int32_t* own_cur, int32_t* bcount, int32_t* bcur, int32_t* ctrl,
                              unsigned long long* stats, int32_t reset_stats);
__global__ void k_phase_pairs(const int32_t* pairs, int32_t P, int32_t* perm, int32_t* trade_of,
                              int32_t* tinfo, int32_t* dep);
__global__ void k_copy_idle_edges(int64_t n, const int64_t* rp, const int32_t* col, const int32_t* trade_of,
                                  int32_t* col_out, int32_t* out_cur, int32_t* ctrl);
__global__ void k_set_draws(uint64_t* seed, uint32_t* round, uint32_t* draw_base, uint64_t s, uint32_t r,
                            uint32_t d);
__global__ void k_set_chain(uint64_t* seed, uint32_t* round, int32_t c, uint64_t s, uint32_t r);
__global__ void k_advance_rounds(uint32_t* round, int32_t count, uint32_t by);
__global__ void k_fill_i32(int32_t* p, int64_t count, int32_t value);
__global__ void k_single_chain(int64_t* node_base, int64_t* trade_base, int32_t* bucket_base,
                               int32_t* left_base, uint64_t* seed, uint32_t* round, uint32_t* draw_base,
                               int64_t n, int32_t nb, uint64_t s, uint32_t r);
__global__ void k_match_count(int64_t n, Chains ch, int32_t* bcount, const int32_t* ctrl);
__global__ void k_match_scan(int32_t nb, const int32_t* bcount, int32_t* bstart,
                             const int32_t* ctrl);
__global__ void k_match_scatter(int64_t n, Chains ch, const int32_t* bstart, int32_t* bcur,
                                int32_t* mtmp, const int32_t* ctrl);
__global__ void k_match_sort(Chains ch, int32_t nb, const int32_t* bstart, int32_t* mtmp,
                             uint64_t* mkey, int32_t* perm, int32_t* trade_of, int32_t* tinfo,
                             const int32_t* giant_id, int32_t* dep, int32_t* ctrl);
__global__ void k_depscan(int64_t n, int64_t nnz, const int64_t* rp, const int32_t* col,
                          const int32_t* trade_of, const int32_t* tinfo, int32_t* col_t,
                          int32_t* dep, GiantSets gs, const int32_t* ctrl);
__global__ void k_sources(int32_t L, const int32_t* dep, const int32_t* perm, const int64_t* rp,
                          int32_t small_max, int32_t* tsz, int32_t* src_list, int32_t* qb,
                          int32_t* ctrl, unsigned long long* stats, Chains ch, int32_t* sb, int pass);
__global__ void k_sources_scan(int32_t* sb, int32_t* ctrl);
__global__ void k_trade(TradeArgs A);
__global__ void k_check_giants_empty(int64_t total_sb, const int32_t* sc, int32_t* ctrl);
__global__ void k_node_info(int64_t n, const int64_t* rp, const int32_t* tinfo, uint4* ninfo);
__global__ void k_check_rows(int64_t n, const int64_t* rp, const int32_t* out_cur,
                             const int32_t* own_cur, int32_t* ctrl);
// The next round's dependency scan, done by the rebuild as it writes each
// row (the next round's matching is already in tinfo / trade_of; tinfo null:
// no scan). Per entry e of row x with neighbour y: col_t[e] = tinfo[y]; if x
// is matched, y's trade comes before x's adds one to dep[trade_of[x]], and a
// giant x puts every other neighbour y into its bitmap set.
struct NextScan {
  const int32_t* tinfo;
  const int32_t* trade_of;
  int32_t* col_t;
  int32_t* dep;
  GiantSets gs;
};
__global__ void k_segsort_small(const int32_t* rows, int64_t nrows, const int64_t* rp,
                                const int32_t* src, int32_t* dst, NextScan N, const int32_t* ctrl);
__global__ void k_segsort_mid(const int32_t* rows, int64_t nrows, const int64_t* rp,
                              const int32_t* src, int32_t* dst, int keybits, NextScan N,
                              const int32_t* ctrl);
__global__ void k_segsort_wide(const int32_t* rows, int64_t nrows, const int64_t* rp, const int32_t* src,
                               int32_t* dst, int keybits, const int32_t* ctrl);
__global__ void k_segsort_huge(const int32_t* rows, int64_t nrows, const int64_t* rp, const int32_t* src,
                               int32_t* dst, int keybits, const int32_t* ctrl);
__global__ void k_big_offsets(const int32_t* rows, int64_t nrows, const int64_t* rp, int64_t* boff);
__global__ void k_scan_big_rows(const int32_t* rows, int64_t nrows, const int64_t* boff, const int64_t* rp,
                                const int32_t* col, NextScan N, const int32_t* ctrl);
__global__ void k_classify_rows(int64_t n, const int64_t* rp, int32_t* rows, int64_t base1,
                                int64_t base2, unsigned long long* cur);
__global__ void k_copy_shift(int32_t* dst, const int32_t* src, int64_t count, int32_t delta);
__global__ void k_validate(int64_t n, int64_t nnz, const int64_t* rp, const int32_t* col,
                           int32_t* ctrl);

}  // namespace cbx
