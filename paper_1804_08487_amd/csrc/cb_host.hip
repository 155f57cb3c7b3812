// Host side of the C ABI declared in include/curveball.h: device buffers of
// one graph of independent chains, the launch sequence of a global trade,
// batched rounds captured as a hipGraph, the autotuner, the variant that
// works in the library's static device scratch, error reporting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "curveball.h"
#include "cb_internal.hpp"
#include "cb_kernels.hpp"

using namespace cbx;

namespace {

// Last error message of this thread (a fixed buffer: reporting allocates nothing).
thread_local char g_last_error[512] = {0};
cb_allocator g_allocator = {nullptr, nullptr, nullptr};

cb_status fail(cb_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
  return s;
}

bool hip_ok(hipError_t e, char* msg, size_t cap, const char* what) {
  if (e == hipSuccess) return true;
  snprintf(msg, cap, "%s: %s", what, hipGetErrorString(e));
  return false;
}
#define HIP_OK(expr, what) hip_ok((expr), msg, sizeof(msg), (what))

int bitlen(uint64_t x) { return x ? 64 - __builtin_clzll(x) : 0; }

constexpr int kTimedSteps = 4;

struct EventSet {
  hipEvent_t ev[kTimedSteps + 1];
};

// Matching buckets of a chain of n nodes: a power of two, about 256-511
// nodes each.
int32_t chain_buckets(int64_t n) { return 1 << std::max(0, bitlen((uint64_t)std::max<int64_t>(n, 1)) - 1 - 8); }

}  // namespace

struct cb_graph {
  int64_t n = 0, nnz = 0;
  int32_t L = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  bool static_storage = false;  // buffers carved from the library's static scratch
  cb_allocator alloc{};
  std::vector<void*> owned;

  // chains (one for graph_upload)
  bool batch = false;          // made by batch_upload (or the server): run with batch_run
  int32_t chains = 1;
  std::vector<int64_t> h_node_base, h_nnz_base;   // chains + 1 (batches only), in internal order
  std::vector<int32_t> h_pos;                     // internal position of each caller chain (batches)
  std::vector<uint64_t> h_seed;                   // batches only
  std::vector<uint32_t> h_round;                  // next round of each chain (batches only)
  int64_t* ch_node_base = nullptr;
  int64_t* ch_trade_base = nullptr;
  int32_t* ch_bucket_base = nullptr;
  int32_t* ch_left_base = nullptr;
  uint64_t* ch_seed = nullptr;
  uint32_t* ch_round = nullptr;
  uint32_t* ch_draw_base = nullptr;
  uint32_t* ch_round_saved = nullptr;   // autotuner: rounds before the trial rounds

  int64_t* rp = nullptr;
  int32_t* col = nullptr;
  int32_t* col_t = nullptr;
  int32_t* col_out = nullptr;
  int32_t* inbox = nullptr;
  int32_t* inbox_cur = nullptr;
  int32_t* out_cur = nullptr;
  int32_t* own_cur = nullptr;
  int32_t* perm = nullptr;
  int32_t* trade_of = nullptr;
  int32_t* tinfo = nullptr;
  int32_t* giant_id = nullptr;
  unsigned long long* gbm = nullptr;
  int32_t* gsc = nullptr;
  int32_t ngiant = 0;
  int64_t giant_deg = 0;        // 0: no giant nodes
  bool giant_dirty = false;     // a partial round left bitmap members behind
  int64_t gwords = 0;
  int32_t* mtmp = nullptr;
  uint64_t* mkey = nullptr;
  int32_t* dep = nullptr;
  int32_t* src_list = nullptr;
  int32_t* src_b = nullptr;       // per bucket of relative position: source counts, starts, cursors
  int32_t* tsz = nullptr;
  uint4* ninfo = nullptr;       // per node: row offset, degree, trade information of the round
  HelpJob* jobs = nullptr;
  int64_t* trace = nullptr;     // allocated when tracing is first switched on
  int32_t* qs = nullptr;
  int32_t* qb = nullptr;
  int32_t* bcount = nullptr;
  int32_t* bstart = nullptr;
  int32_t* bcur = nullptr;
  int32_t* ctrl = nullptr;
  unsigned long long* stats = nullptr;
  unsigned long long* row_cur = nullptr;
  uint64_t* slots = nullptr;
  int32_t* sbpre = nullptr;
  int64_t sbpre_stride = 1;
  int32_t* rows = nullptr;      // rebuild size classes: small, then mid, then big rows
  int64_t* big_off = nullptr;   // entries of the big rows laid end to end (n_big + 1)
  int64_t n_small = 0, n_mid = 0, n_big = 0;
  int64_t big_entries = 0;      // entries in the big rows

  int32_t nb = 1;               // matching buckets of all chains
  int keybits_node = 1, keybits_entry = 1;
  int64_t smax = 1;
  int64_t max_deg = 0;
  int64_t slot_elems = 0;
  int cu_count = 1;
  int occupancy_blocks = 1;
  uint64_t ticks_per_ms = 100000;

  // options
  int32_t small_max = kSmallCap;
  int32_t big_lds_max = kBigCap;
  int32_t nbig = 0;          // 0: automatic
  int32_t nbig_alloc = 0;    // slots allocated
  int32_t grid_blocks = 0;   // 0: automatic
  int32_t stack_cap = 8;
  int32_t help_min = kHelpMinItems;
  int32_t help_groups = 2;
  int32_t help_chunk = kHelpChunk;
  int32_t idle_backoff = 128;
  int32_t cu_pool = 1;
  int64_t watchdog_ms = 20000;
  bool timing = false;
  bool debug_checks = false;
  bool tracing = false;
  uint64_t opt_version = 0;  // bumped by every option change (captured rounds bake options in)
  bool fuse_next = true;     // the rebuild also prepares the next round (matching + dependency scan)

  // a round prepared by the previous one's rebuild: its matching, dependency
  // counts, per-entry trade information and giant bitmap seeds are in place
  bool prepared = false;
  uint64_t prep_seed = 0;    // single chain: the (seed, round) it was prepared for
  uint32_t prep_round = 0;

  // batched rounds captured as a graph
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint32_t exec_rounds = 0;
  uint64_t exec_version = 0;
  bool exec_prepared = false;   // the captured rounds start from a prepared round

  bool poisoned = false;
  char poison_msg[384] = {0};

  std::vector<EventSet> pending, spare;
  double ms_acc[kTimedSteps] = {0, 0, 0, 0};
  int64_t rounds_timed = 0;
};

namespace {

void* dev_alloc(cb_graph* g, size_t bytes) {
  if (bytes == 0) bytes = 8;
  void* p = nullptr;
  if (g->alloc.alloc) {
    p = g->alloc.alloc(bytes, g->alloc.user);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
  }
  if (p) g->owned.push_back(p);
  return p;
}

void dev_free_one(cb_graph* g, void* p) {
  if (!p) return;
  for (auto it = g->owned.begin(); it != g->owned.end(); ++it)
    if (*it == p) { g->owned.erase(it); break; }
  if (g->alloc.free) g->alloc.free(p, g->alloc.user); else (void)hipFree(p);
}

void drop_exec(cb_graph* g) {
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  g->exec = nullptr;
  g->graph = nullptr;
  g->exec_rounds = 0;
}

void release_all(cb_graph* g) {
  drop_exec(g);
  for (void* p : g->owned) {
    if (g->alloc.free) g->alloc.free(p, g->alloc.user);
    else (void)hipFree(p);
  }
  g->owned.clear();
  for (auto& s : g->pending)
    for (auto& e : s.ev) (void)hipEventDestroy(e);
  for (auto& s : g->spare)
    for (auto& e : s.ev) (void)hipEventDestroy(e);
  g->pending.clear();
  g->spare.clear();
  if (g->cap_stream) (void)hipStreamDestroy(g->cap_stream);
  g->cap_stream = nullptr;
  if (g->own_stream && g->stream) (void)hipStreamDestroy(g->stream);
  g->stream = nullptr;
}

template <typename T>
bool alloc_into(cb_graph* g, T** out, int64_t count) {
  *out = static_cast<T*>(dev_alloc(g, (size_t)std::max<int64_t>(count, 1) * sizeof(T)));
  return *out != nullptr;
}

int grid_for(int64_t items, int per_block, int cap) {
  int64_t b = (items + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

// The device buffers of a graph, sized from its fields: one list for the
// allocating paths and for carving the static scratch.
constexpr int kMaxBufs = 48;
struct BufPlan {
  void** ptr[kMaxBufs];
  size_t bytes[kMaxBufs];
  int count = 0;
  template <typename T>
  void add(T** p, int64_t elems) {
    ptr[count] = reinterpret_cast<void**>(p);
    bytes[count] = (size_t)std::max<int64_t>(elems, 1) * sizeof(T);
    ++count;
  }
};

void plan_buffers(cb_graph* g, BufPlan& P, bool with_col = true) {
  const int64_t n = g->n, nnz = g->nnz, L1 = std::max<int64_t>(g->L, 1), C = g->chains;
  P.add(&g->rp, n + 1);
  if (with_col) P.add(&g->col, nnz);
  P.add(&g->col_t, nnz);
  P.add(&g->col_out, nnz);
  P.add(&g->inbox, nnz);
  P.add(&g->inbox_cur, n);
  P.add(&g->out_cur, n);
  P.add(&g->own_cur, n);
  P.add(&g->perm, n);
  P.add(&g->trade_of, n);
  P.add(&g->tinfo, n);
  P.add(&g->giant_id, n);
  P.add(&g->mtmp, n);
  P.add(&g->mkey, n);
  P.add(&g->dep, g->L);
  P.add(&g->src_list, g->L);
  P.add(&g->src_b, 3 * kSrcBuckets);
  P.add(&g->tsz, g->L);
  P.add(&g->ninfo, n);
  P.add(&g->jobs, 2 * kMaxJobs);
  P.add(&g->qs, (int64_t)kQsShards * L1);
  P.add(&g->qb, (int64_t)kQbShards * L1);
  P.add(&g->bcount, g->nb);
  P.add(&g->bstart, g->nb + 1);
  P.add(&g->bcur, g->nb);
  P.add(&g->ctrl, kCtrlInts);
  P.add(&g->stats, kStatCount);
  P.add(&g->row_cur, 4);
  P.add(&g->slots, (int64_t)g->nbig_alloc * g->slot_elems);
  P.add(&g->sbpre, (int64_t)g->nbig_alloc * g->sbpre_stride);
  P.add(&g->rows, n);
  P.add(&g->big_off, g->n_big + 1);
  P.add(&g->ch_node_base, C + 1);
  P.add(&g->ch_trade_base, C + 1);
  P.add(&g->ch_bucket_base, C + 1);
  P.add(&g->ch_left_base, C + 1);
  P.add(&g->ch_seed, C);
  P.add(&g->ch_round, C);
  P.add(&g->ch_draw_base, C);
  P.add(&g->ch_round_saved, C);
}

size_t plan_bytes(const BufPlan& P) {
  size_t total = 0;
  for (int i = 0; i < P.count; ++i) total += (P.bytes[i] + 255) & ~(size_t)255;
  return total;
}

bool alloc_plan(cb_graph* g, const BufPlan& P) {
  for (int i = 0; i < P.count; ++i) {
    *P.ptr[i] = dev_alloc(g, P.bytes[i]);
    if (!*P.ptr[i]) return false;
  }
  return true;
}

void carve_plan(const BufPlan& P, char* base) {
  size_t off = 0;
  for (int i = 0; i < P.count; ++i) {
    *P.ptr[i] = base + off;
    off += (P.bytes[i] + 255) & ~(size_t)255;
  }
}

Chains chains_of(const cb_graph* g) {
  Chains c;
  c.count = g->chains;
  c.node_base = g->ch_node_base;
  c.trade_base = g->ch_trade_base;
  c.bucket_base = g->ch_bucket_base;
  c.left_base = g->ch_left_base;
  c.seed = g->ch_seed;
  c.round = g->ch_round;
  c.draw_base = g->ch_draw_base;
  return c;
}

const char* error_bits_text(int32_t bits, char* buf, size_t cap) {
  buf[0] = 0;
  const struct { int32_t bit; const char* name; } names[] = {
      {kErrWatchdog, "watchdog: trade kernel made no progress"},
      {kErrInbox, "inbox overflow"},
      {kErrOut, "output row overflow"},
      {kErrDep, "dependency counter underflow"},
      {kErrGather, "trade input size mismatch"},
      {kErrCapacity, "tier capacity exceeded"},
      {kErrRows, "rebuilt row size differs from degree"},
      {kErrInvalid, "graph is not a simple symmetric sorted CSR"},
      {kErrMatch, "matching bucket overflow"}};
  for (auto& nm : names)
    if (bits & nm.bit) {
      const size_t len = strlen(buf);
      snprintf(buf + len, cap - len, "%s%s", len ? "; " : "", nm.name);
    }
  return buf;
}

// Drain finished timing event sets into the per-step sums.
void collect_timing(cb_graph* g) {
  for (auto& s : g->pending) {
    for (int i = 0; i < kTimedSteps; ++i) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, s.ev[i], s.ev[i + 1]) == hipSuccess) g->ms_acc[i] += ms;
    }
    g->rounds_timed += 1;
    g->spare.push_back(s);
  }
  g->pending.clear();
}

cb_status poison(cb_graph* g, cb_status s, const char* m) {
  g->poisoned = true;
  snprintf(g->poison_msg, sizeof(g->poison_msg), "%s", m);
  return fail(s, "%s", m);
}

cb_status sync_and_check(cb_graph* g) {
  if (g->poisoned) return fail(CB_EPOISONED, "graph handle poisoned: %s", g->poison_msg);
  char msg[256];
  if (!HIP_OK(hipStreamSynchronize(g->stream), "hipStreamSynchronize")) return poison(g, CB_EDEVICE, msg);
  int32_t err = 0;
  if (!HIP_OK(hipMemcpy(&err, g->ctrl + cw(kCwErr), sizeof(int32_t), hipMemcpyDeviceToHost),
              "hipMemcpy(error word)"))
    return poison(g, CB_EDEVICE, msg);
  if (g->timing) collect_timing(g);
  if (err) {
    int32_t dbg[3] = {0, 0, 0};
    for (int i = 0; i < 3; ++i)
      (void)hipMemcpy(&dbg[i], g->ctrl + cw(kCwDbgBits + i), sizeof(int32_t), hipMemcpyDeviceToHost);
    char bits[256], text[384];
    snprintf(text, sizeof(text), "device reported: %s (first: bits %d, trade %d, detail %d)",
             error_bits_text(err, bits, sizeof(bits)), dbg[0], dbg[1] - 1, dbg[2]);
    return poison(g, (err & kErrWatchdog) ? CB_EWATCHDOG : CB_EDEVICE, text);
  }
  return CB_OK;
}

GiantSets giant_sets(const cb_graph* g) {
  GiantSets gs;
  gs.giant_id = g->giant_id;
  gs.bm = g->gbm;
  gs.sc = g->gsc;
  gs.gwords = g->gwords;
  return gs;
}

// Give every node of degree >= deg (0: none) a bitmap neighbour set. Degrees
// never change, so this is fixed until the next call. Bitmaps start empty
// and are left empty by every completed round.
cb_status setup_giants(cb_graph* g, int64_t deg, const int64_t* host_row_ptr) {
  char msg[256];
  if (!HIP_OK(hipStreamSynchronize(g->stream), "sync")) return fail(CB_EDEVICE, "%s", msg);
  drop_exec(g);
  g->prepared = false;   // a prepared round's bitmap seeds and giant bits are for the old sets
  dev_free_one(g, g->gbm);
  dev_free_one(g, g->gsc);
  g->gbm = nullptr;
  g->gsc = nullptr;
  std::vector<int32_t> gid((size_t)std::max<int64_t>(g->n, 1), -1);
  int32_t ng = 0;
  if (deg > 0 && host_row_ptr)
    for (int64_t x = 0; x < g->n; ++x)
      if (host_row_ptr[x + 1] - host_row_ptr[x] >= deg) gid[x] = ng++;
  g->ngiant = ng;
  g->giant_deg = ng ? deg : 0;
  g->gwords = ((g->n + 4095) / 4096) * 64;
  if (!HIP_OK(hipMemcpyAsync(g->giant_id, gid.data(), gid.size() * sizeof(int32_t), hipMemcpyHostToDevice, g->stream), "copy giant ids") ||
      !HIP_OK(hipStreamSynchronize(g->stream), "sync"))
    return fail(CB_EDEVICE, "%s", msg);
  if (ng == 0) return CB_OK;
  if (!alloc_into(g, &g->gbm, (int64_t)ng * g->gwords) || !alloc_into(g, &g->gsc, (int64_t)ng * (g->gwords >> 6))) {
    dev_free_one(g, g->gbm);
    g->gbm = nullptr;
    g->ngiant = 0;
    g->giant_deg = 0;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(g->n, 256, 4096)), dim3(256), 0, g->stream, g->giant_id, g->n, -1);
    (void)hipStreamSynchronize(g->stream);
    return fail(CB_ENOMEM, "no device memory for giant bitmaps");
  }
  // cleared on the graph's own stream (a non-blocking stream is not ordered
  // after work on the null stream)
  if (!HIP_OK(hipMemsetAsync(g->gbm, 0, (size_t)ng * g->gwords * 8, g->stream), "clear bitmaps") ||
      !HIP_OK(hipMemsetAsync(g->gsc, 0, (size_t)ng * (g->gwords >> 6) * 4, g->stream), "clear counts") ||
      !HIP_OK(hipStreamSynchronize(g->stream), "sync"))
    return fail(CB_EDEVICE, "%s", msg);
  return CB_OK;
}

int32_t effective_nbig(const cb_graph* g) {
  int32_t v = g->nbig > 0 ? g->nbig : std::max(1, g->cu_count / 4);
  return std::min(v, g->nbig_alloc);
}

// Workgroups of the trade kernel. Automatic: one per CU; for a dense graph
// (average degree at least 32) with giant nodes, the workgroup workers plus a
// quarter of the CUs. There a chain of giant trades is bound by the round
// trips of its scattered accesses, and wavefront workers on every CU add
// enough traffic to lengthen them: at n = 2^24, average degree 100, the trade
// kernel took 733 ms on 256 workgroups, 615 ms on 128 (64 + 64) and 636 ms on
// 112. Sparse graphs are mostly wavefront trades and need every worker (a
// sparse 2^24-node graph with a few giants: 129 ms per round on 256
// workgroups, 184 ms on 128), as does a batch of 512 small chains (80 ms on
// 256, 113 ms on 128).
int32_t trade_grid(const cb_graph* g) {
  int32_t blocks = g->grid_blocks;
  if (blocks <= 0) {
    const bool dense_giants = g->ngiant > 0 && g->nnz >= 32 * g->n;
    blocks = dense_giants ? effective_nbig(g) + std::max(1, g->cu_count / 4) : g->cu_count * g->occupancy_blocks;
  }
  return std::max(blocks, effective_nbig(g) + 1);
}

// Trades above this size run on a workgroup (a giant node never runs on a
// wavefront).
int32_t effective_small_max(const cb_graph* g) {
  return g->giant_deg > 0 ? (int32_t)std::min<int64_t>(g->small_max, g->giant_deg - 1) : g->small_max;
}

// Arguments of the trade kernel for the trades 0..L-1 of the current matching.
TradeArgs trade_args(const cb_graph* g, int32_t L) {
  TradeArgs A{};
  A.rp = g->rp;
  A.col = g->col;
  A.col_t = g->col_t;
  A.tinfo = g->tinfo;
  A.gs = giant_sets(g);
  A.perm = g->perm;
  A.inbox = g->inbox;
  A.inbox_cur = g->inbox_cur;
  A.col_out = g->col_out;
  A.out_cur = g->out_cur;
  A.own_cur = g->own_cur;
  A.dep = g->dep;
  A.src_list = g->src_list;
  A.tsz = g->tsz;
  A.ninfo = g->ninfo;
  A.jobs = g->jobs;
  A.trace = g->tracing ? g->trace : nullptr;
  A.qs = g->qs;
  A.qb = g->qb;
  A.ctrl = g->ctrl;
  A.stats = g->stats;
  A.slots = g->slots;
  A.slot_elems = g->slot_elems;
  A.sbpre = g->sbpre;
  A.sbpre_stride = g->sbpre_stride;
  A.smax = g->smax;
  A.n = g->n;
  A.L = L;
  A.small_max = effective_small_max(g);
  A.help_min = g->help_min;
  A.help_groups = g->help_groups;
  A.help_chunk = g->help_chunk;
  A.idle_backoff = g->idle_backoff;
  A.cu_pool = g->cu_pool;
  A.big_lds_max = g->big_lds_max;
  A.nbig = effective_nbig(g);
  A.stack_cap = g->stack_cap;
  A.keybits = g->keybits_entry;
  A.ch = chains_of(g);
  A.watchdog_ticks = (uint64_t)g->watchdog_ms * g->ticks_per_ms;
  return A;
}

// Forget a prepared round (its bitmap seeds are cleared before the next scan).
void unprepare(cb_graph* g) {
  if (g->prepared && g->ngiant > 0) g->giant_dirty = true;
  g->prepared = false;
}

// Matching kernels of the round in the chain table (keys, buckets, pairs,
// trade_of, tinfo, zeroed dep).
void enqueue_matching(cb_graph* g, hipStream_t st) {
  const int64_t n = g->n;
  const Chains ch = chains_of(g);
  hipLaunchKernelGGL(k_match_count, dim3(grid_for(n, 256, 16384)), dim3(256), 0, st, n, ch, g->bcount, g->ctrl);
  hipLaunchKernelGGL(k_match_scan, dim3(1), dim3(1024), 0, st, g->nb, g->bcount, g->bstart, g->ctrl);
  hipLaunchKernelGGL(k_match_scatter, dim3(grid_for(n, 256, 16384)), dim3(256), 0, st, n, ch, g->bstart,
                     g->bcur, g->mtmp, g->ctrl);
  hipLaunchKernelGGL(k_match_sort, dim3(std::min<int32_t>(g->nb, 1 << 20)), dim3(kMatchBlock), 0, st,
                     ch, g->nb, g->bstart, g->mtmp, g->mkey, g->perm, g->trade_of, g->tinfo, g->giant_id,
                     g->dep, g->ctrl);
}

// Enqueue the steps 1..last_step of one global trade of every chain on `st`,
// with the seeds and rounds in the chain table; `advance` adds one to every
// chain's round afterwards. A round prepared by the previous one starts at
// its sources. A full round prepares the next one when fusion is on: the
// next round's matching needs no graph data (it only overwrites this round's
// matching, dead once the trade kernel is done), and the rebuild then scans
// every row it writes for the next round; a single chain is prepared for
// (seed, round + 1), set by `next_seed`/`next_round`. No host
// synchronisation and no memset when nothing is left over from a partial
// round, so the sequence can be captured into a graph (without timing or
// tracing).
cb_status enqueue_round(cb_graph* g, hipStream_t st, int last_step, bool advance,
                        bool single_next = false, uint64_t next_seed = 0, uint32_t next_round = 0) {
  if (g->poisoned) return fail(CB_EPOISONED, "graph handle poisoned: %s", g->poison_msg);
  if (last_step < CB_STEP_MATCHING || last_step > CB_STEP_REBUILD)
    return fail(CB_EINVAL, "last_step out of range");
  if (g->n == 0) {
    if (advance) hipLaunchKernelGGL(k_advance_rounds, dim3(grid_for(g->chains, 256, 64)), dim3(256), 0, st,
                                    g->ch_round, g->chains, 1u);
    return CB_OK;
  }
  char msg[256];
  EventSet evs{};
  const bool timed = g->timing && last_step == CB_STEP_REBUILD;
  if (timed) {
    if (!g->spare.empty()) {
      evs = g->spare.back();
      g->spare.pop_back();
    } else {
      for (auto& e : evs.ev)
        if (hipEventCreate(&e) != hipSuccess) return fail(CB_EDEVICE, "hipEventCreate failed");
    }
    (void)hipEventRecord(evs.ev[0], st);
  }
  const int64_t n = g->n;
  const int32_t L = g->L;
  const Chains ch = chains_of(g);
  const bool from_prepared = g->prepared && last_step == CB_STEP_REBUILD;
  if (!from_prepared) unprepare(g);
  g->prepared = false;
  if (g->giant_dirty) {
    if (!HIP_OK(hipMemsetAsync(g->gbm, 0, (size_t)g->ngiant * g->gwords * 8, st), "clear bitmaps") ||
        !HIP_OK(hipMemsetAsync(g->gsc, 0, (size_t)g->ngiant * (g->gwords >> 6) * 4, st), "clear counts"))
      return fail(CB_EDEVICE, "%s", msg);
    g->giant_dirty = false;
  }
  if (last_step < CB_STEP_TRADE && g->ngiant > 0) g->giant_dirty = true;

  hipLaunchKernelGGL(k_round_reset, dim3(grid_for(std::max<int64_t>({n, (int64_t)g->nb, (int64_t)kCwCount}), 256, 8192)),
                     dim3(256), 0, st, n, g->nb, g->inbox_cur, g->out_cur, g->own_cur, g->bcount,
                     g->bcur, g->ctrl, g->stats, 1);
  // 1. matching
  if (!from_prepared) enqueue_matching(g, st);
  if (timed) (void)hipEventRecord(evs.ev[1], st);
  if (g->debug_checks && g->ngiant > 0 && !from_prepared)
    hipLaunchKernelGGL(k_check_giants_empty, dim3(1024), dim3(256), 0, st,
                       (int64_t)g->ngiant * (g->gwords >> 6), g->gsc, g->ctrl);
  if (last_step >= CB_STEP_DEPSCAN) {
    // 2. dependency scan + sources
    if (g->nnz > 0 && !from_prepared)
      hipLaunchKernelGGL(k_depscan, dim3((unsigned)((g->nnz + kScanChunk - 1) / kScanChunk)), dim3(256),
                         0, st, n, g->nnz, g->rp, g->col, g->trade_of, g->tinfo, g->col_t, g->dep,
                         giant_sets(g), g->ctrl);
    if (L > 0) {
      for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(k_sources, dim3(grid_for(L, 256, 8192)), dim3(256), 0, st, L, g->dep,
                           g->perm, g->rp, effective_small_max(g), g->tsz, g->src_list, g->qb,
                           g->ctrl, g->stats, ch, g->src_b, pass);
        if (pass == 0)
          hipLaunchKernelGGL(k_sources_scan, dim3(1), dim3(kSrcBuckets), 0, st, g->src_b, g->ctrl);
      }
    }
  }
  if (timed) (void)hipEventRecord(evs.ev[2], st);
  if (last_step >= CB_STEP_TRADE && L > 0) {
    // 3. trades
    if (g->tracing) {
      if (!HIP_OK(hipMemsetAsync(g->trace, 0xFF, (size_t)L * kTraceFields * sizeof(int64_t), st), "clear trace"))
        return fail(CB_EDEVICE, "%s", msg);
    }
    hipLaunchKernelGGL(k_node_info, dim3(grid_for(n, 256, 8192)), dim3(256), 0, st, n, g->rp, g->tinfo, g->ninfo);
    const TradeArgs A = trade_args(g, L);
    hipLaunchKernelGGL(k_trade, dim3(trade_grid(g)), dim3(kTradeBlock), 0, st, A);
  }
  if (timed) (void)hipEventRecord(evs.ev[3], st);
  if (last_step >= CB_STEP_TRADE && L > 0)
    hipLaunchKernelGGL(k_check_rows, dim3(grid_for(n, 256, 8192)), dim3(256), 0, st, n, g->rp,
                       g->out_cur, g->own_cur, g->ctrl);
  if (advance)
    hipLaunchKernelGGL(k_advance_rounds, dim3(grid_for(g->chains, 256, 64)), dim3(256), 0, st, g->ch_round,
                       g->chains, 1u);
  // the next round's matching, before the rebuild that scans for it
  const bool lookahead = last_step == CB_STEP_REBUILD && g->fuse_next && (advance || single_next);
  NextScan N{};
  if (lookahead) {
    if (single_next)
      hipLaunchKernelGGL(k_set_chain, dim3(1), dim3(64), 0, st, g->ch_seed, g->ch_round, 0, next_seed, next_round);
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(g->nb, 256, 1024)), dim3(256), 0, st, g->bcount, (int64_t)g->nb, 0);
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(g->nb, 256, 1024)), dim3(256), 0, st, g->bcur, (int64_t)g->nb, 0);
    enqueue_matching(g, st);
    N.tinfo = g->tinfo;
    N.trade_of = g->trade_of;
    N.col_t = g->col_t;
    N.dep = g->dep;
    N.gs = giant_sets(g);
  }
  if (last_step >= CB_STEP_REBUILD && g->nnz > 0) {
    // 4. rebuild: per-row ascending sort of col_out into col (+ the next round's scan)
    const int32_t* rs = g->rows;
    const int32_t* rm = g->rows + g->n_small;
    const int32_t* rb = g->rows + g->n_small + g->n_mid;
    if (g->n_small)
      hipLaunchKernelGGL(k_segsort_small, dim3(grid_for(g->n_small, 4, 65536)), dim3(256), 0, st,
                         rs, g->n_small, g->rp, g->col_out, g->col, N, g->ctrl);
    if (g->n_mid)
      hipLaunchKernelGGL(k_segsort_mid, dim3(grid_for(g->n_mid, 1, 65536)), dim3(256), 0, st,
                         rm, g->n_mid, g->rp, g->col_out, g->col, g->keybits_node, N, g->ctrl);
    if (g->n_big) {
      hipLaunchKernelGGL(k_segsort_wide, dim3(grid_for(g->n_big, 1, 4096)), dim3(kSegWideThreads), 0, st,
                         rb, g->n_big, g->rp, g->col_out, g->col, g->keybits_node, g->ctrl);
      hipLaunchKernelGGL(k_segsort_huge, dim3(grid_for(g->n_big, 1, 4096)), dim3(kSegWideThreads), 0, st,
                         rb, g->n_big, g->rp, g->col_out, g->col, g->keybits_node, g->ctrl);
      if (lookahead) {
        hipLaunchKernelGGL(k_scan_big_rows, dim3((unsigned)std::max<int64_t>(1, (g->big_entries + kScanChunk - 1) / kScanChunk)),
                           dim3(256), 0, st, rb, g->n_big, g->big_off, g->rp, g->col, N, g->ctrl);
      }
    }
  }
  if (lookahead) {
    g->prepared = true;
    g->prep_seed = next_seed;
    g->prep_round = next_round;
  }
  if (timed) {
    (void)hipEventRecord(evs.ev[4], st);
    g->pending.push_back(evs);
  }
  if (!HIP_OK(hipGetLastError(), "kernel launch")) return poison(g, CB_EDEVICE, msg);
  return CB_OK;
}


// Device properties and occupancy of the trade kernel, once per device.
struct DeviceInfo {
  int cu_count = 1;
  int occupancy = 1;
  uint64_t ticks_per_ms = 100000;
};
constexpr int kMaxDevices = 64;
DeviceInfo device_info(int dev) {
  static std::mutex mu;
  static DeviceInfo known[kMaxDevices];
  static bool have[kMaxDevices] = {false};
  std::lock_guard<std::mutex> lock(mu);
  const bool cacheable = dev >= 0 && dev < kMaxDevices;
  if (cacheable && have[dev]) return known[dev];
  DeviceInfo d;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess) d.cu_count = prop.multiProcessorCount;
  int rate_khz = 0;
  if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && rate_khz > 0)
    d.ticks_per_ms = (uint64_t)rate_khz;
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void*>(k_trade), kTradeBlock, 0) ==
          hipSuccess && occ > 0)
    d.occupancy = occ;
  if (cacheable) {
    known[dev] = d;
    have[dev] = true;
  }
  return d;
}

// Host checks of one chain's CSR (the device validation checks the rest).
cb_status check_chain_host(const ChainSrc& c, int64_t* d1, int64_t* d2) {
  if (c.n < 0 || c.n > INT32_MAX) return fail(CB_EINVAL, "n must be in [0, 2^31 - 1]");
  if (!c.rp) return fail(CB_EINVAL, "row_ptr is NULL");
  if (c.rp[0] != 0) return fail(CB_EINVAL, "row_ptr[0] must be 0");
  for (int64_t x = 0; x < c.n; ++x) {
    const int64_t d = c.rp[x + 1] - c.rp[x];
    if (d < 0) return fail(CB_EINVAL, "row_ptr is not monotone");
    if (d >= c.n && d > 0) return fail(CB_ENOTSIMPLE, "a row has more entries than other nodes");
    if (d > *d1) { *d2 = *d1; *d1 = d; } else if (d > *d2) { *d2 = d; }
  }
  const int64_t nnz = c.rp[c.n];
  if (nnz % 2) return fail(CB_ENOTSIMPLE, "odd number of entries cannot be symmetric");
  if (nnz >= INT32_MAX) return fail(CB_EINVAL, "2m must be below 2^31");
  if (nnz > 0 && !c.col) return fail(CB_EINVAL, "col is NULL");
  return CB_OK;
}

// Sizes, tier limits and chain tables of a new graph (no device work).
void size_graph(cb_graph* g, const ChainSrc* src, int32_t count, int64_t d1, int64_t d2) {
  g->chains = count;
  int64_t n = 0, nnz = 0, L = 0, nb = 0;
  for (int32_t c = 0; c < count; ++c) {
    n += src[c].n;
    nnz += src[c].rp[src[c].n];
    L += src[c].n / 2;
    nb += chain_buckets(src[c].n);
  }
  g->n = n;
  g->nnz = nnz;
  g->L = (int32_t)L;
  g->nb = (int32_t)nb;
  g->max_deg = d1;
  g->keybits_node = std::max(1, bitlen((uint64_t)std::max<int64_t>(n - 1, 1)));
  g->keybits_entry = std::max(1, bitlen((uint64_t)std::max<int64_t>(2 * n - 1, 1)));
  g->smax = std::max<int64_t>(d1 + d2, 1);
  g->slot_elems = 3 * g->smax + g->smax / 2 + 1;
  g->sbpre_stride = (n + 4095) / 4096 + 1;
}

// Rows per rebuild size class.
void count_classes(cb_graph* g, const ChainSrc* src, int32_t count) {
  g->n_small = g->n_mid = g->n_big = 0;
  g->big_entries = 0;
  for (int32_t c = 0; c < count; ++c)
    for (int64_t x = 0; x < src[c].n; ++x) {
      const int64_t d = src[c].rp[x + 1] - src[c].rp[x];
      if (d == 0) continue;
      if (d <= kSegSmallMax) ++g->n_small;
      else if (d <= kSegMidMax) ++g->n_mid;
      else { ++g->n_big; g->big_entries += d; }
    }
}

// Device state that every new graph starts from: cleared control words, jobs
// and queues, the rebuild's row lists, and (optionally) validation.
bool init_device_state(cb_graph* g, bool validate, char* msg, size_t cap) {
  hipStream_t st = g->stream;
  const int64_t L1 = std::max<int64_t>(g->L, 1);
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(256), 0, st, g->ctrl, (int64_t)kCtrlInts, 0);
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(256), 0, st, g->src_b, (int64_t)(3 * kSrcBuckets), 0);
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for((int64_t)(2 * kMaxJobs * sizeof(HelpJob) / 4), 256, 64)), dim3(256), 0, st,
                     reinterpret_cast<int32_t*>(g->jobs), (int64_t)(2 * kMaxJobs * sizeof(HelpJob) / 4), 0);
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for((int64_t)kQsShards * L1, 256, 8192)), dim3(256), 0, st, g->qs,
                     (int64_t)kQsShards * L1, -1);
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for((int64_t)kQbShards * L1, 256, 8192)), dim3(256), 0, st, g->qb,
                     (int64_t)kQbShards * L1, -1);
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(g->n, 256, 8192)), dim3(256), 0, st, g->giant_id, g->n, -1);
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, reinterpret_cast<int32_t*>(g->row_cur), (int64_t)8, 0);
  if (g->n > 0)
    hipLaunchKernelGGL(k_classify_rows, dim3(grid_for(g->n, 256, 8192)), dim3(256), 0, st, g->n, g->rp, g->rows,
                       g->n_small, g->n_small + g->n_mid, g->row_cur);
  if (g->n_big > 0)
    hipLaunchKernelGGL(k_big_offsets, dim3(1), dim3(1024), 0, st, g->rows + g->n_small + g->n_mid, g->n_big, g->rp,
                       g->big_off);
  if (validate && g->nnz > 0)
    hipLaunchKernelGGL(k_validate, dim3((unsigned)((g->nnz + kScanChunk - 1) / kScanChunk)), dim3(256), 0, st,
                       g->n, g->nnz, g->rp, g->col, g->ctrl);
  if (!hip_ok(hipGetLastError(), msg, cap, "init launch")) return false;
  if (!hip_ok(hipStreamSynchronize(st), msg, cap, "upload sync")) return false;
  unsigned long long placed[3] = {0, 0, 0};
  if (!hip_ok(hipMemcpy(placed, g->row_cur, sizeof(placed), hipMemcpyDeviceToHost), msg, cap, "read row counts"))
    return false;
  if ((int64_t)placed[0] != g->n_small || (int64_t)placed[1] != g->n_mid || (int64_t)placed[2] != g->n_big) {
    snprintf(msg, cap, "row classes differ from the host's count");
    return false;
  }
  return true;
}

// Read the error word after upload validation: CB_OK or CB_ENOTSIMPLE.
cb_status upload_check_status(cb_graph* g) {
  int32_t err = 0;
  char msg[256];
  if (!HIP_OK(hipMemcpy(&err, g->ctrl + cw(kCwErr), sizeof(int32_t), hipMemcpyDeviceToHost), "read error word"))
    return fail(CB_EDEVICE, "%s", msg);
  if (err) {
    char bits[256];
    return fail(CB_ENOTSIMPLE, "upload validation: %s", error_bits_text(err, bits, sizeof(bits)));
  }
  return CB_OK;
}

// Default giant threshold: max(6144, n / 2048) for one chain; reading a
// giant's set back costs n / 8 bytes of bitmap whatever its degree, sorting a
// list costs in proportion to the degree; measured on MI355X a round at
// n = 2^24 is fastest near degree n / 2048 (8192; 2% faster than 16384, 12%
// faster than 24576), and 6144 keeps every pair below it within one
// workgroup's LDS (at n = 2^22, 4096 was 1% slower than 6144). It rises
// further if the bitmaps would take too much memory. Batches of chains start
// without giant nodes (their bitmaps would span every chain's ids).
int64_t default_giant_threshold(const cb_graph* g, const int64_t* rp) {
  if (g->batch) return 0;
  const int64_t n = g->n;
  const int64_t min_deg = std::max<int64_t>(kGiantMinDeg, n / 2048);
  size_t free_b = 0, total_b = 0;
  (void)hipMemGetInfo(&free_b, &total_b);
  const double budget = std::min(64.0 * (1ull << 30), 0.4 * (double)free_b);
  const int64_t gwords = ((n + 4095) / 4096) * 64;
  const double per_giant = (double)gwords * 8.0 + (double)(gwords >> 6) * 4.0;
  std::vector<int64_t> degs;
  for (int64_t x = 0; x < n; ++x) {
    const int64_t d = rp[x + 1] - rp[x];
    if (d >= min_deg) degs.push_back(d);
  }
  std::sort(degs.begin(), degs.end(), std::greater<int64_t>());
  const int64_t fit = (int64_t)(budget / per_giant);
  int64_t thr = min_deg;
  if ((int64_t)degs.size() > fit) thr = fit > 0 ? degs[(size_t)fit - 1] + 1 : INT64_MAX;
  if (thr == INT64_MAX || degs.empty()) thr = 0;
  return thr;
}

}  // namespace

// Create a graph of `count` chains in allocated device memory.
cb_status cbx::create_graph(const ChainSrc* src_in, int32_t count, void* stream, uint32_t flags, bool batch,
                            cb_graph** out) {
  if (!out) return fail(CB_EINVAL, "out is NULL");
  *out = nullptr;
  if (count < 1) return fail(CB_EINVAL, "a graph needs at least one chain");
  // A batch lays its chains out largest first: their sources are handed out
  // first and their dependency chains, the longest, start earliest. Each
  // chain's result does not depend on where it sits.
  std::vector<int32_t> order((size_t)count);
  for (int32_t c = 0; c < count; ++c) order[c] = c;
  if (batch)
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
      return src_in[a].rp[src_in[a].n] > src_in[b].rp[src_in[b].n];
    });
  std::vector<ChainSrc> sorted_src((size_t)count);
  for (int32_t i = 0; i < count; ++i) sorted_src[i] = src_in[order[i]];
  const ChainSrc* src = sorted_src.data();
  int64_t d1 = 0, d2 = 0, n_total = 0, nnz_total = 0;
  for (int32_t c = 0; c < count; ++c) {
    cb_status s = check_chain_host(src[c], &d1, &d2);
    if (s != CB_OK) return s;
    n_total += src[c].n;
    nnz_total += src[c].rp[src[c].n];
  }
  if (n_total > INT32_MAX) return fail(CB_EINVAL, "the chains hold more than 2^31 - 1 nodes");
  if (nnz_total >= INT32_MAX) return fail(CB_EINVAL, "the chains hold 2^31 or more entries");
  if (n_total / 2 > INT32_MAX / 2) return fail(CB_EINVAL, "too many trades");
  // ids of every chain within its own range (batches; one chain is checked on the device)
  if (count > 1)
    for (int32_t c = 0; c < count; ++c) {
      if (src[c].col_on_device) continue;
      const int64_t e = src[c].rp[src[c].n];
      for (int64_t i = 0; i < e; ++i)
        if (src[c].col[i] < 0 || src[c].col[i] >= src[c].n)
          return fail(CB_ENOTSIMPLE, "chain %d: a neighbour id is outside [0, n)", (int)order[c]);
    }

  cb_graph* g = new cb_graph();
  g->alloc = g_allocator;
  g->batch = batch;
  char msg[256];
  if (!HIP_OK(hipGetDevice(&g->device), "hipGetDevice")) { delete g; return fail(CB_EDEVICE, "%s", msg); }
  if (stream) {
    g->stream = (hipStream_t)stream;
  } else {
    if (!HIP_OK(hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking), "hipStreamCreate")) {
      delete g;
      return fail(CB_EDEVICE, "%s", msg);
    }
    g->own_stream = true;
  }
  const DeviceInfo di = device_info(g->device);
  g->cu_count = di.cu_count;
  g->occupancy_blocks = di.occupancy;
  g->ticks_per_ms = di.ticks_per_ms;
  g->nbig_alloc = std::max(1, g->cu_count / 2);
  size_graph(g, src, count, d1, d2);
  count_classes(g, src, count);

  // chain tables and the union's offsets on the host
  std::vector<int64_t> node_base(count + 1), trade_base(count + 1), nnz_base(count + 1);
  std::vector<int32_t> bucket_base(count + 1), left_base(count + 1);
  std::vector<uint64_t> seeds(count);
  std::vector<uint32_t> rounds(count), draw(count, 0);
  for (int32_t c = 0; c < count; ++c) {
    node_base[c + 1] = node_base[c] + src[c].n;
    trade_base[c + 1] = trade_base[c] + src[c].n / 2;
    nnz_base[c + 1] = nnz_base[c] + src[c].rp[src[c].n];
    bucket_base[c + 1] = bucket_base[c] + chain_buckets(src[c].n);
    left_base[c + 1] = left_base[c] + (int32_t)(src[c].n & 1);
    seeds[c] = src[c].seed;
    rounds[c] = src[c].round;
  }
  BufPlan P;
  plan_buffers(g, P);
  if (!alloc_plan(g, P)) {
    release_all(g);
    delete g;
    return fail(CB_ENOMEM, "device allocation failed");
  }
  hipStream_t st = g->stream;
  bool ok = true;
  std::vector<int64_t> urp;   // the union's offsets (batches)
  const int64_t* rp_host = src[0].rp;
  if (count > 1) {
    urp.resize((size_t)g->n + 1);
    for (int32_t c = 0; c < count; ++c)
      for (int64_t x = 0; x <= src[c].n; ++x) urp[(size_t)(node_base[c] + x)] = nnz_base[c] + src[c].rp[x];
    rp_host = urp.data();
  }
  ok = HIP_OK(hipMemcpyAsync(g->rp, rp_host, (size_t)(g->n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st), "copy row_ptr");
  for (int32_t c = 0; ok && c < count; ++c) {
    const int64_t e = src[c].rp[src[c].n];
    if (e == 0) continue;
    int32_t* dst = g->col + nnz_base[c];
    if (src[c].col_on_device) {
      hipLaunchKernelGGL(k_copy_shift, dim3(grid_for(e, 256, 8192)), dim3(256), 0, st, dst, src[c].col, e,
                         (int32_t)(node_base[c] - src[c].dev_shift));
    } else {
      ok = HIP_OK(hipMemcpyAsync(dst, src[c].col, (size_t)e * sizeof(int32_t), hipMemcpyHostToDevice, st), "copy col");
      if (ok && node_base[c] != 0)
        hipLaunchKernelGGL(k_copy_shift, dim3(grid_for(e, 256, 8192)), dim3(256), 0, st, dst, dst, e,
                           (int32_t)node_base[c]);
    }
  }
  ok = ok &&
       HIP_OK(hipMemcpyAsync(g->ch_node_base, node_base.data(), node_base.size() * 8, hipMemcpyHostToDevice, st), "copy chains") &&
       HIP_OK(hipMemcpyAsync(g->ch_trade_base, trade_base.data(), trade_base.size() * 8, hipMemcpyHostToDevice, st), "copy chains") &&
       HIP_OK(hipMemcpyAsync(g->ch_bucket_base, bucket_base.data(), bucket_base.size() * 4, hipMemcpyHostToDevice, st), "copy chains") &&
       HIP_OK(hipMemcpyAsync(g->ch_left_base, left_base.data(), left_base.size() * 4, hipMemcpyHostToDevice, st), "copy chains") &&
       HIP_OK(hipMemcpyAsync(g->ch_seed, seeds.data(), seeds.size() * 8, hipMemcpyHostToDevice, st), "copy chains") &&
       HIP_OK(hipMemcpyAsync(g->ch_round, rounds.data(), rounds.size() * 4, hipMemcpyHostToDevice, st), "copy chains") &&
       HIP_OK(hipMemcpyAsync(g->ch_draw_base, draw.data(), draw.size() * 4, hipMemcpyHostToDevice, st), "copy chains");
  if (ok) ok = init_device_state(g, (flags & CB_VALIDATE) != 0, msg, sizeof(msg));
  if (!ok) {
    release_all(g);
    delete g;
    return fail(CB_EDEVICE, "%s", msg);
  }
  cb_status s = upload_check_status(g);
  if (s == CB_OK) s = setup_giants(g, default_giant_threshold(g, rp_host), rp_host);
  if (s != CB_OK) {
    release_all(g);
    delete g;
    return s;
  }
  g->batch = batch;
  if (batch) {
    g->h_node_base = node_base;
    g->h_nnz_base = nnz_base;
    g->h_seed = seeds;
    g->h_round = rounds;
    g->h_pos.assign((size_t)count, 0);
    for (int32_t i = 0; i < count; ++i) g->h_pos[order[i]] = i;
  }
  *out = g;
  return CB_OK;
}

cb_status cbx::set_error(cb_status s, const char* msg) { return fail(s, "%s", msg); }

// Device bytes a graph of these chains allocates (before giant bitmaps).
size_t cbx::graph_bytes(const ChainSrc* src, int32_t count) {
  cb_graph g;
  int64_t d1 = 0, d2 = 0;
  for (int32_t c = 0; c < count; ++c)
    for (int64_t x = 0; x < src[c].n; ++x) {
      const int64_t d = src[c].rp[x + 1] - src[c].rp[x];
      if (d > d1) { d2 = d1; d1 = d; } else if (d > d2) { d2 = d; }
    }
  int dev = 0;
  (void)hipGetDevice(&dev);
  g.cu_count = device_info(dev).cu_count;
  g.nbig_alloc = std::max(1, g.cu_count / 2);
  size_graph(&g, src, count, d1, d2);
  BufPlan P;
  plan_buffers(&g, P);
  return plan_bytes(P);
}

// Chain c's adjacency in device memory (global ids: local + *node_base).
int32_t* cbx::chain_col(cb_graph* g, int32_t c, int64_t* node_base) {
  if (!g->batch) {
    *node_base = 0;
    return g->col;
  }
  const int32_t i = g->h_pos[c];
  *node_base = g->h_node_base[i];
  return g->col + g->h_nnz_base[i];
}

namespace {

// ---------------------------------------------------------------- autotuner

struct TuneKey {
  int chains_lg, n_lg, nnz_lg, deg_lg;
  bool operator<(const TuneKey& o) const {
    return std::tie(chains_lg, n_lg, nnz_lg, deg_lg) < std::tie(o.chains_lg, o.n_lg, o.nnz_lg, o.deg_lg);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, cb_tune_result> g_tune_cache;

TuneKey tune_key(const cb_graph* g) {
  return TuneKey{bitlen((uint64_t)g->chains), bitlen((uint64_t)g->n), bitlen((uint64_t)g->nnz),
                 bitlen((uint64_t)g->max_deg)};
}

void apply_tuned(cb_graph* g, const cb_tune_result& r) {
  g->small_max = r.small_max;
  g->help_min = r.help_min;
  g->help_chunk = r.help_chunk;
  g->nbig = r.big_workers;
  g->stack_cap = r.local_stack;
  g->idle_backoff = r.idle_backoff;
  g->cu_pool = r.cu_pool;
  g->grid_blocks = r.grid_blocks;
  g->opt_version++;
}

cb_tune_result current_options(const cb_graph* g) {
  cb_tune_result r{};
  r.small_max = g->small_max;
  r.help_min = g->help_min;
  r.help_chunk = g->help_chunk;
  r.big_workers = effective_nbig(g);
  r.local_stack = g->stack_cap;
  r.idle_backoff = g->idle_backoff;
  r.cu_pool = g->cu_pool;
  r.grid_blocks = g->grid_blocks;
  return r;
}

// Philox4x32-10 on the host (the node pairs of single trades are drawn
// here); the same convention as the device's philox64.
uint64_t host_philox64(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3) {
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c0 = n0;
    c1 = (uint32_t)p1;
    c2 = n2;
    c3 = (uint32_t)p0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return ((uint64_t)c1 << 32) | c0;
}
uint64_t host_bounded(uint64_t x, uint64_t k) { return (uint64_t)(((unsigned __int128)x * k) >> 64); }

constexpr uint32_t kTagPair = 0x43425550u;   // node pair of a single trade
constexpr uint32_t kSingleRound = 0xFFFFFFFFu;   // round word of a single trade's split draws

}  // namespace

extern "C" {

cb_status cb_set_allocator(const cb_allocator* a) {
  if (a && (!a->alloc || !a->free)) return fail(CB_EINVAL, "allocator needs alloc and free");
  g_allocator = a ? *a : cb_allocator{nullptr, nullptr, nullptr};
  return CB_OK;
}

const char* cb_last_error(void) { return g_last_error; }

cb_status graph_upload(int64_t n, const int64_t* row_ptr, const int32_t* col, void* stream,
                       uint32_t flags, cb_graph** out) {
  if (!out) return fail(CB_EINVAL, "out is NULL");
  if (n < 0 || n > INT32_MAX) return fail(CB_EINVAL, "n must be in [0, 2^31 - 1]");
  ChainSrc c{n, row_ptr, col, false, 0, 0, 0};
  return create_graph(&c, 1, stream, flags, false, out);
}

cb_status graph_info(const cb_graph* g, int64_t* n, int64_t* nnz) {
  if (!g) return fail(CB_EINVAL, "null graph");
  if (n) *n = g->n;
  if (nnz) *nnz = g->nnz;
  return CB_OK;
}

cb_status global_trade(cb_graph* g, uint64_t seed, uint32_t round) {
  if (!g) return fail(CB_EINVAL, "null graph");
  if (g->batch) return fail(CB_EINVAL, "global_trade needs a graph from graph_upload (use batch_run)");
  if (g->poisoned) return fail(CB_EPOISONED, "graph handle poisoned: %s", g->poison_msg);
  if (g->prepared && (g->prep_seed != seed || g->prep_round != round)) unprepare(g);
  if (!g->prepared)
    hipLaunchKernelGGL(k_set_chain, dim3(1), dim3(64), 0, g->stream, g->ch_seed, g->ch_round, 0, seed, round);
  // prepare (seed, round + 1), the round a chain applies next
  return enqueue_round(g, g->stream, CB_STEP_REBUILD, false, round != UINT32_MAX, seed, round + 1u);
}

cb_status global_trade_steps(cb_graph* g, uint64_t seed, uint32_t round, int32_t last_step) {
  if (!g) return fail(CB_EINVAL, "null graph");
  if (g->batch) return fail(CB_EINVAL, "global_trade_steps needs a graph from graph_upload");
  if (g->poisoned) return fail(CB_EPOISONED, "graph handle poisoned: %s", g->poison_msg);
  unprepare(g);
  hipLaunchKernelGGL(k_set_chain, dim3(1), dim3(64), 0, g->stream, g->ch_seed, g->ch_round, 0, seed, round);
  return enqueue_round(g, g->stream, last_step, false);
}

cb_status graph_sync(cb_graph* g) {
  if (!g) return fail(CB_EINVAL, "null graph");
  return sync_and_check(g);
}

cb_status graph_download(cb_graph* g, int64_t* row_ptr, int32_t* col) {
  if (!g) return fail(CB_EINVAL, "null graph");
  if (g->batch) return fail(CB_EINVAL, "graph_download needs a graph from graph_upload (use batch_download)");
  if (g->nnz > 0 && !col) return fail(CB_EINVAL, "col is NULL");
  cb_status s = sync_and_check(g);
  if (s != CB_OK) return s;
  char msg[256];
  if (row_ptr && !HIP_OK(hipMemcpy(row_ptr, g->rp, (size_t)(g->n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost), "download row_ptr"))
    return fail(CB_EDEVICE, "%s", msg);
  if (g->nnz > 0 && !HIP_OK(hipMemcpy(col, g->col, (size_t)g->nnz * sizeof(int32_t), hipMemcpyDeviceToHost), "download col"))
    return fail(CB_EDEVICE, "%s", msg);
  return CB_OK;
}

cb_status graph_download_state(cb_graph* g, int32_t which, void* host, int64_t count) {
  if (!g) return fail(CB_EINVAL, "null graph");
  if (count < 0 || (count > 0 && !host)) return fail(CB_EINVAL, "bad buffer");
  const void* src = nullptr;
  int64_t avail = 0;
  size_t elem = sizeof(int32_t);
  switch (which) {
    case CB_STATE_TRACE:
      if (!g->trace) return fail(CB_EINVAL, "tracing was never switched on");
      src = g->trace; avail = kTraceFields * (int64_t)g->L; elem = sizeof(int64_t);
      break;
    case CB_STATE_PERM: src = g->perm; avail = g->n; break;
    case CB_STATE_TRADE_OF: src = g->trade_of; avail = g->n; break;
    case CB_STATE_DEP: src = g->dep; avail = g->L; break;
    case CB_STATE_COL: src = g->col; avail = g->nnz; break;
    case CB_STATE_OUT_CUR: src = g->out_cur; avail = g->n; break;
    case CB_STATE_OWN_CUR: src = g->own_cur; avail = g->n; break;
    case CB_STATE_INBOX_CUR: src = g->inbox_cur; avail = g->n; break;
    default: return fail(CB_EINVAL, "unknown state id");
  }
  if (count > avail) return fail(CB_EINVAL, "count exceeds the state size");
  char msg[256];
  if (!HIP_OK(hipStreamSynchronize(g->stream), "hipStreamSynchronize")) return fail(CB_EDEVICE, "%s", msg);
  if (count > 0 && !HIP_OK(hipMemcpy(host, src, (size_t)count * elem, hipMemcpyDeviceToHost), "download state"))
    return fail(CB_EDEVICE, "%s", msg);
  return CB_OK;
}

cb_status graph_set_option(cb_graph* g, int32_t option, int64_t value) {
  if (!g) return fail(CB_EINVAL, "null graph");
  g->opt_version++;
  switch (option) {
    case CB_OPT_SMALL_MAX:
      if (value < 0 || value > kSmallCap) return fail(CB_EINVAL, "small_max must be in [0, 512]");
      g->small_max = (int32_t)value;
      return CB_OK;
    case CB_OPT_BIG_WORKERS:
      if (value < 1 || value > g->nbig_alloc) return fail(CB_EINVAL, "big workers out of range");
      g->nbig = (int32_t)value;
      return CB_OK;
    case CB_OPT_GRID_BLOCKS:
      if (value < 0 || value > (1 << 20)) return fail(CB_EINVAL, "grid blocks out of range");
      g->grid_blocks = (int32_t)value;
      return CB_OK;
    case CB_OPT_WATCHDOG_MS:
      if (value < 1 || value > 3600 * 1000) return fail(CB_EINVAL, "watchdog out of range");
      g->watchdog_ms = value;
      return CB_OK;
    case CB_OPT_TIMING:
      g->timing = value != 0;
      return CB_OK;
    case CB_OPT_DEBUG_CHECKS:
      g->debug_checks = value != 0;
      return CB_OK;
    case CB_OPT_TRACE:
      if (g->static_storage && value != 0) return fail(CB_EINVAL, "no tracing in static storage");
      if (value != 0 && !g->trace && !alloc_into(g, &g->trace, kTraceFields * (int64_t)g->L))
        return fail(CB_ENOMEM, "trace buffer allocation failed");
      g->tracing = value != 0;
      return CB_OK;
    case CB_OPT_BIG_LDS_MAX:
      if (value < 0 || value > kBigCap) return fail(CB_EINVAL, "big_lds_max must be in [0, 12288]");
      g->big_lds_max = (int32_t)value;
      return CB_OK;
    case CB_OPT_GIANT_DEG: {
      if (value < 0) return fail(CB_EINVAL, "giant degree must be >= 0");
      if (g->static_storage) return fail(CB_EINVAL, "no giant nodes in static storage");
      std::vector<int64_t> rp((size_t)g->n + 1);
      char msg[256];
      if (!HIP_OK(hipStreamSynchronize(g->stream), "sync") ||
          !HIP_OK(hipMemcpy(rp.data(), g->rp, rp.size() * sizeof(int64_t), hipMemcpyDeviceToHost), "read row_ptr"))
        return fail(CB_EDEVICE, "%s", msg);
      return setup_giants(g, value, rp.data());
    }
    case CB_OPT_HELP_MIN:
      if (value < 0 || value > INT32_MAX) return fail(CB_EINVAL, "help_min must be in [0, 2^31 - 1]");
      g->help_min = (int32_t)value;
      return CB_OK;
    case CB_OPT_HELP_GROUPS:
      if (value < 1 || value > kMaxJobs || kMaxJobs % value != 0)
        return fail(CB_EINVAL, "help groups must divide 64");
      g->help_groups = (int32_t)value;
      return CB_OK;
    case CB_OPT_HELP_CHUNK:
      if (value < 64 || value > 4096 || value % 64 != 0)
        return fail(CB_EINVAL, "help chunk must be a multiple of 64 in [64, 4096]");
      g->help_chunk = (int32_t)value;
      return CB_OK;
    case CB_OPT_CU_POOL:
      if (value != 0 && value != 1) return fail(CB_EINVAL, "pool must be 0 or 1");
      g->cu_pool = (int32_t)value;
      return CB_OK;
    case CB_OPT_IDLE_BACKOFF:
      if (value < 1 || value > 1024) return fail(CB_EINVAL, "idle back-off must be in [1, 1024]");
      g->idle_backoff = (int32_t)value;
      return CB_OK;
    case CB_OPT_FUSE_NEXT:
      if (value != 0 && value != 1) return fail(CB_EINVAL, "fuse must be 0 or 1");
      g->fuse_next = value != 0;
      return CB_OK;
    case CB_OPT_LOCAL_STACK:
      if (value < 0 || value > kStackCap) return fail(CB_EINVAL, "local stack must be in [0, 16]");
      g->stack_cap = (int32_t)value;
      return CB_OK;
    default:
      return fail(CB_EINVAL, "unknown option");
  }
}

cb_status graph_stats(cb_graph* g, cb_round_stats* out) {
  if (!g || !out) return fail(CB_EINVAL, "null argument");
  cb_status s = sync_and_check(g);
  if (s != CB_OK) return s;
  unsigned long long st[kStatCount] = {0};
  char msg[256];
  if (!HIP_OK(hipMemcpy(st, g->stats, sizeof(st), hipMemcpyDeviceToHost), "read stats"))
    return fail(CB_EDEVICE, "%s", msg);
  out->trades = g->L;
  out->small_trades = (int64_t)st[kStatSmall];
  out->big_trades = (int64_t)st[kStatBig];
  out->sources = (int64_t)st[kStatSources];
  out->queue_pushes = (int64_t)st[kStatPush];
  out->work = (int64_t)st[kStatWork];
  out->forwarded = (int64_t)st[kStatForward];
  out->emitted = (int64_t)st[kStatEmit];
  const double us = 1000.0 / (double)g->ticks_per_ms;
  out->small_busy_us = (double)st[kStatSmallTicks] * us;
  out->big_busy_us = (double)st[kStatBigTicks] * us;
  out->big_gather_us = (double)st[kStatBigGather] * us;
  out->big_split_us = (double)st[kStatBigSplit] * us;
  out->big_write_us = (double)st[kStatBigWrite] * us;
  out->big_release_us = (double)st[kStatBigRelease] * us;
  out->big_max_us = (double)st[kStatBigMaxTicks] * us;
  out->small_workers = (int64_t)(trade_grid(g) - effective_nbig(g)) * kWavesPerBlock;
  out->big_workers = effective_nbig(g);
  out->moved = (int64_t)st[kStatMoved];
  out->counted_trades = (int64_t)st[kStatCounted];
  return CB_OK;
}

cb_status graph_kernel_times(cb_graph* g, double* ms, int32_t count, int64_t* rounds) {
  if (!g) return fail(CB_EINVAL, "null graph");
  cb_status s = sync_and_check(g);
  if (s != CB_OK) return s;
  const int64_t r = g->rounds_timed;
  for (int i = 0; i < count && i < kTimedSteps; ++i) ms[i] = r ? g->ms_acc[i] / (double)r : 0.0;
  if (rounds) *rounds = r;
  for (double& a : g->ms_acc) a = 0.0;
  g->rounds_timed = 0;
  return CB_OK;
}

void graph_free(cb_graph* g) {
  if (!g) return;
  if (g->stream) (void)hipStreamSynchronize(g->stream);
  release_all(g);
  delete g;
}

// ---------------------------------------------------------------- batches

cb_status batch_upload(int32_t chains, const int64_t* n, const int64_t* const* row_ptr,
                       const int32_t* const* col, const uint64_t* seeds, const uint32_t* first_round,
                       void* stream, uint32_t flags, cb_graph** out) {
  if (!out) return fail(CB_EINVAL, "out is NULL");
  if (chains < 1 || !n || !row_ptr || !col || !seeds) return fail(CB_EINVAL, "null or empty chain arrays");
  std::vector<ChainSrc> src((size_t)chains);
  for (int32_t c = 0; c < chains; ++c)
    src[c] = ChainSrc{n[c], row_ptr[c], col[c], false, 0, seeds[c], first_round ? first_round[c] : 0u};
  return create_graph(src.data(), chains, stream, flags, true, out);
}

cb_status batch_info(const cb_graph* g, int32_t chain, int64_t* n, int64_t* nnz, uint32_t* next_round) {
  if (!g) return fail(CB_EINVAL, "null graph");
  if (chain < 0 || chain >= g->chains) return fail(CB_EINVAL, "chain out of range");
  if (!g->batch) {
    if (n) *n = g->n;
    if (nnz) *nnz = g->nnz;
    if (next_round) *next_round = 0;
    return CB_OK;
  }
  const int32_t i = g->h_pos[chain];
  if (n) *n = g->h_node_base[i + 1] - g->h_node_base[i];
  if (nnz) *nnz = g->h_nnz_base[i + 1] - g->h_nnz_base[i];
  if (next_round) *next_round = g->h_round[i];
  return CB_OK;
}

cb_status batch_run(cb_graph* g, uint32_t rounds) {
  if (!g) return fail(CB_EINVAL, "null graph");
  if (g->poisoned) return fail(CB_EPOISONED, "graph handle poisoned: %s", g->poison_msg);
  if (rounds == 0) return CB_OK;
  if (!g->batch) return fail(CB_EINVAL, "batch_run needs a graph from batch_upload (use global_trade)");
  char msg[256];
  const bool eager = g->timing || g->tracing || g->giant_dirty;
  if (eager) {
    for (uint32_t r = 0; r < rounds; ++r) {
      cb_status s = enqueue_round(g, g->stream, CB_STEP_REBUILD, true);
      if (s != CB_OK) return s;
    }
  } else {
    if (!g->exec || g->exec_rounds != rounds || g->exec_version != g->opt_version ||
        g->exec_prepared != g->prepared) {
      const bool start_prepared = g->prepared;
      drop_exec(g);
      if (!g->cap_stream && !HIP_OK(hipStreamCreateWithFlags(&g->cap_stream, hipStreamNonBlocking), "capture stream"))
        return fail(CB_EDEVICE, "%s", msg);
      if (!HIP_OK(hipStreamBeginCapture(g->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture"))
        return fail(CB_EDEVICE, "%s", msg);
      cb_status s = CB_OK;
      for (uint32_t r = 0; r < rounds && s == CB_OK; ++r) s = enqueue_round(g, g->cap_stream, CB_STEP_REBUILD, true);
      hipGraph_t graph = nullptr;
      const hipError_t e = hipStreamEndCapture(g->cap_stream, &graph);
      if (s != CB_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return s;
      }
      if (!HIP_OK(e, "end capture")) return fail(CB_EDEVICE, "%s", msg);
      g->graph = graph;
      if (!HIP_OK(hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0), "instantiate")) {
        drop_exec(g);
        return fail(CB_EDEVICE, "%s", msg);
      }
      g->exec_rounds = rounds;
      g->exec_version = g->opt_version;
      g->exec_prepared = start_prepared;
    } else {
      // replaying: the state moves through the same rounds as when captured
      g->prepared = g->fuse_next;
    }
    if (!HIP_OK(hipGraphLaunch(g->exec, g->stream), "graph launch")) return poison(g, CB_EDEVICE, msg);
  }
  for (auto& r : g->h_round) r += rounds;
  return CB_OK;
}

cb_status batch_download(cb_graph* g, int32_t chain, int32_t* col) {
  if (!g) return fail(CB_EINVAL, "null graph");
  if (chain < 0 || chain >= g->chains) return fail(CB_EINVAL, "chain out of range");
  if (!g->batch) return graph_download(g, nullptr, col);
  const int32_t ci = g->h_pos[chain];
  const int64_t e0 = g->h_nnz_base[ci], e = g->h_nnz_base[ci + 1] - e0;
  if (e > 0 && !col) return fail(CB_EINVAL, "col is NULL");
  cb_status s = sync_and_check(g);
  if (s != CB_OK) return s;
  char msg[256];
  if (e > 0 && !HIP_OK(hipMemcpy(col, g->col + e0, (size_t)e * sizeof(int32_t), hipMemcpyDeviceToHost), "download col"))
    return fail(CB_EDEVICE, "%s", msg);
  const int32_t shift = (int32_t)g->h_node_base[ci];
  if (shift)
    for (int64_t i = 0; i < e; ++i) col[i] -= shift;
  return CB_OK;
}

// ---------------------------------------------------------------- autotuner

cb_status graph_autotune(cb_graph* g, uint32_t trial_rounds, int32_t use_cache, cb_tune_result* out) {
  if (!g || !out) return fail(CB_EINVAL, "null argument");
  if (trial_rounds < 1 || trial_rounds > 64) return fail(CB_EINVAL, "trial rounds must be in [1, 64]");
  if (g->static_storage) return fail(CB_EINVAL, "no autotuning in static storage");
  cb_status s = sync_and_check(g);
  if (s != CB_OK) return s;
  const TuneKey key = tune_key(g);
  if (use_cache) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      *out = it->second;
      out->cached = 1;
      apply_tuned(g, *out);
      return CB_OK;
    }
  }
  if (g->L == 0 || g->nnz == 0) {
    *out = current_options(g);
    return CB_OK;
  }
  char msg[256];
  int32_t* saved = nullptr;
  if (!alloc_into(g, &saved, g->nnz)) return fail(CB_ENOMEM, "no device memory for the tuner's copy");
  hipStream_t st = g->stream;
  const bool timing = g->timing, tracing = g->tracing;
  g->timing = false;
  g->tracing = false;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  bool ok = HIP_OK(hipEventCreate(&e0), "event") && HIP_OK(hipEventCreate(&e1), "event") &&
            HIP_OK(hipMemcpyAsync(saved, g->col, (size_t)g->nnz * 4, hipMemcpyDeviceToDevice, st), "save col") &&
            HIP_OK(hipMemcpyAsync(g->ch_round_saved, g->ch_round, (size_t)g->chains * 4, hipMemcpyDeviceToDevice, st), "save rounds");
  // time trial_rounds rounds from the saved state under the current options
  auto trial = [&](double* ms_out) -> cb_status {
    unprepare(g);
    if (!HIP_OK(hipMemcpyAsync(g->col, saved, (size_t)g->nnz * 4, hipMemcpyDeviceToDevice, st), "restore col") ||
        !HIP_OK(hipMemcpyAsync(g->ch_round, g->ch_round_saved, (size_t)g->chains * 4, hipMemcpyDeviceToDevice, st), "restore rounds") ||
        !HIP_OK(hipEventRecord(e0, st), "event"))
      return fail(CB_EDEVICE, "%s", msg);
    for (uint32_t r = 0; r < trial_rounds; ++r) {
      cb_status t = enqueue_round(g, st, CB_STEP_REBUILD, true);
      if (t != CB_OK) return t;
    }
    if (!HIP_OK(hipEventRecord(e1, st), "event")) return fail(CB_EDEVICE, "%s", msg);
    cb_status t = sync_and_check(g);
    if (t != CB_OK) return t;
    float ms = 0.f;
    if (!HIP_OK(hipEventElapsedTime(&ms, e0, e1), "elapsed")) return fail(CB_EDEVICE, "%s", msg);
    *ms_out = (double)ms / trial_rounds;
    return CB_OK;
  };
  cb_tune_result best = current_options(g);
  if (!ok) s = fail(CB_EDEVICE, "%s", msg);
  if (s == CB_OK) {
    apply_tuned(g, best);
    double ms = 0;
    s = trial(&ms);   // warm-up (first use of every buffer)
    if (s == CB_OK) s = trial(&ms);
    best.ms_per_round = best.default_ms_per_round = ms;
    best.evaluated = 2;
  }
  // coordinate descent over the kernel's workgroups (a grid below the
  // workgroup workers plus one is raised to that), the workgroup pool, the
  // idle wavefronts' back-off, their local stack of ready trades, the
  // wavefront/workgroup threshold, the size from which write phases are
  // shared, their chunk size and the workgroup workers
  struct Param {
    int32_t cb_tune_result::*field;
    int32_t values[6];
    int count;
  };
  const int32_t cu = g->cu_count;
  const Param params[] = {
      {&cb_tune_result::grid_blocks, {0, cu, cu * 3 / 4, cu * 5 / 8, cu / 2}, 5},
      {&cb_tune_result::cu_pool, {0, 1}, 2},
      {&cb_tune_result::idle_backoff, {2, 8, 32, 128}, 4},
      {&cb_tune_result::local_stack, {0, 1, 2, 4, 8, 16}, 6},
      {&cb_tune_result::small_max, {128, 256, 384, 512}, 4},
      {&cb_tune_result::help_min, {1024, 2048, 4096, 8192, 0}, 5},
      {&cb_tune_result::help_chunk, {64, 128, 256, 512}, 4},
      {&cb_tune_result::big_workers, {16, 32, 48, 64}, 4},
  };
  for (const Param& P : params) {
    if (s != CB_OK) break;
    for (int i = 0; i < P.count && s == CB_OK; ++i) {
      cb_tune_result cand = best;
      int32_t* field = &(cand.*P.field);
      if (*field == P.values[i]) continue;
      if (P.field == &cb_tune_result::big_workers && P.values[i] > g->nbig_alloc) continue;
      const int32_t* set = P.values;
      *field = set[i];
      apply_tuned(g, cand);
      double ms = 0;
      s = trial(&ms);
      best.evaluated++;
      // a candidate must beat the best by more than round-to-round noise
      if (s == CB_OK && ms < 0.99 * best.ms_per_round) {
        const int ev = best.evaluated;
        best = cand;
        best.ms_per_round = ms;
        best.evaluated = ev;
      }
    }
  }
  // back to the state before tuning, with the best options
  unprepare(g);
  (void)hipMemcpyAsync(g->col, saved, (size_t)g->nnz * 4, hipMemcpyDeviceToDevice, st);
  (void)hipMemcpyAsync(g->ch_round, g->ch_round_saved, (size_t)g->chains * 4, hipMemcpyDeviceToDevice, st);
  (void)hipStreamSynchronize(st);
  dev_free_one(g, saved);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  g->timing = timing;
  g->tracing = tracing;
  if (s != CB_OK) return s;
  apply_tuned(g, best);
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune_cache[key] = best;
  }
  *out = best;
  return CB_OK;
}

}  // extern "C"


// ---------------------------------------------------------------- static scratch
// One global trade of a caller-held graph with every buffer in this array
// (for callers that cannot allocate device memory). Each GPU holds its own
// copy of the array, at its own address, from library load to process end.
namespace {
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
struct StaticDevice {
  std::mutex mu;           // calls on one device run one after the other
  bool ready = false;
  char* ptr = nullptr;     // device address of this device's `scratch`
  cb_graph g;              // host-side state of the last call
};
StaticDevice g_static[kMaxDevices];
}  // namespace

extern "C" cb_status global_trade_static(int64_t n, const int64_t* row_ptr, int32_t* col, uint64_t seed,
                                         uint32_t round, void* stream) {
  if (n < 0 || n > INT32_MAX) return fail(CB_EINVAL, "n must be in [0, 2^31 - 1]");
  int dev = 0;
  char msg[256];
  if (!HIP_OK(hipGetDevice(&dev), "hipGetDevice")) return fail(CB_EDEVICE, "%s", msg);
  if (dev < 0 || dev >= kMaxDevices) return fail(CB_EINVAL, "device index beyond %d", kMaxDevices);
  StaticDevice& S = g_static[dev];
  std::lock_guard<std::mutex> lock(S.mu);
  if (!S.ready) {
    // the array's name is a host-side stand-in: its device address comes from
    // the runtime, once per device, with that device current
    void* p = nullptr;
    if (!HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)"))
      return fail(CB_EDEVICE, "%s", msg);
    S.ptr = static_cast<char*>(p);
    S.ready = true;
  }
  ChainSrc c{n, row_ptr, col, true, 0, seed, round};
  int64_t d1 = 0, d2 = 0;
  cb_status s = check_chain_host(c, &d1, &d2);
  if (s != CB_OK) return s;
  cb_graph* g = &S.g;
  *g = cb_graph();
  g->static_storage = true;
  g->device = dev;
  g->stream = (hipStream_t)stream;
  const DeviceInfo di = device_info(dev);
  g->cu_count = di.cu_count;
  g->occupancy_blocks = di.occupancy;
  g->ticks_per_ms = di.ticks_per_ms;
  g->nbig_alloc = std::max(1, std::min(16, g->cu_count / 2));
  size_graph(g, &c, 1, d1, d2);
  count_classes(g, &c, 1);
  BufPlan P;
  plan_buffers(g, P, false);
  const size_t need = plan_bytes(P);
  if (need > kStaticScratchBytes)
    return fail(CB_EINVAL, "graph needs %zu bytes of scratch; the static array holds %zu", need, kStaticScratchBytes);
  carve_plan(P, S.ptr);
  g->col = col;
  hipStream_t st = g->stream;
  if (!HIP_OK(hipMemcpyAsync(g->rp, row_ptr, (size_t)(n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st), "copy row_ptr"))
    return fail(CB_EDEVICE, "%s", msg);
  hipLaunchKernelGGL(k_single_chain, dim3(1), dim3(64), 0, st, g->ch_node_base, g->ch_trade_base, g->ch_bucket_base,
                     g->ch_left_base, g->ch_seed, g->ch_round, g->ch_draw_base, n, g->nb, seed, round);
  if (!init_device_state(g, false, msg, sizeof(msg))) return fail(CB_EDEVICE, "%s", msg);
  g->gwords = ((n + 4095) / 4096) * 64;
  s = enqueue_round(g, st, CB_STEP_REBUILD, false);
  if (s != CB_OK) return s;
  return sync_and_check(g);
}

// ---------------------------------------------------------------- single trades
// Steps step0 .. step0 + steps - 1 of the uniform single-trade chain. Step s
// trades the pair u = bounded(philox64(seed; s_lo, s_hi, 0, TAG_U), n),
// v = bounded(philox64(seed; s_lo, s_hi, 1, TAG_U), n - 1) (+1 if >= u), its
// split drawn from philox64(seed; s, 0xFFFFFFFF, j, TAG_F). Consecutive steps
// whose pairs share no node form a phase, applied in step order as one
// partial global trade (the dependency counts order them exactly as the
// sequential chain does); a step that meets a node of the current phase
// starts the next phase.
extern "C" cb_status cbu_trades(cb_graph* g, uint64_t seed, uint64_t step0, uint64_t steps) {
  if (!g) return fail(CB_EINVAL, "null graph");
  if (g->batch) return fail(CB_EINVAL, "single trades need a graph from graph_upload");
  if (g->poisoned) return fail(CB_EPOISONED, "graph handle poisoned: %s", g->poison_msg);
  if (step0 + steps > ((uint64_t)1 << 32) || step0 + steps < step0)
    return fail(CB_EINVAL, "single-trade steps must stay below 2^32");
  if (g->ngiant > 0) return fail(CB_EINVAL, "single trades need giant nodes off (CB_OPT_GIANT_DEG 0)");
  if (g->n < 2 || steps == 0) return CB_OK;
  const int64_t n = g->n;
  char msg[256];
  // every step's pair, and where each phase starts
  std::vector<int32_t> pairs((size_t)(2 * steps));
  std::vector<uint64_t> phase_start;
  std::vector<uint32_t> stamp((size_t)n, 0);
  uint32_t phase = 0;
  for (uint64_t t = 0; t < steps; ++t) {
    const uint64_t s = step0 + t;
    const int64_t u = (int64_t)host_bounded(host_philox64(seed, (uint32_t)s, (uint32_t)(s >> 32), 0u, kTagPair), (uint64_t)n);
    int64_t v = (int64_t)host_bounded(host_philox64(seed, (uint32_t)s, (uint32_t)(s >> 32), 1u, kTagPair), (uint64_t)(n - 1));
    if (v >= u) ++v;
    if (phase == 0 || stamp[(size_t)u] == phase || stamp[(size_t)v] == phase) {
      ++phase;
      phase_start.push_back(t);
    }
    stamp[(size_t)u] = stamp[(size_t)v] = phase;
    pairs[(size_t)(2 * t)] = (int32_t)u;
    pairs[(size_t)(2 * t + 1)] = (int32_t)v;
  }
  phase_start.push_back(steps);
  int32_t* dpairs = nullptr;
  if (!alloc_into(g, &dpairs, (int64_t)pairs.size())) return fail(CB_ENOMEM, "no device memory for the pairs");
  hipStream_t st = g->stream;
  unprepare(g);
  bool ok = HIP_OK(hipMemcpyAsync(dpairs, pairs.data(), pairs.size() * sizeof(int32_t), hipMemcpyHostToDevice, st),
                   "copy pairs");
  const Chains ch = chains_of(g);
  (void)ch;
  for (size_t p = 0; ok && p + 1 < phase_start.size(); ++p) {
    const uint64_t t0 = phase_start[p];
    const int32_t P = (int32_t)(phase_start[p + 1] - t0);
    hipLaunchKernelGGL(k_round_reset, dim3(grid_for(std::max<int64_t>({n, (int64_t)g->nb, (int64_t)kCwCount}), 256, 8192)),
                       dim3(256), 0, st, n, g->nb, g->inbox_cur, g->out_cur, g->own_cur, g->bcount, g->bcur, g->ctrl,
                       g->stats, p == 0 ? 1 : 0);
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, 256, 8192)), dim3(256), 0, st, g->trade_of, n, kUnmatched);
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, 256, 8192)), dim3(256), 0, st, g->tinfo, n, kUnmatched);
    hipLaunchKernelGGL(k_phase_pairs, dim3(grid_for(P, 256, 1024)), dim3(256), 0, st, dpairs + 2 * t0, P, g->perm,
                       g->trade_of, g->tinfo, g->dep);
    hipLaunchKernelGGL(k_set_draws, dim3(1), dim3(64), 0, st, g->ch_seed, g->ch_round, g->ch_draw_base, seed,
                       kSingleRound, (uint32_t)(step0 + t0));
    if (g->nnz > 0) {
      hipLaunchKernelGGL(k_depscan, dim3((unsigned)((g->nnz + kScanChunk - 1) / kScanChunk)), dim3(256), 0, st, n,
                         g->nnz, g->rp, g->col, g->trade_of, g->tinfo, g->col_t, g->dep, giant_sets(g), g->ctrl);
      hipLaunchKernelGGL(k_copy_idle_edges, dim3(grid_for(n, 256, 8192)), dim3(256), 0, st, n, g->rp, g->col,
                         g->trade_of, g->col_out, g->out_cur, g->ctrl);
    }
    for (int pass = 0; pass < 2; ++pass) {
      hipLaunchKernelGGL(k_sources, dim3(grid_for(P, 256, 8192)), dim3(256), 0, st, P, g->dep, g->perm, g->rp,
                         effective_small_max(g), g->tsz, g->src_list, g->qb, g->ctrl, g->stats, chains_of(g),
                         g->src_b, pass);
      if (pass == 0)
        hipLaunchKernelGGL(k_sources_scan, dim3(1), dim3(kSrcBuckets), 0, st, g->src_b, g->ctrl);
    }
    hipLaunchKernelGGL(k_node_info, dim3(grid_for(n, 256, 8192)), dim3(256), 0, st, n, g->rp, g->tinfo, g->ninfo);
    const TradeArgs A = trade_args(g, P);
    hipLaunchKernelGGL(k_trade, dim3(trade_grid(g)), dim3(kTradeBlock), 0, st, A);
    hipLaunchKernelGGL(k_check_rows, dim3(grid_for(n, 256, 8192)), dim3(256), 0, st, n, g->rp, g->out_cur,
                       g->own_cur, g->ctrl);
    if (g->nnz > 0) {
      const NextScan none{};
      if (g->n_small)
        hipLaunchKernelGGL(k_segsort_small, dim3(grid_for(g->n_small, 4, 65536)), dim3(256), 0, st, g->rows,
                           g->n_small, g->rp, g->col_out, g->col, none, g->ctrl);
      if (g->n_mid)
        hipLaunchKernelGGL(k_segsort_mid, dim3(grid_for(g->n_mid, 1, 65536)), dim3(256), 0, st,
                           g->rows + g->n_small, g->n_mid, g->rp, g->col_out, g->col, g->keybits_node, none, g->ctrl);
      if (g->n_big) {
        hipLaunchKernelGGL(k_segsort_wide, dim3(grid_for(g->n_big, 1, 4096)), dim3(kSegWideThreads), 0, st,
                           g->rows + g->n_small + g->n_mid, g->n_big, g->rp, g->col_out, g->col, g->keybits_node,
                           g->ctrl);
        hipLaunchKernelGGL(k_segsort_huge, dim3(grid_for(g->n_big, 1, 4096)), dim3(kSegWideThreads), 0, st,
                           g->rows + g->n_small + g->n_mid, g->n_big, g->rp, g->col_out, g->col, g->keybits_node,
                           g->ctrl);
      }
    }
    ok = HIP_OK(hipGetLastError(), "kernel launch");
  }
  // the draw offset goes back to the global-trade convention
  hipLaunchKernelGGL(k_set_draws, dim3(1), dim3(64), 0, st, g->ch_seed, g->ch_round, g->ch_draw_base, seed, 0u, 0u);
  const hipError_t se = hipStreamSynchronize(st);
  dev_free_one(g, dpairs);
  if (!ok) return poison(g, CB_EDEVICE, msg);
  if (se != hipSuccess) return poison(g, CB_EDEVICE, hipGetErrorString(se));
  return sync_and_check(g);
}
