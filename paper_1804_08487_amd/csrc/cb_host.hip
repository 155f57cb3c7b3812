// Host side of the C ABI declared in include/curveball.h: device buffers of
// one chain, the launch sequence of a global trade, error reporting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "curveball.h"
#include "cb_kernels.hpp"

using namespace cbx;

namespace {

thread_local std::string g_last_error;
cb_allocator g_allocator = {nullptr, nullptr, nullptr};

cb_status fail(cb_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

bool hip_ok(hipError_t e, std::string* msg, const char* what) {
  if (e == hipSuccess) return true;
  *msg = std::string(what) + ": " + hipGetErrorString(e);
  return false;
}

int bitlen(uint64_t x) { return x ? 64 - __builtin_clzll(x) : 0; }

constexpr int kTimedSteps = 4;

struct EventSet {
  hipEvent_t ev[kTimedSteps + 1];
};

}  // namespace

struct cb_graph {
  int64_t n = 0, nnz = 0;
  int32_t L = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  cb_allocator alloc{};
  std::vector<void*> owned;

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
  int32_t* tsz = nullptr;
  HelpJob* jobs = nullptr;
  int64_t* trace = nullptr;     // allocated when tracing is first switched on
  int32_t* qs = nullptr;
  int32_t* qb = nullptr;
  int32_t* bcount = nullptr;
  int32_t* bstart = nullptr;
  int32_t* bcur = nullptr;
  int32_t* ctrl = nullptr;
  unsigned long long* stats = nullptr;
  uint64_t* slots = nullptr;
  int32_t* sbpre = nullptr;
  int64_t sbpre_stride = 1;
  int32_t* rows_small = nullptr;
  int32_t* rows_mid = nullptr;
  int32_t* rows_big = nullptr;
  int64_t n_small = 0, n_mid = 0, n_big = 0;

  int nb_log2 = 0;
  int32_t nb = 1;
  int keybits_node = 1, keybits_entry = 1;
  int64_t smax = 1;
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
  int64_t watchdog_ms = 20000;
  bool timing = false;
  bool debug_checks = false;
  bool tracing = false;

  bool poisoned = false;
  std::string poison_msg;

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

void release_all(cb_graph* g) {
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

std::string error_bits_text(int32_t bits) {
  std::string s;
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
    if (bits & nm.bit) { if (!s.empty()) s += "; "; s += nm.name; }
  return s;
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

cb_status sync_and_check(cb_graph* g) {
  if (g->poisoned) return fail(CB_EPOISONED, "graph handle poisoned: " + g->poison_msg);
  std::string msg;
  if (!hip_ok(hipStreamSynchronize(g->stream), &msg, "hipStreamSynchronize")) {
    g->poisoned = true;
    g->poison_msg = msg;
    return fail(CB_EDEVICE, msg);
  }
  int32_t err = 0;
  if (!hip_ok(hipMemcpy(&err, g->ctrl + cw(kCwErr), sizeof(int32_t), hipMemcpyDeviceToHost), &msg,
              "hipMemcpy(error word)")) {
    g->poisoned = true;
    g->poison_msg = msg;
    return fail(CB_EDEVICE, msg);
  }
  if (g->timing) collect_timing(g);
  if (err) {
    int32_t dbg[3] = {0, 0, 0};
    for (int i = 0; i < 3; ++i)
      (void)hipMemcpy(&dbg[i], g->ctrl + cw(kCwDbgBits + i), sizeof(int32_t), hipMemcpyDeviceToHost);
    g->poisoned = true;
    g->poison_msg = error_bits_text(err) + " (first: bits " + std::to_string(dbg[0]) + ", trade " +
                    std::to_string(dbg[1] - 1) + ", detail " + std::to_string(dbg[2]) + ")";
    return fail((err & kErrWatchdog) ? CB_EWATCHDOG : CB_EDEVICE,
                "device reported: " + g->poison_msg);
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
  std::string msg;
  if (!hip_ok(hipStreamSynchronize(g->stream), &msg, "sync")) return fail(CB_EDEVICE, msg);
  auto drop = [&](void* p) {
    if (!p) return;
    for (auto it = g->owned.begin(); it != g->owned.end(); ++it)
      if (*it == p) { g->owned.erase(it); break; }
    if (g->alloc.free) g->alloc.free(p, g->alloc.user); else (void)hipFree(p);
  };
  drop(g->gbm);
  drop(g->gsc);
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
  if (!hip_ok(hipMemcpyAsync(g->giant_id, gid.data(), gid.size() * sizeof(int32_t), hipMemcpyHostToDevice, g->stream), &msg, "copy giant ids") ||
      !hip_ok(hipStreamSynchronize(g->stream), &msg, "sync"))
    return fail(CB_EDEVICE, msg);
  if (ng == 0) return CB_OK;
  if (!alloc_into(g, &g->gbm, (int64_t)ng * g->gwords) || !alloc_into(g, &g->gsc, (int64_t)ng * (g->gwords >> 6))) {
    drop(g->gbm);
    g->gbm = nullptr;
    g->ngiant = 0;
    g->giant_deg = 0;
    std::vector<int32_t> none(gid.size(), -1);
    (void)hipMemcpyAsync(g->giant_id, none.data(), none.size() * sizeof(int32_t), hipMemcpyHostToDevice, g->stream);
    (void)hipStreamSynchronize(g->stream);
    return fail(CB_ENOMEM, "no device memory for giant bitmaps");
  }
  // cleared on the graph's own stream (a non-blocking stream is not ordered
  // after work on the null stream)
  if (!hip_ok(hipMemsetAsync(g->gbm, 0, (size_t)ng * g->gwords * 8, g->stream), &msg, "clear bitmaps") ||
      !hip_ok(hipMemsetAsync(g->gsc, 0, (size_t)ng * (g->gwords >> 6) * 4, g->stream), &msg, "clear counts") ||
      !hip_ok(hipStreamSynchronize(g->stream), &msg, "sync"))
    return fail(CB_EDEVICE, msg);
  return CB_OK;
}

int32_t effective_nbig(const cb_graph* g) {
  int32_t v = g->nbig > 0 ? g->nbig : std::max(1, g->cu_count / 4);
  return std::min(v, g->nbig_alloc);
}

int32_t trade_grid(const cb_graph* g) {
  int32_t blocks = g->grid_blocks > 0 ? g->grid_blocks : g->cu_count * g->occupancy_blocks;
  return std::max(blocks, effective_nbig(g) + 1);
}

// Trades above this size run on a workgroup (a giant node never runs on a
// wavefront).
int32_t effective_small_max(const cb_graph* g) {
  return g->giant_deg > 0 ? (int32_t)std::min<int64_t>(g->small_max, g->giant_deg - 1) : g->small_max;
}

cb_status enqueue_round(cb_graph* g, uint64_t seed, uint32_t round, int last_step) {
  if (!g) return fail(CB_EINVAL, "null graph");
  if (g->poisoned) return fail(CB_EPOISONED, "graph handle poisoned: " + g->poison_msg);
  if (last_step < CB_STEP_MATCHING || last_step > CB_STEP_REBUILD)
    return fail(CB_EINVAL, "last_step out of range");
  if (g->n == 0) return CB_OK;
  hipStream_t st = g->stream;
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
  if (g->giant_dirty) {
    std::string msg;
    if (!hip_ok(hipMemsetAsync(g->gbm, 0, (size_t)g->ngiant * g->gwords * 8, st), &msg, "clear bitmaps") ||
        !hip_ok(hipMemsetAsync(g->gsc, 0, (size_t)g->ngiant * (g->gwords >> 6) * 4, st), &msg, "clear counts"))
      return fail(CB_EDEVICE, msg);
    g->giant_dirty = false;
  }
  if (last_step < CB_STEP_TRADE && g->ngiant > 0) g->giant_dirty = true;

  hipLaunchKernelGGL(k_round_reset, dim3(grid_for(std::max<int64_t>({n, (int64_t)g->nb, (int64_t)kCwCount}), 256, 8192)),
                     dim3(256), 0, st, n, g->nb, g->inbox_cur, g->out_cur, g->own_cur, g->bcount,
                     g->bcur, g->ctrl, g->stats);
  // 1. matching
  hipLaunchKernelGGL(k_match_count, dim3(grid_for(n, 256, 16384)), dim3(256), 0, st, n, seed, round,
                     g->nb_log2, g->bcount, g->ctrl);
  hipLaunchKernelGGL(k_match_scan, dim3(1), dim3(1024), 0, st, g->nb, g->bcount, g->bstart, g->ctrl);
  hipLaunchKernelGGL(k_match_scatter, dim3(grid_for(n, 256, 16384)), dim3(256), 0, st, n, seed,
                     round, g->nb_log2, g->bstart, g->bcur, g->mtmp, g->ctrl);
  hipLaunchKernelGGL(k_match_sort, dim3(std::min<int32_t>(g->nb, 1 << 20)), dim3(kMatchBlock), 0, st,
                     n, seed, round, g->nb, g->bstart, g->mtmp, g->mkey, g->perm, g->trade_of,
                     g->tinfo, g->giant_id, g->dep, g->ctrl);
  if (timed) (void)hipEventRecord(evs.ev[1], st);
  if (g->debug_checks && g->ngiant > 0)
    hipLaunchKernelGGL(k_check_giants_empty, dim3(1024), dim3(256), 0, st,
                       (int64_t)g->ngiant * (g->gwords >> 6), g->gsc, g->ctrl);
  if (last_step >= CB_STEP_DEPSCAN) {
    // 2. dependency scan + sources
    if (g->nnz > 0)
      hipLaunchKernelGGL(k_depscan, dim3((unsigned)((g->nnz + kScanChunk - 1) / kScanChunk)), dim3(256),
                         0, st, n, g->nnz, g->rp, g->col, g->trade_of, g->tinfo, g->col_t, g->dep,
                         giant_sets(g), g->ctrl);
    if (L > 0)
      hipLaunchKernelGGL(k_sources, dim3(grid_for(L, 256, 8192)), dim3(256), 0, st, L, g->dep,
                         g->perm, g->rp, effective_small_max(g), g->tsz, g->src_list, g->qb,
                         g->ctrl, g->stats);
  }
  if (timed) (void)hipEventRecord(evs.ev[2], st);
  if (last_step >= CB_STEP_TRADE && L > 0) {
    // 3. trades
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
    A.jobs = g->jobs;
    A.trace = g->tracing ? g->trace : nullptr;
    if (g->tracing) {
      std::string msg;
      if (!hip_ok(hipMemsetAsync(g->trace, 0xFF, (size_t)L * kTraceFields * sizeof(int64_t), st), &msg, "clear trace"))
        return fail(CB_EDEVICE, msg);
    }
    A.qs = g->qs;
    A.qb = g->qb;
    A.ctrl = g->ctrl;
    A.stats = g->stats;
    A.slots = g->slots;
    A.slot_elems = g->slot_elems;
    A.sbpre = g->sbpre;
    A.sbpre_stride = g->sbpre_stride;
    A.smax = g->smax;
    A.n = n;
    A.L = L;
    A.small_max = effective_small_max(g);
    A.help_min = g->help_min;
    A.help_groups = g->help_groups;
    A.big_lds_max = g->big_lds_max;
    A.nbig = effective_nbig(g);
    A.stack_cap = g->stack_cap;
    A.keybits = g->keybits_entry;
    A.round = round;
    A.seed = seed;
    A.watchdog_ticks = (uint64_t)g->watchdog_ms * g->ticks_per_ms;
    hipLaunchKernelGGL(k_trade, dim3(trade_grid(g)), dim3(kTradeBlock), 0, st, A);
  }
  if (timed) (void)hipEventRecord(evs.ev[3], st);
  if (last_step >= CB_STEP_TRADE && L > 0)
    hipLaunchKernelGGL(k_check_rows, dim3(grid_for(n, 256, 8192)), dim3(256), 0, st, n, g->rp,
                       g->out_cur, g->own_cur, g->ctrl);
  if (last_step >= CB_STEP_REBUILD && g->nnz > 0) {
    // 4. rebuild: per-row ascending sort of col_out into col
    if (g->n_small)
      hipLaunchKernelGGL(k_segsort_small, dim3(grid_for(g->n_small, 4, 65536)), dim3(256), 0, st,
                         g->rows_small, g->n_small, g->rp, g->col_out, g->col, g->ctrl);
    if (g->n_mid)
      hipLaunchKernelGGL(k_segsort_mid, dim3(grid_for(g->n_mid, 1, 65536)), dim3(256), 0, st,
                         g->rows_mid, g->n_mid, g->rp, g->col_out, g->col, g->keybits_node, g->ctrl);
    if (g->n_big)
      hipLaunchKernelGGL(k_segsort_big, dim3(grid_for(g->n_big, 1, 8192)), dim3(256), 0, st,
                         g->rows_big, g->n_big, g->rp, g->col_out, g->col, g->keybits_node, g->ctrl);
  }
  if (timed) {
    (void)hipEventRecord(evs.ev[4], st);
    g->pending.push_back(evs);
  }
  std::string msg;
  if (!hip_ok(hipGetLastError(), &msg, "kernel launch")) {
    g->poisoned = true;
    g->poison_msg = msg;
    return fail(CB_EDEVICE, msg);
  }
  return CB_OK;
}

}  // namespace

extern "C" {

cb_status cb_set_allocator(const cb_allocator* a) {
  if (a && (!a->alloc || !a->free)) return fail(CB_EINVAL, "allocator needs alloc and free");
  g_allocator = a ? *a : cb_allocator{nullptr, nullptr, nullptr};
  return CB_OK;
}

const char* cb_last_error(void) { return g_last_error.c_str(); }

cb_status graph_upload(int64_t n, const int64_t* row_ptr, const int32_t* col, void* stream,
                       uint32_t flags, cb_graph** out) {
  if (!out) return fail(CB_EINVAL, "out is NULL");
  *out = nullptr;
  if (n < 0 || n > INT32_MAX) return fail(CB_EINVAL, "n must be in [0, 2^31 - 1]");
  if (!row_ptr) return fail(CB_EINVAL, "row_ptr is NULL");
  if (row_ptr[0] != 0) return fail(CB_EINVAL, "row_ptr[0] must be 0");
  int64_t d1 = 0, d2 = 0;
  for (int64_t x = 0; x < n; ++x) {
    const int64_t d = row_ptr[x + 1] - row_ptr[x];
    if (d < 0) return fail(CB_EINVAL, "row_ptr is not monotone");
    if (d >= n && d > 0) return fail(CB_ENOTSIMPLE, "a row has more entries than other nodes");
    if (d > d1) { d2 = d1; d1 = d; } else if (d > d2) { d2 = d; }
  }
  const int64_t nnz = row_ptr[n];
  if (nnz % 2) return fail(CB_ENOTSIMPLE, "odd number of entries cannot be symmetric");
  if (nnz >= INT32_MAX) return fail(CB_EINVAL, "2m must be below 2^31");
  if (nnz > 0 && !col) return fail(CB_EINVAL, "col is NULL");

  cb_graph* g = new cb_graph();
  g->alloc = g_allocator;
  g->n = n;
  g->nnz = nnz;
  g->L = (int32_t)(n / 2);
  std::string msg;
  if (!hip_ok(hipGetDevice(&g->device), &msg, "hipGetDevice")) { delete g; return fail(CB_EDEVICE, msg); }
  if (stream) {
    g->stream = (hipStream_t)stream;
  } else {
    if (!hip_ok(hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking), &msg, "hipStreamCreate")) {
      delete g;
      return fail(CB_EDEVICE, msg);
    }
    g->own_stream = true;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, g->device) == hipSuccess) g->cu_count = prop.multiProcessorCount;
  int rate_khz = 0;
  if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, g->device) == hipSuccess &&
      rate_khz > 0)
    g->ticks_per_ms = (uint64_t)rate_khz;
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void*>(k_trade),
                                                   kTradeBlock, 0) == hipSuccess && occ > 0)
    g->occupancy_blocks = occ;

  g->nb_log2 = std::max(0, bitlen((uint64_t)std::max<int64_t>(n, 1)) - 1 - 8);
  g->nb = 1 << g->nb_log2;
  g->keybits_node = std::max(1, bitlen((uint64_t)std::max<int64_t>(n - 1, 1)));
  g->keybits_entry = std::max(1, bitlen((uint64_t)std::max<int64_t>(2 * n - 1, 1)));
  g->smax = std::max<int64_t>(d1 + d2, 1);
  g->slot_elems = 3 * g->smax + g->smax / 2 + 1;
  g->sbpre_stride = (n + 4095) / 4096 + 1;
  g->nbig_alloc = std::max(1, g->cu_count / 2);

  // size classes of the per-row rebuild (degrees never change)
  std::vector<int32_t> rs, rm, rb;
  for (int64_t x = 0; x < n; ++x) {
    const int64_t d = row_ptr[x + 1] - row_ptr[x];
    if (d == 0) continue;
    if (d <= kSegSmallMax) rs.push_back((int32_t)x);
    else if (d <= kSegMidMax) rm.push_back((int32_t)x);
    else rb.push_back((int32_t)x);
  }
  g->n_small = (int64_t)rs.size();
  g->n_mid = (int64_t)rm.size();
  g->n_big = (int64_t)rb.size();

  bool ok = alloc_into(g, &g->rp, n + 1) && alloc_into(g, &g->col, nnz) &&
            alloc_into(g, &g->col_t, nnz) && alloc_into(g, &g->col_out, nnz) &&
            alloc_into(g, &g->inbox, nnz) && alloc_into(g, &g->inbox_cur, n) &&
            alloc_into(g, &g->out_cur, n) && alloc_into(g, &g->own_cur, n) && alloc_into(g, &g->perm, n) &&
            alloc_into(g, &g->trade_of, n) && alloc_into(g, &g->tinfo, n) &&
            alloc_into(g, &g->giant_id, n) && alloc_into(g, &g->mtmp, n) &&
            alloc_into(g, &g->mkey, n) && alloc_into(g, &g->dep, g->L) &&
            alloc_into(g, &g->src_list, g->L) && alloc_into(g, &g->tsz, g->L) &&
            alloc_into(g, &g->jobs, 2 * kMaxJobs) && alloc_into(g, &g->qs, (int64_t)kQsShards * std::max<int64_t>(g->L, 1)) &&
            alloc_into(g, &g->qb, (int64_t)kQbShards * std::max<int64_t>(g->L, 1)) && alloc_into(g, &g->bcount, g->nb) &&
            alloc_into(g, &g->bstart, g->nb + 1) && alloc_into(g, &g->bcur, g->nb) &&
            alloc_into(g, &g->ctrl, kCtrlInts) && alloc_into(g, &g->stats, kStatCount) &&
            alloc_into(g, &g->slots, (int64_t)g->nbig_alloc * g->slot_elems) &&
            alloc_into(g, &g->sbpre, (int64_t)g->nbig_alloc * g->sbpre_stride) &&
            alloc_into(g, &g->rows_small, g->n_small) && alloc_into(g, &g->rows_mid, g->n_mid) &&
            alloc_into(g, &g->rows_big, g->n_big);
  if (!ok) {
    release_all(g);
    delete g;
    return fail(CB_ENOMEM, "device allocation failed");
  }
  hipStream_t st = g->stream;
  ok = hip_ok(hipMemcpyAsync(g->rp, row_ptr, (size_t)(n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st), &msg, "copy row_ptr") &&
       (nnz == 0 || hip_ok(hipMemcpyAsync(g->col, col, (size_t)nnz * sizeof(int32_t), hipMemcpyHostToDevice, st), &msg, "copy col")) &&
       (rs.empty() || hip_ok(hipMemcpyAsync(g->rows_small, rs.data(), rs.size() * sizeof(int32_t), hipMemcpyHostToDevice, st), &msg, "copy rows")) &&
       (rm.empty() || hip_ok(hipMemcpyAsync(g->rows_mid, rm.data(), rm.size() * sizeof(int32_t), hipMemcpyHostToDevice, st), &msg, "copy rows")) &&
       (rb.empty() || hip_ok(hipMemcpyAsync(g->rows_big, rb.data(), rb.size() * sizeof(int32_t), hipMemcpyHostToDevice, st), &msg, "copy rows")) &&
       hip_ok(hipMemsetAsync(g->ctrl, 0, kCtrlInts * sizeof(int32_t), st), &msg, "clear ctrl") &&
       hip_ok(hipMemsetAsync(g->jobs, 0, 2 * kMaxJobs * sizeof(HelpJob), st), &msg, "clear jobs") &&
       hip_ok(hipMemsetAsync(g->qs, 0xFF, (size_t)kQsShards * std::max<int64_t>(g->L, 1) * sizeof(int32_t), st), &msg, "clear queues") &&
       hip_ok(hipMemsetAsync(g->qb, 0xFF, (size_t)kQbShards * std::max<int64_t>(g->L, 1) * sizeof(int32_t), st), &msg, "clear queues");
  if (ok && (flags & CB_VALIDATE) && nnz > 0) {
    hipLaunchKernelGGL(k_validate, dim3((unsigned)((nnz + kScanChunk - 1) / kScanChunk)), dim3(256), 0, st,
                       n, nnz, g->rp, g->col, g->ctrl);
    ok = hip_ok(hipGetLastError(), &msg, "k_validate launch");
  }
  if (ok) ok = hip_ok(hipStreamSynchronize(st), &msg, "upload sync");
  int32_t err = 0;
  if (ok) ok = hip_ok(hipMemcpy(&err, g->ctrl + cw(kCwErr), sizeof(int32_t), hipMemcpyDeviceToHost), &msg, "read error word");
  if (!ok) {
    release_all(g);
    delete g;
    return fail(CB_EDEVICE, msg);
  }
  if (err) {
    release_all(g);
    delete g;
    return fail(CB_ENOTSIMPLE, "upload validation: " + error_bits_text(err));
  }
  // giant nodes: the default threshold is max(6144, n / 2048). Reading a
  // giant's set back costs n / 8 bytes of bitmap whatever its degree, sorting
  // a list costs in proportion to the degree; measured on MI355X a round at
  // n = 2^24 is fastest near degree n / 2048 (8192; 2% faster than 16384,
  // 12% faster than 24576), and 6144 keeps every pair below it within one
  // workgroup's LDS (at n = 2^22, 4096 was 1% slower than 6144). It rises
  // further if the bitmaps would take too much memory.
  {
    const int64_t min_deg = std::max<int64_t>(kGiantMinDeg, n / 2048);
    size_t free_b = 0, total_b = 0;
    (void)hipMemGetInfo(&free_b, &total_b);
    const double budget = std::min(64.0 * (1ull << 30), 0.4 * (double)free_b);
    const int64_t gwords = ((n + 4095) / 4096) * 64;
    const double per_giant = (double)gwords * 8.0 + (double)(gwords >> 6) * 4.0;
    std::vector<int64_t> degs;
    for (int64_t x = 0; x < n; ++x) {
      const int64_t d = row_ptr[x + 1] - row_ptr[x];
      if (d >= min_deg) degs.push_back(d);
    }
    std::sort(degs.begin(), degs.end(), std::greater<int64_t>());
    const int64_t fit = (int64_t)(budget / per_giant);
    int64_t thr = min_deg;
    if ((int64_t)degs.size() > fit) thr = fit > 0 ? degs[(size_t)fit - 1] + 1 : INT64_MAX;
    if (thr == INT64_MAX || degs.empty()) thr = 0;
    cb_status gs = setup_giants(g, thr, row_ptr);
    if (gs != CB_OK) {
      release_all(g);
      delete g;
      return gs;
    }
  }
  *out = g;
  return CB_OK;
}

cb_status graph_info(const cb_graph* g, int64_t* n, int64_t* nnz) {
  if (!g) return fail(CB_EINVAL, "null graph");
  if (n) *n = g->n;
  if (nnz) *nnz = g->nnz;
  return CB_OK;
}

cb_status global_trade(cb_graph* g, uint64_t seed, uint32_t round) {
  return enqueue_round(g, seed, round, CB_STEP_REBUILD);
}

cb_status global_trade_steps(cb_graph* g, uint64_t seed, uint32_t round, int32_t last_step) {
  return enqueue_round(g, seed, round, last_step);
}

cb_status graph_sync(cb_graph* g) {
  if (!g) return fail(CB_EINVAL, "null graph");
  return sync_and_check(g);
}

cb_status graph_download(cb_graph* g, int64_t* row_ptr, int32_t* col) {
  if (!g) return fail(CB_EINVAL, "null graph");
  if (g->nnz > 0 && !col) return fail(CB_EINVAL, "col is NULL");
  cb_status s = sync_and_check(g);
  if (s != CB_OK) return s;
  std::string msg;
  if (row_ptr && !hip_ok(hipMemcpy(row_ptr, g->rp, (size_t)(g->n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost), &msg, "download row_ptr"))
    return fail(CB_EDEVICE, msg);
  if (g->nnz > 0 && !hip_ok(hipMemcpy(col, g->col, (size_t)g->nnz * sizeof(int32_t), hipMemcpyDeviceToHost), &msg, "download col"))
    return fail(CB_EDEVICE, msg);
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
  std::string msg;
  if (!hip_ok(hipStreamSynchronize(g->stream), &msg, "hipStreamSynchronize")) return fail(CB_EDEVICE, msg);
  if (count > 0 && !hip_ok(hipMemcpy(host, src, (size_t)count * elem, hipMemcpyDeviceToHost), &msg, "download state"))
    return fail(CB_EDEVICE, msg);
  return CB_OK;
}

cb_status graph_set_option(cb_graph* g, int32_t option, int64_t value) {
  if (!g) return fail(CB_EINVAL, "null graph");
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
      std::vector<int64_t> rp((size_t)g->n + 1);
      std::string msg;
      if (!hip_ok(hipStreamSynchronize(g->stream), &msg, "sync") ||
          !hip_ok(hipMemcpy(rp.data(), g->rp, rp.size() * sizeof(int64_t), hipMemcpyDeviceToHost), &msg, "read row_ptr"))
        return fail(CB_EDEVICE, msg);
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
  std::string msg;
  if (!hip_ok(hipMemcpy(st, g->stats, sizeof(st), hipMemcpyDeviceToHost), &msg, "read stats"))
    return fail(CB_EDEVICE, msg);
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

}  // extern "C"
