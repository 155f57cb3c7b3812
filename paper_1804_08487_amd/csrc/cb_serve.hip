// Request server: "k samples of G after r global trades" requests served by
// continuous batching. Every admitted request becomes k independent chains
// (sample j of a request with seed s is the chain with seed s + j, rounds
// 0..r-1). All active chains of all admitted requests form one union graph
// that advances one round per server step (batch_run); chains that finish
// are downloaded and leave, queued requests are admitted as their device
// memory fits the budget, and the union is rebuilt on the device (each
// chain's current adjacency copied with its ids moved to their new range)
// whenever its membership changes. A chain's result depends only on its
// graph, seed and rounds, so it is the same alone and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <deque>
#include <map>
#include <memory>
#include <vector>

#include "curveball.h"
#include "cb_internal.hpp"

namespace {

struct ServeRequest {
  int64_t id = 0;
  int64_t n = 0, nnz = 0;
  std::vector<int64_t> rp;
  std::vector<int32_t> col;          // host copy until its chains join the union
  int32_t samples = 0;
  uint32_t rounds = 0;
  uint64_t seed = 0;
  size_t bytes = 0;                  // device bytes its chains add to a union (estimate)
  int32_t* dev_col = nullptr;        // device copy while its chains wait to join
  std::vector<std::vector<int32_t>> results;
  int32_t samples_done = 0;
  int32_t chains_waiting = 0;        // chains not yet in the union
};

struct ServeChain {
  ServeRequest* req;
  int32_t sample;
  uint32_t done_rounds;
  int32_t slot;                      // index in the current union, -1: not in it yet
};

}  // namespace

struct cb_server {
  size_t budget = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::deque<ServeRequest*> queue;
  std::map<int64_t, std::unique_ptr<ServeRequest>> requests;
  std::vector<ServeChain> active;
  cb_graph* uni = nullptr;
  bool dirty = false;
  size_t active_bytes = 0;
  int64_t next_id = 1;
  int64_t steps = 0, repacks = 0, finished = 0;
};

namespace {

cb_status sfail(cb_status s, const char* msg) { return cbx::set_error(s, msg); }

// SplitMix64 finaliser of (a, b): the symmetry checksum of submitted graphs.
uint64_t pair_hash(uint64_t a, uint64_t b) {
  uint64_t z = (a << 32 | b) + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Options of every union: the batched workload's tuned schedule (deep local
// stacks and long idle back-off pay off when many chains share the device).
void serving_options(cb_graph* g) {
  (void)graph_set_option(g, CB_OPT_LOCAL_STACK, 16);
  (void)graph_set_option(g, CB_OPT_IDLE_BACKOFF, 128);
  (void)graph_set_option(g, CB_OPT_SMALL_MAX, 384);
  (void)graph_set_option(g, CB_OPT_HELP_MIN, 1024);
}

cb_status finish_sample(cb_server* s, ServeChain& c) {
  ServeRequest* q = c.req;
  q->samples_done += 1;
  if (q->samples_done == q->samples) {
    s->finished += 1;
    s->active_bytes -= std::min(s->active_bytes, q->bytes);
  }
  return CB_OK;
}

// Build the union of the active chains on the device (existing chains from
// the current union, new ones from their request's device copy).
cb_status repack(cb_server* s) {
  cb_graph* old = s->uni;
  if (s->active.empty()) {
    if (old) graph_free(old);
    s->uni = nullptr;
    s->dirty = false;
    return CB_OK;
  }
  std::vector<cbx::ChainSrc> src(s->active.size());
  for (size_t i = 0; i < s->active.size(); ++i) {
    ServeChain& c = s->active[i];
    ServeRequest* q = c.req;
    cbx::ChainSrc& d = src[i];
    d.n = q->n;
    d.rp = q->rp.data();
    d.col_on_device = true;
    d.seed = q->seed + (uint64_t)c.sample;
    d.round = c.done_rounds;
    if (c.slot >= 0) {
      int64_t nb = 0;
      d.col = cbx::chain_col(old, c.slot, &nb);
      d.dev_shift = (int32_t)nb;
    } else {
      d.col = q->dev_col;
      d.dev_shift = 0;
    }
  }
  cb_graph* nu = nullptr;
  cb_status st = cbx::create_graph(src.data(), (int32_t)src.size(), s->stream, 0, true, &nu);
  if (st != CB_OK) return st;
  serving_options(nu);
  if (old) graph_free(old);
  s->uni = nu;
  for (size_t i = 0; i < s->active.size(); ++i) {
    ServeChain& c = s->active[i];
    if (c.slot < 0) {
      c.req->chains_waiting -= 1;
      if (c.req->chains_waiting == 0 && c.req->dev_col) {
        (void)hipFree(c.req->dev_col);
        c.req->dev_col = nullptr;
      }
    }
    c.slot = (int32_t)i;
  }
  s->dirty = false;
  s->repacks += 1;
  return CB_OK;
}

// Admit queued requests, first come first served, while their chains fit half
// the budget (the other half holds the union being replaced during a repack).
cb_status admit(cb_server* s) {
  while (!s->queue.empty()) {
    ServeRequest* q = s->queue.front();
    if (s->active_bytes + q->bytes > s->budget / 2) break;
    s->queue.pop_front();
    s->active_bytes += q->bytes;
    q->results.assign((size_t)q->samples, std::vector<int32_t>());
    if (q->rounds == 0) {   // nothing to trade: every sample is the graph itself
      for (auto& r : q->results) r = q->col;
      q->samples_done = q->samples;
      s->finished += 1;
      s->active_bytes -= std::min(s->active_bytes, q->bytes);
      continue;
    }
    const size_t cb = (size_t)std::max<int64_t>(q->nnz, 1) * sizeof(int32_t);
    if (hipMalloc(&q->dev_col, cb) != hipSuccess) {
      (void)hipGetLastError();
      return sfail(CB_ENOMEM, "no device memory for an admitted request");
    }
    if (q->nnz > 0 &&
        hipMemcpyAsync(q->dev_col, q->col.data(), (size_t)q->nnz * sizeof(int32_t), hipMemcpyHostToDevice,
                       s->stream) != hipSuccess)
      return sfail(CB_EDEVICE, "request upload failed");
    q->chains_waiting = q->samples;
    for (int32_t j = 0; j < q->samples; ++j) s->active.push_back(ServeChain{q, j, 0u, -1});
    s->dirty = true;
  }
  return CB_OK;
}

}  // namespace

extern "C" {

cb_status server_create(size_t hbm_budget_bytes, void* stream, cb_server** out) {
  if (!out) return sfail(CB_EINVAL, "out is NULL");
  *out = nullptr;
  if (hbm_budget_bytes < ((size_t)1 << 20)) return sfail(CB_EINVAL, "budget below 1 MiB");
  cb_server* s = new cb_server();
  s->budget = hbm_budget_bytes;
  if (stream) {
    s->stream = (hipStream_t)stream;
  } else {
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
      delete s;
      return sfail(CB_EDEVICE, "hipStreamCreate failed");
    }
    s->own_stream = true;
  }
  *out = s;
  return CB_OK;
}

cb_status server_submit(cb_server* s, int64_t n, const int64_t* row_ptr, const int32_t* col, int32_t samples,
                        uint32_t rounds, uint64_t seed, int64_t* request_id) {
  if (!s || !request_id) return sfail(CB_EINVAL, "null argument");
  if (samples < 1) return sfail(CB_EINVAL, "a request needs at least one sample");
  if (n < 0 || n > INT32_MAX || !row_ptr || row_ptr[0] != 0) return sfail(CB_EINVAL, "bad graph sizes");
  const int64_t nnz = row_ptr[n];
  if (nnz < 0 || nnz >= INT32_MAX || (nnz > 0 && !col)) return sfail(CB_EINVAL, "bad graph sizes");
  for (int64_t x = 0; x < n; ++x)
    if (row_ptr[x + 1] < row_ptr[x]) return sfail(CB_EINVAL, "row_ptr is not monotone");
  // simple, sorted and symmetric: rows strictly ascending without the own id,
  // and the sum of a hash over (x, y) equals that over (y, x) (an asymmetric
  // entry breaks it with probability 1 - 2^-64)
  uint64_t acc = 0;
  for (int64_t x = 0; x < n; ++x)
    for (int64_t e = row_ptr[x]; e < row_ptr[x + 1]; ++e) {
      const int32_t y = col[e];
      if (y < 0 || y >= n) return sfail(CB_ENOTSIMPLE, "a neighbour id is outside [0, n)");
      if (y == x || (e > row_ptr[x] && col[e - 1] >= y))
        return sfail(CB_ENOTSIMPLE, "rows must be strictly ascending without the own id");
      acc += pair_hash((uint64_t)x, (uint64_t)y) - pair_hash((uint64_t)y, (uint64_t)x);
    }
  if (acc != 0) return sfail(CB_ENOTSIMPLE, "the adjacency is not symmetric");
  auto q = std::make_unique<ServeRequest>();
  q->id = s->next_id++;
  q->n = n;
  q->nnz = nnz;
  q->rp.assign(row_ptr, row_ptr + n + 1);
  q->col.assign(col, col + nnz);
  q->samples = samples;
  q->rounds = rounds;
  q->seed = seed;
  std::vector<cbx::ChainSrc> src((size_t)samples,
                                 cbx::ChainSrc{n, q->rp.data(), q->col.data(), false, 0, seed, 0});
  q->bytes = cbx::graph_bytes(src.data(), samples) + (size_t)nnz * sizeof(int32_t);
  if (q->bytes > s->budget / 2) return sfail(CB_ENOMEM, "request larger than half the memory budget");
  *request_id = q->id;
  s->queue.push_back(q.get());
  s->requests[q->id] = std::move(q);
  return CB_OK;
}

cb_status server_step(cb_server* s, cb_server_status* out) {
  if (!s) return sfail(CB_EINVAL, "null server");
  cb_status st = admit(s);
  if (st != CB_OK) return st;
  if (s->dirty) {
    st = repack(s);
    if (st != CB_OK) return st;
  }
  if (s->uni) {
    st = batch_run(s->uni, 1);
    if (st != CB_OK) return st;
    s->steps += 1;
    bool any = false;
    for (ServeChain& c : s->active) {
      c.done_rounds += 1;
      if (c.done_rounds == c.req->rounds) {
        std::vector<int32_t>& r = c.req->results[(size_t)c.sample];
        r.resize((size_t)c.req->nnz);
        st = batch_download(s->uni, c.slot, r.data());
        if (st != CB_OK) return st;
        finish_sample(s, c);
        any = true;
      }
    }
    if (any) {
      s->active.erase(std::remove_if(s->active.begin(), s->active.end(),
                                     [](const ServeChain& c) { return c.done_rounds == c.req->rounds; }),
                      s->active.end());
      s->dirty = true;
    }
  }
  if (out) {
    out->queued = (int64_t)s->queue.size();
    out->active_chains = (int64_t)s->active.size();
    out->finished_requests = s->finished;
    out->steps = s->steps;
    out->repacks = s->repacks;
    out->active_bytes = (int64_t)s->active_bytes;
    out->budget_bytes = (int64_t)s->budget;
  }
  return CB_OK;
}

cb_status server_request_state(cb_server* s, int64_t request_id, int32_t* finished) {
  if (!s || !finished) return sfail(CB_EINVAL, "null argument");
  auto it = s->requests.find(request_id);
  if (it == s->requests.end()) return sfail(CB_EINVAL, "unknown request");
  *finished = it->second->samples_done == it->second->samples && !it->second->results.empty();
  return CB_OK;
}

cb_status server_result(cb_server* s, int64_t request_id, int32_t sample, int32_t* col) {
  if (!s) return sfail(CB_EINVAL, "null server");
  auto it = s->requests.find(request_id);
  if (it == s->requests.end()) return sfail(CB_EINVAL, "unknown request");
  ServeRequest* q = it->second.get();
  if (sample < 0 || sample >= q->samples) return sfail(CB_EINVAL, "sample out of range");
  if (q->results.empty() || q->results[(size_t)sample].size() != (size_t)q->nnz)
    return sfail(CB_EINVAL, "sample not finished");
  if (q->nnz > 0 && !col) return sfail(CB_EINVAL, "col is NULL");
  std::copy(q->results[(size_t)sample].begin(), q->results[(size_t)sample].end(), col);
  return CB_OK;
}

cb_status server_release(cb_server* s, int64_t request_id) {
  if (!s) return sfail(CB_EINVAL, "null server");
  auto it = s->requests.find(request_id);
  if (it == s->requests.end()) return sfail(CB_EINVAL, "unknown request");
  ServeRequest* q = it->second.get();
  if (q->samples_done != q->samples) return sfail(CB_EINVAL, "request not finished");
  s->requests.erase(it);
  return CB_OK;
}

void server_free(cb_server* s) {
  if (!s) return;
  if (s->uni) graph_free(s->uni);
  for (auto& kv : s->requests)
    if (kv.second->dev_col) (void)hipFree(kv.second->dev_col);
  if (s->own_stream && s->stream) {
    (void)hipStreamSynchronize(s->stream);
    (void)hipStreamDestroy(s->stream);
  }
  delete s;
}

}  // extern "C"
