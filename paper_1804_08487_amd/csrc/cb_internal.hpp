// Host-side pieces of the library shared between its translation units
// (graph creation from host or device chains, used by the C ABI and by the
// request server). Not part of the C ABI.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "curveball.h"

namespace cbx {

// One chain of a graph being created: n nodes, host CSR offsets rp[0..n] and
// its adjacency (local ids) in host memory, or in device memory with every id
// shifted by dev_shift from local.
struct ChainSrc {
  int64_t n;
  const int64_t* rp;
  const int32_t* col;
  bool col_on_device;
  int32_t dev_shift;
  uint64_t seed;
  uint32_t round;
};

// A new graph of `count` chains (batch: run with batch_run, one chain per
// sample) on the current device, ordered on `stream`.
cb_status create_graph(const ChainSrc* src, int32_t count, void* stream, uint32_t flags, bool batch,
                       cb_graph** out);

// Device bytes such a graph allocates (before giant bitmaps).
size_t graph_bytes(const ChainSrc* src, int32_t count);

// Record `msg` as this thread's last error (cb_last_error) and return s.
cb_status set_error(cb_status s, const char* msg);

// Chain c's adjacency in device memory; its ids are local + *node_base.
int32_t* chain_col(cb_graph* g, int32_t c, int64_t* node_base);

}  // namespace cbx
