/*
 * curveball.h - C ABI of the MI355X (gfx950) global Curveball super-step.
 *
 * One call of global_trade() applies one undirected global trade (Def.
 * "Undirected Global Trade", Sec. 3.3 of Carstens et al., "Parallel and
 * I/O-efficient Randomisation of Massive Networks using Global Curveball
 * Trades") to a device-resident simple graph: floor(n/2) Curveball trades
 * (Def. "Simple Undirected Trade", Sec. 3.2), paired and ordered by a
 * hash-keyed sort of the node ids (Def. "Relaxed global trade", appendix on
 * EM-GCB), each trade keeping the shared neighbours and the u-v edge of its
 * pair and re-splitting the disjoint neighbours uniformly (Sec. 4, trade
 * procedure). The result is the sequential definition's, byte for byte.
 *
 * Random-number convention (the paper leaves the generator open):
 *   philox64(seed; c0..c3) = (w1 << 32) | w0 of Philox4x32-10 (Salmon et al.,
 *     SC'11) keyed by (seed_lo32, seed_hi32), counter (c0, c1, c2, c3);
 *   node v's sort key in round r:  philox64(seed; v, r, 0, 0x4D415443);
 *     trade i pairs the nodes at sorted positions 2i (u) and 2i+1 (v),
 *     ties broken by ascending id; with odd n the last node sits out;
 *   draw j of trade i in round r:   philox64(seed; i, r, j, 0x46595348);
 *   bounded(x, k) = floor(x * k / 2^64);
 *   split of the ascending disjoint set D (|D| = N, a = |A_u \ (A_v u {v})|):
 *     if a <= N - a: for j = 0..a-1:   swap D[j], D[j + bounded(draw j, N - j)]
 *     else:          for j = N-1..a:   swap D[j], D[bounded(draw j, j + 1)]
 *     u receives D[0..a), v receives D[a..N).
 *
 * Graph form: simple undirected graph as symmetric CSR; row_ptr int64[n+1]
 * with row_ptr[0] = 0, col int32[row_ptr[n]] (= 2m), each row strictly
 * ascending, no self id, 0 <= n <= 2^31 - 1, 2m < 2^31. Degrees never change,
 * so row_ptr is the same after every round; rows stay ascending.
 *
 * Errors: every call returns cb_status; no exception crosses the ABI.
 * cb_last_error() gives a thread-local message for the last failure.
 * Argument and validation errors return at once and change nothing. A fault
 * found on the device (a watchdog time-out of the trade kernel, an
 * impossible counter) is reported by the next synchronising call
 * (graph_sync, graph_download, graph_stats); the handle is then poisoned and
 * only graph_free is valid.
 */
#ifndef CURVEBALL_H
#define CURVEBALL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cb_graph cb_graph;

typedef enum {
    CB_OK = 0,
    CB_EINVAL = 1,      /* bad argument */
    CB_ENOTSIMPLE = 2,  /* upload validation: not a simple symmetric sorted CSR */
    CB_ENOMEM = 3,      /* device allocation failed; nothing was kept */
    CB_EDEVICE = 4,     /* HIP error or device-side invariant violation */
    CB_EWATCHDOG = 5,   /* trade kernel made no progress within the limit */
    CB_EPOISONED = 6    /* handle unusable after an earlier device error */
} cb_status;

/* Device memory provider. alloc returns device memory of `bytes` (or NULL);
 * free releases it. Both run on the host, never inside a kernel. */
typedef struct {
    void* (*alloc)(size_t bytes, void* user);
    void (*free)(void* ptr, void* user);
    void* user;
} cb_allocator;

/* Set the provider used by later graph_upload calls (NULL: hipMalloc). */
cb_status cb_set_allocator(const cb_allocator* allocator);

/* Upload flags. */
#define CB_VALIDATE 1u  /* check simple / sorted / symmetric on the device */

/* Copy a host CSR (row_ptr: n+1 int64, col: row_ptr[n] int32; the caller
 * keeps ownership) to the current HIP device and create a handle that owns
 * all device state of one chain. The graph is the paper's simple undirected
 * graph on nodes 0..n-1 (Sec. 2, Preliminaries and Notation): no loops, no
 * multi-edges, each edge {x, y} stored in both rows, as the trade's
 * neighbourhoods A_x (Def. "Simple Undirected Trade", Sec. 3.2). With
 * CB_VALIDATE the device checks that form (CB_ENOTSIMPLE otherwise).
 * stream: a hipStream_t on which every later call of this handle is ordered
 * (NULL: the handle creates its own). Synchronises the stream before
 * returning. Errors: CB_EINVAL (sizes, NULL pointers, offsets),
 * CB_ENOTSIMPLE, CB_ENOMEM (nothing is kept), CB_EDEVICE. */
cb_status graph_upload(int64_t n, const int64_t* row_ptr, const int32_t* col,
                       void* stream, uint32_t flags, cb_graph** out);

/* Sizes for download buffers: n and nnz = 2m (each undirected edge of the
 * graph, Sec. 2, counts once in each of its two rows). */
cb_status graph_info(const cb_graph* g, int64_t* n, int64_t* nnz);

/* Apply one global trade (Def. "Undirected Global Trade", Sec. 3.3) with
 * the given chain seed and round number, under the random-number convention
 * above. Asynchronous: enqueued on the handle's stream, returns before it
 * runs; device-side faults surface at the next synchronising call. For a
 * graph from batch_upload: CB_EINVAL (use batch_run). */
cb_status global_trade(cb_graph* g, uint64_t seed, uint32_t round);

/* Wait for all enqueued work; report device-side faults. */
cb_status graph_sync(cb_graph* g);

/* Synchronise and copy the current graph into caller buffers of n+1 and
 * nnz entries (row_ptr may be NULL: it equals the uploaded one, because a
 * trade preserves every degree, Sec. 3.2). Rows come back strictly
 * ascending. Reports device-side faults (then the handle is poisoned). */
cb_status graph_download(cb_graph* g, int64_t* row_ptr, int32_t* col);

/* Release all device memory of the handle (NULL is a no-op). */
void graph_free(cb_graph* g);

/* Message of the last failed call on this thread ("" if none). */
const char* cb_last_error(void);

/* ---- step-wise execution and state readout (parity tests) ------------- */

/* Steps of one global trade, in order. */
#define CB_STEP_MATCHING 1  /* keys, bucket sort, perm, trade_of */
#define CB_STEP_DEPSCAN  2  /* per-trade count of edges to earlier trades */
#define CB_STEP_TRADE    3  /* persistent trade kernel (col_out filled) */
#define CB_STEP_REBUILD  4  /* per-row sort of col_out into col */

/* Run the steps 1..last_step of global_trade(seed, round). A call with
 * last_step < CB_STEP_REBUILD leaves the graph state unusable for further
 * trades until graph_upload; it exists to read intermediate state. */
cb_status global_trade_steps(cb_graph* g, uint64_t seed, uint32_t round, int32_t last_step);

/* Device state readable after a (partial) round. */
#define CB_STATE_PERM     1  /* int32[n]: nodes in sorted key order */
#define CB_STATE_TRADE_OF 2  /* int32[n]: trade of each node, INT32_MAX if none */
#define CB_STATE_DEP      3  /* int32[n/2]: dependency counts after DEPSCAN */
#define CB_STATE_COL      4  /* int32[nnz]: current adjacency (rows ascending) */
#define CB_STATE_OUT_CUR  5  /* int32[n]: final edges written into each row from
                                its front this round */
#define CB_STATE_OWN_CUR  8  /* int32[n]: edges a workgroup trade wrote into its
                                own rows from their back (with OUT_CUR the
                                degree after a full round) */
#define CB_STATE_INBOX_CUR 6 /* int32[n]: edges handed to each row this round */
#define CB_STATE_TRACE    7  /* int64[24 * floor(n/2)] (CB_OPT_TRACE): per trade k
                                at 24k + i: i=0 tick at which it became ready
                                (-1: a source), 1 start and 2 end of its
                                execution, 3 trade whose release made it ready
                                (-1: a source); for trades run by a workgroup
                                also 4 both lists collected, 5 sorted or merged,
                                6 classified, 7 split and own rows reserved,
                                8 deg u + deg v, 9 kind (1 giant node, 2 in LDS,
                                3 in global scratch), 10 deg u, 11 deg v,
                                12 disjoint entries, 13 of which u's, 14 end of
                                the bit pass of a giant node's list (the last
                                one taken; with a small other side, the end of
                                the one fused pass), 15 fused pass: counts
                                and ranges set up; for a write phase shared
                                with helpers 16 arrays published, 17 own
                                chunks done, 18 all chunks done, 19 chunks
                                written by the owner; fused pass: 20 last
                                bitmap reader done, 21 last entry writer
                                done, 22 waits of its bitmap readers for
                                ring space, 23 waits of its entry writers
                                for ring entries. Ticks of
                                the device's constant 100 MHz clock; -1 where
                                not recorded */

/* Synchronise and copy `count` elements of state `which` to host memory
 * (elements are int32 except for CB_STATE_TRACE, int64). Also valid on a
 * poisoned handle (diagnosis after a device error). */
cb_status graph_download_state(cb_graph* g, int32_t which, void* host, int64_t count);

/* ---- options ------------------------------------------------------------ */
#define CB_OPT_SMALL_MAX     1  /* trades with deg u + deg v <= this run on one
                                   wavefront (0..512); larger ones on a whole
                                   workgroup. Default 512. */
#define CB_OPT_BIG_WORKERS   2  /* workgroups reserved for large trades (>= 1) */
#define CB_OPT_GRID_BLOCKS   3  /* workgroups of the trade kernel (0 = auto: one per
                                   CU; for a graph with giant nodes and average
                                   degree at least 32, the workgroup workers
                                   plus a quarter of the CUs) */
#define CB_OPT_WATCHDOG_MS   4  /* idle time after which the trade kernel gives up */
#define CB_OPT_TIMING        5  /* 1: time every kernel with HIP events */
#define CB_OPT_LOCAL_STACK   6  /* ready trades a wavefront keeps for itself (0..16) */
#define CB_OPT_BIG_LDS_MAX   7  /* workgroup trades with deg u + deg v <= this
                                   stay in LDS (0..12288); larger ones use a
                                   global scratch slot. Default 12288. */
#define CB_OPT_DEBUG_CHECKS  9  /* 1: extra invariant checks between kernels */
#define CB_OPT_HELP_MIN     11  /* workgroup trades with deg u + deg v >= this
                                   let idle wavefronts of the kernel share their
                                   write phase (0 = never). Default 4096. */
#define CB_OPT_HELP_GROUPS  12  /* workgroup workers help the shared phases of
                                   owners in their residue class modulo this
                                   (a divisor of 64; default 2) */
#define CB_OPT_TRACE        10  /* 1: record per-trade times (CB_STATE_TRACE);
                                   allocates 192 bytes per trade on first use */
#define CB_OPT_GIANT_DEG     8  /* nodes of at least this degree keep the edges
                                   handed to them in a bitmap over all node ids
                                   (n/8 bytes each) instead of a list; 0 = none.
                                   Default max(6144, n/2048), raised while the
                                   bitmaps would exceed min(64 GiB, 40% of free
                                   memory). */

#define CB_OPT_HELP_CHUNK   13  /* items per chunk a helper claims from a shared
                                   write phase (a multiple of 64 in [64, 4096];
                                   default 128) */

#define CB_OPT_IDLE_BACKOFF 15  /* longest sleep of an idle wavefront worker
                                   between polls of the ready queues, in units of
                                   2048 cycles (1..1024; default 128, about
                                   110 us) */
#define CB_OPT_CU_POOL      16  /* 1 (default): ready small trades beyond a wavefront's
                                   local stack go first to a pool in its
                                   workgroup's LDS, where idle wavefronts of the
                                   same CU take them; 0: straight to the global
                                   queues */
#define CB_OPT_FUSE_NEXT    14  /* 1 (default): a full round also prepares the next
                                   one (its matching, run once this round's trade
                                   kernel is done, and its dependency scan, done
                                   by the rebuild as it writes each row); the next
                                   round then starts at its sources. A single
                                   chain is prepared for (seed, round + 1); a
                                   call with another (seed, round) starts over.
                                   After a full round the state arrays
                                   (CB_STATE_PERM, _TRADE_OF, _DEP) hold the
                                   prepared round's. 0: every round runs all
                                   steps. */

/* Set an option of a graph (any option may change between rounds; none
 * changes the result, only how the work is scheduled). */
cb_status graph_set_option(cb_graph* g, int32_t option, int64_t value);

/* Counters of the last completed round (synchronises). */
typedef struct {
    int64_t trades;          /* floor(n/2) */
    int64_t small_trades;    /* run by one wavefront */
    int64_t big_trades;      /* run by a workgroup */
    int64_t sources;         /* trades with no earlier neighbour */
    int64_t queue_pushes;    /* ready trades handed over through global queues */
    int64_t work;            /* sum of deg u + deg v over trades */
    int64_t forwarded;       /* edges handed to a later trade */
    int64_t emitted;         /* final edges written (both directions counted once) */
    int64_t small_workers;   /* wavefront workers of the trade kernel */
    int64_t big_workers;     /* workgroup workers of the trade kernel */
    double small_busy_us;    /* summed time wavefronts spent inside trades */
    double big_busy_us;      /* summed time workgroups spent inside trades */
    double big_gather_us;    /* ... collecting and sorting the two lists */
    double big_split_us;     /* ... classifying and splitting */
    double big_write_us;     /* ... writing final edges, forwarding and
                                unlocking later trades */
    double big_release_us;   /* 0: unlocking is part of the write phase */
    double big_max_us;       /* longest single workgroup trade */
    int64_t moved;           /* disjoint neighbours that changed sides, over the
                                counted trades (a swap moves two: the paper's
                                swap fraction is moved / work, appendix on
                                swaps performed) */
    int64_t counted_trades;  /* trades whose moves were counted: all except those
                                whose write phase was shared (CB_OPT_HELP_MIN 0
                                counts every trade) */
} cb_round_stats;

cb_status graph_stats(cb_graph* g, cb_round_stats* out);

/* Kernel timing (CB_OPT_TIMING): mean milliseconds per round of each step,
 * ms[0..4) = matching, depscan, trade, rebuild; rounds timed in *rounds. */
cb_status graph_kernel_times(cb_graph* g, double* ms, int32_t count, int64_t* rounds);

/* ---- batched chains --------------------------------------------------------
 * Many independent chains on their own graphs advance together: each round of
 * a batch is one undirected global trade (Def. "Undirected Global Trade",
 * Sec. 3.3) of every chain, run as one global trade of the disjoint union of
 * the chains' graphs whose pairing and split draws are those of each chain on
 * its own (the chain's seed, its round counter, its local node ids and trade
 * indices). No edge joins two chains, so no trade of one chain changes the
 * edges another chain sees, and every chain's result is byte for byte the one
 * it would have alone (Def. "Relaxed global trade", appendix on EM-GCB: the
 * pairing is the sort order of a hash of the node ids). This is how many
 * null-model samples share one GPU: one launch sequence per round for all
 * chains, the dependency chains of different graphs overlapping in one
 * persistent trade kernel. */

/* Upload `chains` graphs (chain c: n[c] nodes, host CSR row_ptr[c] of n[c]+1
 * int64 and col[c] of row_ptr[c][n[c]] int32 with local ids 0..n[c]-1, the
 * graph form above) with chain seeds seeds[c] and first rounds first_round[c]
 * (NULL: all 0). The caller keeps ownership of every host array. One handle
 * owns the device state of all chains. Synchronises `stream` (NULL: the
 * handle creates its own) before returning. Errors as graph_upload; ids
 * outside [0, n[c]) give CB_ENOTSIMPLE. */
cb_status batch_upload(int32_t chains, const int64_t* n, const int64_t* const* row_ptr,
                       const int32_t* const* col, const uint64_t* seeds, const uint32_t* first_round,
                       void* stream, uint32_t flags, cb_graph** out);

/* Run `rounds` rounds of every chain of a batch (chain c applies its rounds
 * r_c, r_c + 1, ...; each chain's round counter then advances by `rounds`).
 * The launch sequence of `rounds` rounds is captured once as a hipGraph (again
 * after an option change) and launched on the handle's stream; asynchronous.
 * With timing or tracing on, the rounds are launched one by one instead. */
cb_status batch_run(cb_graph* g, uint32_t rounds);

/* Size of chain `chain` (nodes, entries) and the round it applies next. */
cb_status batch_info(const cb_graph* g, int32_t chain, int64_t* n, int64_t* nnz, uint32_t* next_round);

/* Synchronise and copy chain `chain`'s adjacency (local ids, rows ascending,
 * row_ptr unchanged) into col (its nnz entries). */
cb_status batch_download(cb_graph* g, int32_t chain, int32_t* col);

/* ---- autotuner --------------------------------------------------------------
 * Chooses the trade kernel's workgroups (CB_OPT_GRID_BLOCKS), the workgroup
 * pool (CB_OPT_CU_POOL), the idle wavefronts' back-off
 * (CB_OPT_IDLE_BACKOFF), their local
 * stack of ready trades (CB_OPT_LOCAL_STACK), the wavefront/workgroup size
 * threshold (CB_OPT_SMALL_MAX), the size from which write phases are shared
 * (CB_OPT_HELP_MIN), their chunk size (CB_OPT_HELP_CHUNK) and the workgroup
 * workers (CB_OPT_BIG_WORKERS) by
 * timing `trial_rounds` rounds per candidate from the graph's current state
 * (coordinate descent from the current options; a candidate replaces the
 * best only when it is more than 1% faster), then restores that state and
 * keeps the fastest options. The schedule never changes a result. Results are
 * cached for the process by the shape of the graph (log2 of chains, nodes,
 * entries and largest degree); with use_cache != 0 a cached choice is applied
 * without timing. Synchronises. Allocates a temporary copy of the adjacency. */
typedef struct {
    int32_t small_max;
    int32_t help_min;
    int32_t help_chunk;
    int32_t big_workers;
    int32_t local_stack;          /* CB_OPT_LOCAL_STACK */
    int32_t idle_backoff;         /* CB_OPT_IDLE_BACKOFF */
    int32_t cu_pool;              /* CB_OPT_CU_POOL */
    int32_t grid_blocks;          /* CB_OPT_GRID_BLOCKS */
    double ms_per_round;          /* of the chosen options */
    double default_ms_per_round;  /* of the options the tuner started from */
    int32_t evaluated;            /* timed candidates (0 when taken from the cache) */
    int32_t cached;               /* 1: taken from the cache */
} cb_tune_result;

cb_status graph_autotune(cb_graph* g, uint32_t trial_rounds, int32_t use_cache, cb_tune_result* out);

/* ---- uniform single trades ------------------------------------------------
 * Simple Undirected Curveball (Sec. 3.2, the paragraph after the trade
 * figure): a chain of single trades, each of a node pair drawn uniformly at
 * random with a uniform split (the comparison chain of the mixing study,
 * Sec. 5.1, where n/2 single trades make one super-step). Step s of the chain
 * with seed `seed` trades u = bounded(philox64(seed; s_lo, s_hi, 0,
 * 0x43425550), n) and v = bounded(philox64(seed; s_lo, s_hi, 1, 0x43425550),
 * n - 1), plus one if v >= u; its split draws philox64(seed; s, 0xFFFFFFFF,
 * j, 0x46595348) with the rule above (u is the first node).
 * Apply steps step0 .. step0 + steps - 1 (below 2^32) to a graph from
 * graph_upload, one after the other in effect: runs of steps whose pairs share
 * no node go through the trade kernel as one partial global trade. Needs
 * giant nodes off (CB_OPT_GIANT_DEG 0). Synchronises. Round statistics
 * (graph_stats) then sum over the steps. */
cb_status cbu_trades(cb_graph* g, uint64_t seed, uint64_t step0, uint64_t steps);

/* ---- request server (continuous batching) ----------------------------------
 * Serves requests "`samples` samples of G after `rounds` global trades": sample
 * j of a request with seed s is G after rounds 0..rounds-1 of the chain with
 * seed s + j (Def. "Undirected Global Trade", Sec. 3.3; each sample is an
 * independent run of the chain, for null-model sampling). Requests queue in
 * arrival order and are admitted while the device memory of their chains
 * fits half of `hbm_budget_bytes` (the other half covers the rebuild of the
 * union below). All chains of all admitted requests advance together, one
 * round per server_step, as one batch (see batch_run); a chain that finishes
 * is copied to host memory and leaves; requests admitted later join the
 * running batch, whose device state is rebuilt on the device whenever its
 * chains change (every chain keeps its adjacency, seed and round). Chain
 * state stays on the device from admission to the last round. A result
 * depends only on (G, seed, sample, rounds): it is the same alone and in any
 * mix. One host thread drives a server. */
typedef struct cb_server cb_server;
typedef struct {
    int64_t queued;             /* requests waiting for admission */
    int64_t active_chains;      /* chains on the device */
    int64_t finished_requests;  /* requests whose samples are all done */
    int64_t steps;              /* rounds run */
    int64_t repacks;            /* rebuilds of the batch after admissions/retirements */
    int64_t active_bytes;       /* device bytes held for admitted requests */
    int64_t budget_bytes;
} cb_server_status;

/* A server on the current device, ordered on `stream` (NULL: its own). */
cb_status server_create(size_t hbm_budget_bytes, void* stream, cb_server** out);

/* Queue a request (host CSR in the graph form above, copied; samples >= 1).
 * CB_ENOMEM if its chains alone need more than half the budget. */
cb_status server_submit(cb_server* s, int64_t n, const int64_t* row_ptr, const int32_t* col,
                        int32_t samples, uint32_t rounds, uint64_t seed, int64_t* request_id);

/* One scheduling step: admit what fits, rebuild the batch if its chains
 * changed, run one round of every active chain, copy out finished chains.
 * Synchronises when a chain finishes. `status` may be NULL. */
cb_status server_step(cb_server* s, cb_server_status* status);

/* *finished = 1 once every sample of the request is done. */
cb_status server_request_state(cb_server* s, int64_t request_id, int32_t* finished);

/* Copy sample `sample` of a finished request into col (row_ptr[n] entries). */
cb_status server_result(cb_server* s, int64_t request_id, int32_t sample, int32_t* col);

/* Forget a finished request (its results). */
cb_status server_release(cb_server* s, int64_t request_id);

/* Release the server and all its device memory (NULL is a no-op). */
void server_free(cb_server* s);

/* ---- no device allocation -------------------------------------------------
 * For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc). One global trade
 * (the result of graph_upload + global_trade(seed, round) + graph_download,
 * byte for byte) of a graph the caller holds: row_ptr in host memory (n+1
 * int64), col in device memory (row_ptr[n] int32, the graph form above; read
 * and overwritten with the result). Every other buffer lives in the library's
 * static device array of 64 MiB (each GPU the library runs on holds its own
 * copy until the process ends); no device or host allocation is made. A graph
 * that needs more than the array holds is rejected with CB_EINVAL before any
 * device work. Calls on one GPU run one after the other (the array keeps the
 * last call's contents and every call sets up what it needs); the call
 * synchronises `stream` (NULL: the null stream) before returning. Errors are
 * reported by the return value; there is no handle to poison. Giant-node
 * bitmaps, tracing and timing are not available on this path. */
cb_status global_trade_static(int64_t n, const int64_t* row_ptr, int32_t* col, uint64_t seed,
                              uint32_t round, void* stream);

#ifdef __cplusplus
}
#endif
#endif
