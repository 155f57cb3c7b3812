/*
 * CPU oracle for the global Curveball super-step (Carstens, Hamann, Meyer,
 * Penschuck, Tran, Wagner: "Parallel and I/O-efficient Randomisation of
 * Massive Networks using Global Curveball Trades").
 *
 * TEST INFRASTRUCTURE. Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py load this library. The GPU library shares no
 * code, header, table or constant generator with it and never links it.
 *
 * Graph form: simple undirected graph as symmetric CSR. row_ptr int64[n+1],
 * col int32[row_ptr[n]], every row strictly ascending, no self id. Degrees
 * are invariant under trades, so row_ptr never changes.
 *
 * Randomness (the paper fixes no generator; this is the project's own
 * convention, shared with the GPU path only as a written specification):
 *   philox64(seed; c0,c1,c2,c3) = (w1 << 32) | w0 of Philox4x32-10 with
 *     key (seed_lo32, seed_hi32) and counter (c0,c1,c2,c3)  [Salmon et al.,
 *     "Parallel random numbers: as easy as 1, 2, 3", SC'11].
 *   matching key of node v in round r: philox64(seed; v, r, 0, TAG_M)
 *   draw j of trade i in round r:        philox64(seed; i, r, j, TAG_F)
 *   bounded(x, k) = floor(x * k / 2^64)  (multiply-high, no rejection)
 */
#ifndef CURVEBALL_ORACLE_H
#define CURVEBALL_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_TAG_M 0x4D415443u /* "MATC" */
#define ORC_TAG_F 0x46595348u /* "FYSH" */
#define ORC_TAG_U 0x43425550u /* "CBUP": node pair of a uniform single trade */
#define ORC_CBU_ROUND 0xFFFFFFFFu /* round word of a single trade's split draws */
#define ORC_UNMATCHED INT32_MAX

typedef struct {
    int64_t trades;    /* floor(n/2) */
    int64_t work;      /* sum over trades of deg(u) + deg(v) */
    int64_t common;    /* sum of |C| (shared neighbours, kept) */
    int64_t disjoint;  /* sum of |D| (disjoint neighbours, re-split) */
    int64_t moved;     /* sum of |X \ U| + |Y \ W| (edges that changed side) */
    int64_t uv_edges;  /* trades whose two nodes are adjacent */
    int64_t max_s;     /* max over trades of deg(u) + deg(v) */
    int64_t unmatched; /* node left out when n is odd, else -1 */
    int64_t dep_mismatch; /* O2 only: trades whose received count != depcount */
    double setup_seconds; /* O2 only: wall time before the first trade */
    double trade_seconds; /* O2 only: wall time of the trades run */
    double rebuild_seconds; /* O2 only: wall time of the final row rebuild */
} orc_stats;

/* Philox4x32-10, one block. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
uint64_t orc_philox64(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3);
uint64_t orc_bounded(uint64_t x, uint64_t k);

/* Matching (Def. "Undirected Global Trade" with a relaxed hash-defined
 * permutation, Def. "Relaxed global trade"): order[] = nodes sorted by
 * (key, id). Trade i pairs order[2i] (called u) and order[2i+1] (called v).
 * trade_of[x] = position/2, or ORC_UNMATCHED for the last node if n is odd.
 * Either output may be NULL. */
int orc_matching(int64_t n, uint64_t seed, uint32_t round, int32_t* order, int32_t* trade_of);

/* Partial Durstenfeld shuffle of D[0..N) that decides which a elements go
 * to u (positions [0,a) afterwards) and which N-a go to v. */
void orc_split(int32_t* D, int64_t N, int64_t a, uint64_t seed, uint32_t round, uint32_t trade);

/* One trade (Def. "Simple Undirected Trade"). Au (du), Av (dv) ascending.
 * If arrangement != NULL it is sigma: a permutation of D (length |D|) whose
 * first |A_{u-v}| entries go to u; otherwise orc_split decides.
 * Outputs Bu (du), Bv (dv) ascending; moved_to_v receives X \ U, moved_to_u
 * receives Y \ W (each may be NULL), with their counts. Returns 0 on success,
 * negative on an invariant violation. info (may be NULL) gets
 * {|C|, a, b, uv, moved_to_v count, moved_to_u count}. */
int orc_trade_apply(const int32_t* Au, int64_t du, const int32_t* Av, int64_t dv,
                    int32_t u, int32_t v, const int32_t* arrangement,
                    uint64_t seed, uint32_t round, uint32_t trade,
                    int32_t* Bu, int32_t* Bv,
                    int32_t* moved_to_v, int32_t* moved_to_u, int64_t info[6]);

/* Number of edges between the pair of trade k and pairs of earlier trades,
 * at the start of the round (the dependency count). dep has floor(n/2). */
int orc_depcount(int64_t n, const int64_t* row_ptr, const int32_t* col,
                 const int32_t* trade_of, const int32_t* order, int32_t* dep);

/* O1: definition-literal global trade. Rows are sorted arrays; trades are
 * applied one after another; passive neighbours are relabelled in place. */
int orc_global_trade_o1(int64_t n, const int64_t* row_ptr, int32_t* col,
                        uint64_t seed, uint32_t round, orc_stats* st);

/* O2: the same global trade computed the way IM-CB does it (one stored copy
 * per edge, at the endpoint traded first; each trade pushes its edges to the
 * endpoint traded next). Must give the same bytes as O1.
 * max_trades < 0 runs the whole round; otherwise it stops after that many
 * trades and leaves col untouched (timing samples only). */
int orc_global_trade_o2(int64_t n, const int64_t* row_ptr, int32_t* col,
                        uint64_t seed, uint32_t round, orc_stats* st,
                        int64_t max_trades);

/* 0 if the CSR is simple, rows strictly ascending and symmetric. */
int orc_check_graph(int64_t n, const int64_t* row_ptr, const int32_t* col);

/* Uniform single-trade chain (Simple Undirected Curveball, Sec. 3.2): step s
 * draws the node pair u = bounded(philox64(seed; s_lo, s_hi, 0, TAG_U), n),
 * v' = bounded(philox64(seed; s_lo, s_hi, 1, TAG_U), n - 1), v = v' + (v' >= u)
 * (a uniform ordered pair of distinct nodes, so a uniform unordered pair),
 * then trades u and v with the split drawn from philox64(seed; s, CBU_ROUND,
 * j, TAG_F) (steps below 2^32). */
void orc_cbu_pair(int64_t n, uint64_t seed, uint64_t step, int32_t* u, int32_t* v);

/* Apply steps step0 .. step0 + steps - 1 to the graph in place, one trade
 * after the other, as the definition states (both trading rows rewritten,
 * passive rows relabelled). st->trades counts the steps, st->moved the
 * disjoint neighbours that changed sides, st->work the sum of deg u + deg v.
 * Returns 0 or a negative code (n < 2: no step is possible, nothing changes). */
int orc_cbu_o1(int64_t n, const int64_t* row_ptr, int32_t* col, uint64_t seed,
               uint64_t step0, uint64_t steps, orc_stats* st);

#ifdef __cplusplus
}
#endif
#endif
