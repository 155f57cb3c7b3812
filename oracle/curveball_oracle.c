/*
 * CPU oracle for the global Curveball super-step. TEST INFRASTRUCTURE:
 * only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline use it.
 * Plain, sequential, obviously-correct C. See curveball_oracle.h for the
 * graph form and the random-number convention.
 *
 * Paper passages followed:
 *  - Def. "Simple Undirected Trade" (Sec. 3.2) and its worked example
 *    figure: i and j keep their shared neighbours and the i-j edge; the
 *    disjoint neighbours D = A_{i-j} u A_{j-i} are re-split by a random
 *    arrangement sigma, i taking |A_{i-j}| of them; passive neighbours are
 *    relabelled so the adjacency stays symmetric.
 *  - Def. "Undirected Global Trade" (Sec. 3.3): floor(n/2) trades given by
 *    consecutive pairs of a permutation, applied one after the other; with
 *    odd n one node is left out (footnote in Sec. 1 and Sec. 3.3).
 *  - Def. "Relaxed global trade" (appendix on EM-GCB): the permutation is the
 *    sort order of an injective hash of the node ids.
 *  - Sec. 4 (trade procedure and its footnote): the algorithm draws sigma
 *    itself, choosing |N(u) n D| elements of D for u uniformly at random.
 *  - IM-CB (Sec. 4.2 and its algorithm in the appendix): each edge is stored
 *    once, at the endpoint traded first; a trade pushes each resulting edge
 *    to the endpoint whose trade comes next.
 *  - Simple Undirected Curveball (Sec. 3.2, the paragraph after the trade
 *    figure): a chain of single trades, each of a node pair drawn uniformly
 *    at random with a uniform split.
 */
#define _POSIX_C_SOURCE 199309L
#include <time.h>
#include "curveball_oracle.h"

#include <stdlib.h>
#include <string.h>

/* Wall-clock seconds (timing of the IM-CB form's phases only). */
static double orc_now(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).                  */
/* ------------------------------------------------------------------ */

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {                 /* Weyl key schedule between rounds */
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

uint64_t orc_philox64(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3)
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    return ((uint64_t)out[1] << 32) | out[0];
}

uint64_t orc_bounded(uint64_t x, uint64_t k)
{
    return (uint64_t)(((unsigned __int128)x * k) >> 64);
}

/* ------------------------------------------------------------------ */
/* Small sorting helpers (ascending int32, non-negative values).       */
/* ------------------------------------------------------------------ */

static void insertion_sort_i32(int32_t* a, int64_t n)
{
    for (int64_t i = 1; i < n; ++i) {
        int32_t x = a[i];
        int64_t j = i - 1;
        while (j >= 0 && a[j] > x) { a[j + 1] = a[j]; --j; }
        a[j + 1] = x;
    }
}

/* LSD radix sort, 8-bit digits, with caller temp of n entries. */
static void radix_sort_i32(int32_t* a, int32_t* tmp, int64_t n)
{
    if (n <= 48) { insertion_sort_i32(a, n); return; }
    int32_t* src = a;
    int32_t* dst = tmp;
    for (int shift = 0; shift < 32; shift += 8) {
        int64_t cnt[257];
        memset(cnt, 0, sizeof(cnt));
        for (int64_t i = 0; i < n; ++i) cnt[(((uint32_t)src[i]) >> shift & 0xFFu) + 1]++;
        if (cnt[1] == n && shift > 0) continue; /* all digits zero: nothing moves */
        for (int d = 0; d < 256; ++d) cnt[d + 1] += cnt[d];
        for (int64_t i = 0; i < n; ++i) dst[cnt[((uint32_t)src[i]) >> shift & 0xFFu]++] = src[i];
        int32_t* t = src; src = dst; dst = t;
    }
    if (src != a) memcpy(a, src, (size_t)n * sizeof(int32_t));
}

static int64_t find_sorted(const int32_t* a, int64_t n, int32_t x)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (a[mid] < x) lo = mid + 1; else hi = mid;
    }
    return (lo < n && a[lo] == x) ? lo : -1;
}

/* ------------------------------------------------------------------ */
/* Matching.                                                           */
/* ------------------------------------------------------------------ */

typedef struct { uint64_t key; int32_t id; } keyed_node;

static int cmp_keyed(const void* pa, const void* pb)
{
    const keyed_node* a = (const keyed_node*)pa;
    const keyed_node* b = (const keyed_node*)pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    return (a->id > b->id) - (a->id < b->id);
}

int orc_matching(int64_t n, uint64_t seed, uint32_t round, int32_t* order, int32_t* trade_of)
{
    if (n < 0) return -1;
    keyed_node* kn = (keyed_node*)malloc((size_t)(n > 0 ? n : 1) * sizeof(keyed_node));
    if (!kn) return -2;
    for (int64_t v = 0; v < n; ++v) {
        kn[v].key = orc_philox64(seed, (uint32_t)v, round, 0u, ORC_TAG_M);
        kn[v].id = (int32_t)v;
    }
    qsort(kn, (size_t)n, sizeof(keyed_node), cmp_keyed);
    for (int64_t p = 0; p < n; ++p) {
        if (order) order[p] = kn[p].id;
        if (trade_of) {
            int32_t t = (int32_t)(p / 2);
            if ((n & 1) && p == n - 1) t = ORC_UNMATCHED;
            trade_of[kn[p].id] = t;
        }
    }
    free(kn);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Split of the disjoint neighbours.                                   */
/* ------------------------------------------------------------------ */

void orc_split(int32_t* D, int64_t N, int64_t a, uint64_t seed, uint32_t round, uint32_t trade)
{
    int64_t b = N - a;
    if (a <= b) {
        /* front-to-back: position j receives a uniform pick of D[j..N) */
        for (int64_t j = 0; j < a; ++j) {
            uint64_t x = orc_philox64(seed, trade, round, (uint32_t)j, ORC_TAG_F);
            int64_t r = j + (int64_t)orc_bounded(x, (uint64_t)(N - j));
            int32_t t = D[j]; D[j] = D[r]; D[r] = t;
        }
    } else {
        /* back-to-front: position j receives a uniform pick of D[0..j] */
        for (int64_t j = N - 1; j >= a; --j) {
            uint64_t x = orc_philox64(seed, trade, round, (uint32_t)j, ORC_TAG_F);
            int64_t r = (int64_t)orc_bounded(x, (uint64_t)(j + 1));
            int32_t t = D[j]; D[j] = D[r]; D[r] = t;
        }
    }
}

/* ------------------------------------------------------------------ */
/* One trade.                                                          */
/* ------------------------------------------------------------------ */

int orc_trade_apply(const int32_t* Au, int64_t du, const int32_t* Av, int64_t dv,
                    int32_t u, int32_t v, const int32_t* arrangement,
                    uint64_t seed, uint32_t round, uint32_t trade,
                    int32_t* Bu, int32_t* Bv,
                    int32_t* moved_to_v, int32_t* moved_to_u, int64_t info[6])
{
    int rc = 0;
    int64_t cap = du + dv + 1;
    int32_t* C = (int32_t*)malloc((size_t)cap * sizeof(int32_t));
    int32_t* X = (int32_t*)malloc((size_t)cap * sizeof(int32_t));
    int32_t* Y = (int32_t*)malloc((size_t)cap * sizeof(int32_t));
    int32_t* D = (int32_t*)malloc((size_t)cap * sizeof(int32_t));
    int32_t* U = (int32_t*)malloc((size_t)cap * sizeof(int32_t));
    int32_t* W = (int32_t*)malloc((size_t)cap * sizeof(int32_t));
    int32_t* tmp = (int32_t*)malloc((size_t)cap * sizeof(int32_t));
    if (!C || !X || !Y || !D || !U || !W || !tmp) { rc = -100; goto out; }

    /* The i-j edge is never traded: A_{i-j} = A_i \ (A_j u {j}). */
    int uv_in_u = find_sorted(Au, du, v) >= 0;
    int vu_in_v = find_sorted(Av, dv, u) >= 0;
    if (uv_in_u != vu_in_v) { rc = -1; goto out; }           /* asymmetric input */
    if (find_sorted(Au, du, u) >= 0 || find_sorted(Av, dv, v) >= 0) { rc = -2; goto out; }

    /* C = shared, X = A_{u-v}, Y = A_{v-u}, by a merge of the sorted lists. */
    int64_t nc = 0, a = 0, b = 0, i = 0, j = 0;
    while (i < du || j < dv) {
        int32_t x = i < du ? Au[i] : INT32_MAX;
        int32_t y = j < dv ? Av[j] : INT32_MAX;
        if (i < du && x == v) { ++i; continue; }
        if (j < dv && y == u) { ++j; continue; }
        if (i < du && j < dv && x == y) { C[nc++] = x; ++i; ++j; }
        else if (j >= dv || (i < du && x < y)) { X[a++] = x; ++i; }
        else { Y[b++] = y; ++j; }
    }
    /* D = X u Y in ascending order. */
    int64_t N = 0;
    i = 0; j = 0;
    while (i < a || j < b) {
        if (j >= b || (i < a && X[i] < Y[j])) D[N++] = X[i++];
        else D[N++] = Y[j++];
    }

    if (arrangement) {
        /* sigma must be a permutation of D */
        memcpy(tmp, arrangement, (size_t)N * sizeof(int32_t));
        radix_sort_i32(tmp, U, N);
        for (int64_t k = 0; k < N; ++k) if (tmp[k] != D[k]) { rc = -3; goto out; }
        memcpy(D, arrangement, (size_t)N * sizeof(int32_t));
    } else {
        orc_split(D, N, a, seed, round, trade);
    }
    /* u takes the elements at 0-based ranks < |A_{u-v}| (ranks count the
     * elements in front, so "rank <= |A_{i-j}|" would hand u one too many). */
    memcpy(U, D, (size_t)a * sizeof(int32_t));
    memcpy(W, D + a, (size_t)b * sizeof(int32_t));
    radix_sort_i32(U, tmp, a);
    radix_sort_i32(W, tmp, b);

    /* Bu = C u U u {v if uv}; Bv = C u W u {u if uv}; both ascending. */
    int64_t nu = 0, nv = 0;
    {
        int64_t p = 0, q = 0;
        int vdone = !uv_in_u;
        while (p < nc || q < a || !vdone) {
            int32_t c = p < nc ? C[p] : INT32_MAX;
            int32_t x = q < a ? U[q] : INT32_MAX;
            int32_t w = !vdone ? v : INT32_MAX;
            if (!vdone && w < c && w < x) { Bu[nu++] = w; vdone = 1; }
            else if (p < nc && c < x) Bu[nu++] = C[p++];
            else Bu[nu++] = U[q++];
        }
    }
    {
        int64_t p = 0, q = 0;
        int udone = !vu_in_v;
        while (p < nc || q < b || !udone) {
            int32_t c = p < nc ? C[p] : INT32_MAX;
            int32_t y = q < b ? W[q] : INT32_MAX;
            int32_t w = !udone ? u : INT32_MAX;
            if (!udone && w < c && w < y) { Bv[nv++] = w; udone = 1; }
            else if (p < nc && c < y) Bv[nv++] = C[p++];
            else Bv[nv++] = W[q++];
        }
    }
    if (nu != du || nv != dv) { rc = -4; goto out; }        /* degrees preserved */

    /* Moved edges: X \ U went to v, Y \ W went to u (both sorted merges). */
    int64_t mv = 0, mu = 0;
    {
        int64_t p = 0, q = 0;
        while (p < a) {
            while (q < a && U[q] < X[p]) ++q;
            if (!(q < a && U[q] == X[p])) { if (moved_to_v) moved_to_v[mv] = X[p]; ++mv; }
            ++p;
        }
        p = 0; q = 0;
        while (p < b) {
            while (q < b && W[q] < Y[p]) ++q;
            if (!(q < b && W[q] == Y[p])) { if (moved_to_u) moved_to_u[mu] = Y[p]; ++mu; }
            ++p;
        }
    }
    if (mv != mu) { rc = -5; goto out; }                      /* a swap moves pairs */
    if (info) {
        info[0] = nc; info[1] = a; info[2] = b; info[3] = uv_in_u; info[4] = mv; info[5] = mu;
    }
out:
    free(C); free(X); free(Y); free(D); free(U); free(W); free(tmp);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Dependency count at round start.                                    */
/* ------------------------------------------------------------------ */

int orc_depcount(int64_t n, const int64_t* row_ptr, const int32_t* col,
                 const int32_t* trade_of, const int32_t* order, int32_t* dep)
{
    int64_t L = n / 2;
    for (int64_t k = 0; k < L; ++k) {
        int64_t cnt = 0;
        for (int side = 0; side < 2; ++side) {
            int32_t x = order[2 * k + side];
            for (int64_t e = row_ptr[x]; e < row_ptr[x + 1]; ++e)
                if (trade_of[col[e]] < k) ++cnt;
        }
        dep[k] = (int32_t)cnt;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* O1: definition-literal.                                             */
/* ------------------------------------------------------------------ */

/* In sorted row r (length len), replace value old by value nw, keeping the
 * row sorted. Returns 0, or -1 if old is missing or nw already present. */
static int row_replace(int32_t* r, int64_t len, int32_t old, int32_t nw)
{
    int64_t p = find_sorted(r, len, old);
    if (p < 0 || find_sorted(r, len, nw) >= 0) return -1;
    if (nw > old) {
        while (p + 1 < len && r[p + 1] < nw) { r[p] = r[p + 1]; ++p; }
    } else {
        while (p > 0 && r[p - 1] > nw) { r[p] = r[p - 1]; --p; }
    }
    r[p] = nw;
    return 0;
}

int orc_global_trade_o1(int64_t n, const int64_t* row_ptr, int32_t* col,
                        uint64_t seed, uint32_t round, orc_stats* st)
{
    int rc = 0;
    int64_t L = n / 2;
    int32_t* order = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int64_t dmax = 0;
    for (int64_t x = 0; x < n; ++x) {
        int64_t d = row_ptr[x + 1] - row_ptr[x];
        if (d > dmax) dmax = d;
    }
    int64_t cap = 2 * dmax + 2;
    int32_t* Bu = (int32_t*)malloc((size_t)cap * sizeof(int32_t));
    int32_t* Bv = (int32_t*)malloc((size_t)cap * sizeof(int32_t));
    int32_t* mtv = (int32_t*)malloc((size_t)cap * sizeof(int32_t));
    int32_t* mtu = (int32_t*)malloc((size_t)cap * sizeof(int32_t));
    if (!order || !Bu || !Bv || !mtv || !mtu) { rc = -100; goto out; }
    if ((rc = orc_matching(n, seed, round, order, NULL)) != 0) goto out;

    orc_stats s;
    memset(&s, 0, sizeof(s));
    s.trades = L;
    s.unmatched = (n & 1) ? order[n - 1] : -1;

    for (int64_t i = 0; i < L; ++i) {
        int32_t u = order[2 * i], v = order[2 * i + 1];
        int32_t* Au = col + row_ptr[u];
        int32_t* Av = col + row_ptr[v];
        int64_t du = row_ptr[u + 1] - row_ptr[u];
        int64_t dv = row_ptr[v + 1] - row_ptr[v];
        int64_t info[6];
        rc = orc_trade_apply(Au, du, Av, dv, u, v, NULL, seed, round, (uint32_t)i,
                             Bu, Bv, mtv, mtu, info);
        if (rc) goto out;
        memcpy(Au, Bu, (size_t)du * sizeof(int32_t));
        memcpy(Av, Bv, (size_t)dv * sizeof(int32_t));
        /* symmetric relabel of the passive lists */
        for (int64_t q = 0; q < info[4]; ++q) {
            int32_t x = mtv[q];
            if (row_replace(col + row_ptr[x], row_ptr[x + 1] - row_ptr[x], u, v)) { rc = -10; goto out; }
        }
        for (int64_t q = 0; q < info[5]; ++q) {
            int32_t y = mtu[q];
            if (row_replace(col + row_ptr[y], row_ptr[y + 1] - row_ptr[y], v, u)) { rc = -11; goto out; }
        }
        s.work += du + dv;
        s.common += info[0];
        s.disjoint += info[1] + info[2];
        s.moved += info[4] + info[5];
        s.uv_edges += info[3];
        if (du + dv > s.max_s) s.max_s = du + dv;
    }
    if (st) *st = s;
out:
    free(order); free(Bu); free(Bv); free(mtv); free(mtu);
    return rc;
}

/* ------------------------------------------------------------------ */
/* O2: IM-CB-style.                                                    */
/* ------------------------------------------------------------------ */

int orc_global_trade_o2(int64_t n, const int64_t* row_ptr, int32_t* col,
                        uint64_t seed, uint32_t round, orc_stats* st,
                        int64_t max_trades)
{
    const double t_begin = orc_now();
    int rc = 0;
    int64_t L = n / 2;
    int64_t nnz = row_ptr[n];
    const int64_t INF = INT64_MAX;
    int32_t* order = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int32_t* trade_of = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int64_t* tau = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t* fill = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int32_t* recv = (int32_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
    int32_t* dep = (int32_t*)malloc((size_t)(L > 0 ? L : 1) * sizeof(int32_t));
    int32_t* AG = (int32_t*)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
    int64_t dmax = 0;
    for (int64_t x = 0; x < n; ++x) {
        int64_t d = row_ptr[x + 1] - row_ptr[x];
        if (d > dmax) dmax = d;
    }
    int64_t cap = 2 * dmax + 2;
    int32_t* Nu = (int32_t*)malloc((size_t)cap * sizeof(int32_t));
    int32_t* Nv = (int32_t*)malloc((size_t)cap * sizeof(int32_t));
    int32_t* Bu = (int32_t*)malloc((size_t)cap * sizeof(int32_t));
    int32_t* Bv = (int32_t*)malloc((size_t)cap * sizeof(int32_t));
    int32_t* tmp = (int32_t*)malloc((size_t)cap * sizeof(int32_t));
    if (!order || !trade_of || !tau || !fill || !recv || !dep || !AG || !Nu || !Nv ||
        !Bu || !Bv || !tmp) { rc = -100; goto out; }

    if ((rc = orc_matching(n, seed, round, order, trade_of)) != 0) goto out;
    if ((rc = orc_depcount(n, row_ptr, col, trade_of, order, dep)) != 0) goto out;

    orc_stats s;
    memset(&s, 0, sizeof(s));
    s.trades = L;
    s.unmatched = (n & 1) ? order[n - 1] : -1;

    /* tau[x]: index of the next trade of x in this round (INF if none). */
    for (int64_t x = 0; x < n; ++x) {
        tau[x] = trade_of[x] == ORC_UNMATCHED ? INF : trade_of[x];
        fill[x] = row_ptr[x];
    }
    /* Store every edge once, at the endpoint traded first. */
    for (int64_t a = 0; a < n; ++a) {
        for (int64_t e = row_ptr[a]; e < row_ptr[a + 1]; ++e) {
            int32_t b = col[e];
            if (b < a) continue;                  /* each undirected edge once */
            if (tau[a] <= tau[b]) AG[fill[a]++] = b;
            else AG[fill[b]++] = (int32_t)a;
        }
    }

    int64_t limit = (max_trades >= 0 && max_trades < L) ? max_trades : L;
    const double t_trades = orc_now();
    s.setup_seconds = t_trades - t_begin;
    for (int64_t i = 0; i < limit; ++i) {
        int32_t u = order[2 * i], v = order[2 * i + 1];
        int64_t du = row_ptr[u + 1] - row_ptr[u];
        int64_t dv = row_ptr[v + 1] - row_ptr[v];
        if (recv[u] + recv[v] != dep[i]) s.dep_mismatch++;  /* count invariance */
        /* Gather the stored edges of u and v, then reset their buffers. */
        int64_t gu = fill[u] - row_ptr[u], gv = fill[v] - row_ptr[v];
        int64_t nu = 0, nv = 0;
        int uv_at_v = 0, uv_at_u = 0;
        for (int64_t q = 0; q < gu; ++q) {
            int32_t x = AG[row_ptr[u] + q];
            if (x == v) uv_at_u = 1;
            Nu[nu++] = x;
        }
        for (int64_t q = 0; q < gv; ++q) {
            int32_t x = AG[row_ptr[v] + q];
            if (x == u) uv_at_v = 1;
            Nv[nv++] = x;
        }
        if (uv_at_v) Nu[nu++] = v;   /* the u-v edge is stored at one endpoint */
        if (uv_at_u) Nv[nv++] = u;
        if (nu != du || nv != dv) { rc = -20; goto out; }
        fill[u] = row_ptr[u];
        fill[v] = row_ptr[v];
        tau[u] = INF;
        tau[v] = INF;
        radix_sort_i32(Nu, tmp, nu);
        radix_sort_i32(Nv, tmp, nv);

        int64_t info[6];
        rc = orc_trade_apply(Nu, du, Nv, dv, u, v, NULL, seed, round, (uint32_t)i,
                             Bu, Bv, NULL, NULL, info);
        if (rc) goto out;

        /* Push every resulting edge to the endpoint whose trade is next:
         * tau[u] = tau[v] = INF now, so each edge goes to its other end. */
        for (int side = 0; side < 2; ++side) {
            int32_t a = side ? v : u;
            const int32_t* B = side ? Bv : Bu;
            int64_t d = side ? dv : du;
            for (int64_t q = 0; q < d; ++q) {
                int32_t b = B[q];
                if (side == 1 && b == u) continue;  /* u-v edge pushed once */
                if (tau[a] < tau[b]) AG[fill[a]++] = b;
                else {
                    AG[fill[b]++] = a;
                    if (tau[b] != INF) recv[b]++;
                }
            }
        }
        s.work += du + dv;
        s.common += info[0];
        s.disjoint += info[1] + info[2];
        s.moved += info[4] + info[5];
        s.uv_edges += info[3];
        if (du + dv > s.max_s) s.max_s = du + dv;
    }
    s.trade_seconds = orc_now() - t_trades;
    const double t_rebuild = orc_now();
    if (limit == L) {
        /* Rebuild the symmetric CSR from the single stored copies: node y's
         * stored edges are AG[row_ptr[y] .. fill[y]). */
        int64_t* cur = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
        if (!cur) { rc = -100; goto out; }
        for (int64_t x = 0; x < n; ++x) cur[x] = row_ptr[x];
        for (int64_t y = 0; y < n; ++y) {
            for (int64_t q = row_ptr[y]; q < fill[y]; ++q) {
                int32_t x = AG[q];
                if (cur[x] >= row_ptr[x + 1] || cur[y] >= row_ptr[y + 1]) { free(cur); rc = -21; goto out; }
                col[cur[x]++] = (int32_t)y;
                col[cur[y]++] = x;
            }
        }
        for (int64_t x = 0; x < n; ++x) {
            if (cur[x] != row_ptr[x + 1]) { free(cur); rc = -22; goto out; }
            int64_t d = row_ptr[x + 1] - row_ptr[x];
            if (d > cap) { free(cur); rc = -23; goto out; }
            radix_sort_i32(col + row_ptr[x], tmp, d);
        }
        free(cur);
    }
    s.rebuild_seconds = orc_now() - t_rebuild;
    if (st) *st = s;
out:
    free(order); free(trade_of); free(tau); free(fill); free(recv); free(dep); free(AG);
    free(Nu); free(Nv); free(Bu); free(Bv); free(tmp);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Graph check.                                                        */
/* ------------------------------------------------------------------ */

int orc_check_graph(int64_t n, const int64_t* row_ptr, const int32_t* col)
{
    if (n < 0 || row_ptr[0] != 0) return -1;
    for (int64_t x = 0; x < n; ++x) {
        if (row_ptr[x + 1] < row_ptr[x]) return -2;
        for (int64_t e = row_ptr[x]; e < row_ptr[x + 1]; ++e) {
            int32_t y = col[e];
            if (y < 0 || y >= n) return -3;
            if (y == x) return -4;
            if (e > row_ptr[x] && col[e - 1] >= y) return -5;
            if (find_sorted(col + row_ptr[y], row_ptr[y + 1] - row_ptr[y], (int32_t)x) < 0) return -6;
        }
    }
    if (row_ptr[n] % 2) return -7;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Uniform single trades (Simple Undirected Curveball).                */
/* ------------------------------------------------------------------ */

void orc_cbu_pair(int64_t n, uint64_t seed, uint64_t step, int32_t* u, int32_t* v)
{
    uint32_t lo = (uint32_t)step, hi = (uint32_t)(step >> 32);
    int64_t a = (int64_t)orc_bounded(orc_philox64(seed, lo, hi, 0u, ORC_TAG_U), (uint64_t)n);
    int64_t b = (int64_t)orc_bounded(orc_philox64(seed, lo, hi, 1u, ORC_TAG_U), (uint64_t)(n - 1));
    if (b >= a) ++b;
    *u = (int32_t)a;
    *v = (int32_t)b;
}

int orc_cbu_o1(int64_t n, const int64_t* row_ptr, int32_t* col, uint64_t seed,
               uint64_t step0, uint64_t steps, orc_stats* st)
{
    orc_stats s;
    memset(&s, 0, sizeof(s));
    s.unmatched = -1;
    if (n < 2 || steps == 0) { if (st) *st = s; return 0; }
    if (step0 + steps > ((uint64_t)1 << 32)) return -30;
    int rc = 0;
    int64_t dmax = 0;
    for (int64_t x = 0; x < n; ++x) {
        int64_t d = row_ptr[x + 1] - row_ptr[x];
        if (d > dmax) dmax = d;
    }
    int64_t cap = 2 * dmax + 2;
    int32_t* Bu = (int32_t*)malloc((size_t)cap * sizeof(int32_t));
    int32_t* Bv = (int32_t*)malloc((size_t)cap * sizeof(int32_t));
    int32_t* mtv = (int32_t*)malloc((size_t)cap * sizeof(int32_t));
    int32_t* mtu = (int32_t*)malloc((size_t)cap * sizeof(int32_t));
    if (!Bu || !Bv || !mtv || !mtu) { rc = -100; goto out; }
    for (uint64_t t = 0; t < steps; ++t) {
        uint64_t step = step0 + t;
        int32_t u, v;
        orc_cbu_pair(n, seed, step, &u, &v);
        int32_t* Au = col + row_ptr[u];
        int32_t* Av = col + row_ptr[v];
        int64_t du = row_ptr[u + 1] - row_ptr[u];
        int64_t dv = row_ptr[v + 1] - row_ptr[v];
        int64_t info[6];
        rc = orc_trade_apply(Au, du, Av, dv, u, v, NULL, seed, ORC_CBU_ROUND, (uint32_t)step,
                             Bu, Bv, mtv, mtu, info);
        if (rc) goto out;
        memcpy(Au, Bu, (size_t)du * sizeof(int32_t));
        memcpy(Av, Bv, (size_t)dv * sizeof(int32_t));
        /* the passive rows follow the moved edges */
        for (int64_t q = 0; q < info[4]; ++q)
            if (row_replace(col + row_ptr[mtv[q]], row_ptr[mtv[q] + 1] - row_ptr[mtv[q]], u, v)) { rc = -10; goto out; }
        for (int64_t q = 0; q < info[5]; ++q)
            if (row_replace(col + row_ptr[mtu[q]], row_ptr[mtu[q] + 1] - row_ptr[mtu[q]], v, u)) { rc = -11; goto out; }
        s.trades += 1;
        s.work += du + dv;
        s.common += info[0];
        s.disjoint += info[1] + info[2];
        s.moved += info[4] + info[5];
        s.uv_edges += info[3];
        if (du + dv > s.max_s) s.max_s = du + dv;
    }
    if (st) *st = s;
out:
    free(Bu); free(Bv); free(mtv); free(mtu);
    return rc;
}
