/*
 * Seeded synthetic input generator: i.i.d. degrees from a discrete power law
 * Pld([a,b), gamma) (P[X=k] proportional to k^-gamma for a <= k < b), then
 * an erased configuration model (uniform random pairing of the degree
 * stubs, self-loops dropped, multi-edges collapsed), written as a simple
 * symmetric CSR with ascending rows.
 *
 * This module holds none of the Curveball arithmetic. Its random numbers are
 * SplitMix64 outputs (Steele, Lea, Flood, OOPSLA 2014) indexed by (seed,
 * stream, counter), so the graph is the same for any thread count.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

static inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Output `i` of the SplitMix64 sequence started at a (seed, stream) state. */
static inline uint64_t gg_rand(uint64_t seed, uint64_t stream, uint64_t i)
{
    uint64_t state = mix64(seed * 0x9E3779B97F4A7C15ull + stream * 0xD1B54A32D192ED03ull + 0x632BE59BD9B4E019ull);
    return mix64(state + (i + 1) * 0x9E3779B97F4A7C15ull);
}

static inline double gg_u01(uint64_t h) { return (double)(h >> 11) * 0x1.0p-53; }

static inline uint64_t gg_below(uint64_t h, uint64_t k)
{
    return (uint64_t)(((unsigned __int128)h * k) >> 64);
}

/* ------------------------------------------------------------------ */
/* A small fork/join helper.                                           */
/* ------------------------------------------------------------------ */

typedef void (*gg_body)(void* ctx, int tid, int nthreads);
typedef struct { gg_body fn; void* ctx; int tid; int nthreads; } gg_job;

static void* gg_run(void* p)
{
    gg_job* j = (gg_job*)p;
    j->fn(j->ctx, j->tid, j->nthreads);
    return NULL;
}

static void gg_parallel(int nthreads, gg_body fn, void* ctx)
{
    pthread_t th[256];
    gg_job jobs[256];
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    for (int t = 0; t < nthreads; ++t) {
        jobs[t].fn = fn; jobs[t].ctx = ctx; jobs[t].tid = t; jobs[t].nthreads = nthreads;
    }
    for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, gg_run, &jobs[t]);
    gg_run(&jobs[0]);
    for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
}

static inline void gg_range(int64_t n, int tid, int nt, int64_t* lo, int64_t* hi)
{
    *lo = n * tid / nt;
    *hi = n * (tid + 1) / nt;
}

/* ------------------------------------------------------------------ */
/* Degrees.                                                            */
/* ------------------------------------------------------------------ */

typedef struct {
    int64_t n; int64_t a; int64_t b; uint64_t seed;
    const double* cdf; int32_t* deg; int64_t* partial;
} deg_ctx;

static int64_t pld_draw(const double* cdf, int64_t a, int64_t b, uint64_t h)
{
    double x = gg_u01(h) * cdf[b - a - 1];
    int64_t lo = 0, hi = b - a - 1;          /* first index with cdf > x */
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (cdf[mid] > x) hi = mid; else lo = mid + 1;
    }
    return a + lo;
}

static void deg_body(void* p, int tid, int nt)
{
    deg_ctx* c = (deg_ctx*)p;
    int64_t lo, hi, s = 0;
    gg_range(c->n, tid, nt, &lo, &hi);
    for (int64_t v = lo; v < hi; ++v) {
        c->deg[v] = (int32_t)pld_draw(c->cdf, c->a, c->b, gg_rand(c->seed, 1, (uint64_t)v));
        s += c->deg[v];
    }
    c->partial[tid] = s;
}

/* Fill deg[0..n) from Pld([a,b), gamma); the sum is made even by redrawing
 * the last node's degree. Returns the stub total, or -1 on bad arguments. */
int64_t gg_degrees(int64_t n, int64_t a, int64_t b, double gamma, uint64_t seed,
                   int nthreads, int32_t* deg)
{
    if (n < 0 || a < 0 || b <= a || b - a > (1ll << 31)) return -1;
    if (n == 0) return 0;
    double* cdf = (double*)malloc((size_t)(b - a) * sizeof(double));
    int64_t partial[256];
    if (!cdf) return -2;
    double acc = 0.0;
    for (int64_t k = a; k < b; ++k) {
        acc += (k == 0) ? (gamma == 0.0 ? 1.0 : 0.0) : pow((double)k, -gamma);
        cdf[k - a] = acc;
    }
    if (nthreads > 256) nthreads = 256;
    deg_ctx c = {n, a, b, seed, cdf, deg, partial};
    gg_parallel(nthreads, deg_body, &c);
    int64_t total = 0;
    for (int t = 0; t < (nthreads < 1 ? 1 : nthreads); ++t) total += partial[t];
    for (uint64_t attempt = 0; (total & 1) && attempt < 1000; ++attempt) {
        total -= deg[n - 1];
        deg[n - 1] = (int32_t)pld_draw(cdf, a, b, gg_rand(seed, 2, attempt));
        total += deg[n - 1];
    }
    if ((total & 1) && deg[n - 1] > 0) { deg[n - 1] -= 1; total -= 1; }
    free(cdf);
    return total;
}

/* ------------------------------------------------------------------ */
/* Configuration model.                                                */
/* ------------------------------------------------------------------ */

typedef struct {
    int64_t n, S, NB;
    uint64_t seed;
    const int32_t* deg;
    const int64_t* off;      /* stub offsets per node, n+1 */
    int32_t* shuf;           /* S: stubs after the shuffle */
    int64_t* bcount;         /* nthreads x NB */
    int64_t* bstart;         /* NB+1 */
    int64_t* ecount;         /* n: entries per node before erasure (atomic) */
    int64_t* eoff;           /* n+1 */
    int64_t* ecur;           /* n (atomic cursors) */
    int32_t* ecol;           /* entries before erasure */
    int64_t* newdeg;         /* n: after erasure */
    const int64_t* row_ptr;  /* n+1 final */
    int32_t* col;            /* final */
    int64_t next_row;        /* dynamic scheduling cursor */
    int64_t dmax;
} cm_ctx;

static inline int64_t stub_bucket(const cm_ctx* c, int64_t p)
{
    return (int64_t)gg_below(gg_rand(c->seed, 3, (uint64_t)p), (uint64_t)c->NB);
}

static inline int32_t stub_node(const cm_ctx* c, int64_t p)
{
    /* node owning stub p: last v with off[v] <= p */
    int64_t lo = 0, hi = c->n - 1;
    while (lo < hi) {
        int64_t mid = (lo + hi + 1) / 2;
        if (c->off[mid] <= p) lo = mid; else hi = mid - 1;
    }
    return (int32_t)lo;
}

static void cm_count(void* p, int tid, int nt)
{
    cm_ctx* c = (cm_ctx*)p;
    int64_t lo, hi;
    gg_range(c->S, tid, nt, &lo, &hi);
    int64_t* cnt = c->bcount + (int64_t)tid * c->NB;
    memset(cnt, 0, (size_t)c->NB * sizeof(int64_t));
    for (int64_t q = lo; q < hi; ++q) cnt[stub_bucket(c, q)]++;
}

static void cm_scatter(void* p, int tid, int nt)
{
    cm_ctx* c = (cm_ctx*)p;
    int64_t lo, hi;
    gg_range(c->S, tid, nt, &lo, &hi);
    int64_t* cur = c->bcount + (int64_t)tid * c->NB;   /* turned into cursors */
    int32_t v = lo < hi ? stub_node(c, lo) : 0;
    for (int64_t q = lo; q < hi; ++q) {
        while (c->off[v + 1] <= q) ++v;
        c->shuf[cur[stub_bucket(c, q)]++] = v;
    }
}

static void cm_shuffle(void* p, int tid, int nt)
{
    cm_ctx* c = (cm_ctx*)p;
    int64_t lo, hi;
    gg_range(c->NB, tid, nt, &lo, &hi);
    for (int64_t bk = lo; bk < hi; ++bk) {
        int64_t s0 = c->bstart[bk], len = c->bstart[bk + 1] - s0;
        int32_t* a = c->shuf + s0;
        for (int64_t j = len - 1; j > 0; --j) {   /* Durstenfeld within the bucket */
            int64_t r = (int64_t)gg_below(gg_rand(c->seed, 4, ((uint64_t)bk << 32) ^ (uint64_t)j), (uint64_t)(j + 1));
            int32_t t = a[j]; a[j] = a[r]; a[r] = t;
        }
    }
}

static void cm_edge_count(void* p, int tid, int nt)
{
    cm_ctx* c = (cm_ctx*)p;
    int64_t lo, hi;
    gg_range(c->S / 2, tid, nt, &lo, &hi);
    for (int64_t i = lo; i < hi; ++i) {
        int32_t x = c->shuf[2 * i], y = c->shuf[2 * i + 1];
        if (x == y) continue;
        __atomic_fetch_add(&c->ecount[x], 1, __ATOMIC_RELAXED);
        __atomic_fetch_add(&c->ecount[y], 1, __ATOMIC_RELAXED);
    }
}

static void cm_edge_fill(void* p, int tid, int nt)
{
    cm_ctx* c = (cm_ctx*)p;
    int64_t lo, hi;
    gg_range(c->S / 2, tid, nt, &lo, &hi);
    for (int64_t i = lo; i < hi; ++i) {
        int32_t x = c->shuf[2 * i], y = c->shuf[2 * i + 1];
        if (x == y) continue;
        c->ecol[__atomic_fetch_add(&c->ecur[x], 1, __ATOMIC_RELAXED)] = y;
        c->ecol[__atomic_fetch_add(&c->ecur[y], 1, __ATOMIC_RELAXED)] = x;
    }
}

static void sort_row(int32_t* a, int64_t n, int32_t* tmp)
{
    if (n <= 32) {
        for (int64_t i = 1; i < n; ++i) {
            int32_t x = a[i]; int64_t j = i - 1;
            while (j >= 0 && a[j] > x) { a[j + 1] = a[j]; --j; }
            a[j + 1] = x;
        }
        return;
    }
    int32_t* src = a; int32_t* dst = tmp;
    for (int shift = 0; shift < 32; shift += 8) {
        int64_t cnt[257];
        memset(cnt, 0, sizeof(cnt));
        for (int64_t i = 0; i < n; ++i) cnt[(((uint32_t)src[i]) >> shift & 0xFFu) + 1]++;
        if (cnt[1] == n && shift > 0) continue;
        for (int d = 0; d < 256; ++d) cnt[d + 1] += cnt[d];
        for (int64_t i = 0; i < n; ++i) dst[cnt[((uint32_t)src[i]) >> shift & 0xFFu]++] = src[i];
        int32_t* t = src; src = dst; dst = t;
    }
    if (src != a) memcpy(a, src, (size_t)n * sizeof(int32_t));
}

static void cm_sort_unique(void* p, int tid, int nt)
{
    (void)tid; (void)nt;
    cm_ctx* c = (cm_ctx*)p;
    int32_t* tmp = (int32_t*)malloc((size_t)(c->dmax > 0 ? c->dmax : 1) * sizeof(int32_t));
    for (;;) {
        int64_t r0 = __atomic_fetch_add(&c->next_row, 4096, __ATOMIC_RELAXED);
        if (r0 >= c->n) break;
        int64_t r1 = r0 + 4096 < c->n ? r0 + 4096 : c->n;
        for (int64_t x = r0; x < r1; ++x) {
            int32_t* a = c->ecol + c->eoff[x];
            int64_t len = c->eoff[x + 1] - c->eoff[x];
            sort_row(a, len, tmp);
            int64_t w = 0;
            for (int64_t i = 0; i < len; ++i)
                if (w == 0 || a[w - 1] != a[i]) a[w++] = a[i];
            c->newdeg[x] = w;
        }
    }
    free(tmp);
}

static void cm_copy(void* p, int tid, int nt)
{
    cm_ctx* c = (cm_ctx*)p;
    int64_t lo, hi;
    gg_range(c->n, tid, nt, &lo, &hi);
    for (int64_t x = lo; x < hi; ++x)
        memcpy(c->col + c->row_ptr[x], c->ecol + c->eoff[x],
               (size_t)(c->row_ptr[x + 1] - c->row_ptr[x]) * sizeof(int32_t));
}

/* Build the erased configuration model for the given degrees. row_ptr has
 * n+1 entries; col has room for col_cap entries (the stub total suffices).
 * Returns the number of CSR entries (2m), or a negative error. */
int64_t gg_configuration_model(int64_t n, const int32_t* deg, uint64_t seed, int nthreads,
                               int64_t* row_ptr, int32_t* col, int64_t col_cap)
{
    if (n < 0) return -1;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    row_ptr[0] = 0;
    if (n == 0) return 0;
    int64_t* off = (int64_t*)malloc((size_t)(n + 1) * sizeof(int64_t));
    if (!off) return -2;
    off[0] = 0;
    for (int64_t v = 0; v < n; ++v) off[v + 1] = off[v] + deg[v];
    int64_t S = off[n];
    if (S & 1) { free(off); return -3; }
    if (S > col_cap) { free(off); return -4; }

    cm_ctx c;
    memset(&c, 0, sizeof(c));
    c.n = n; c.S = S; c.seed = seed; c.deg = deg; c.off = off;
    c.NB = S >> 12; if (c.NB < 1) c.NB = 1;
    c.shuf = (int32_t*)malloc((size_t)(S > 0 ? S : 1) * sizeof(int32_t));
    c.bcount = (int64_t*)malloc((size_t)nthreads * (size_t)c.NB * sizeof(int64_t));
    c.bstart = (int64_t*)malloc((size_t)(c.NB + 1) * sizeof(int64_t));
    if (!c.shuf || !c.bcount || !c.bstart) { free(off); free(c.shuf); free(c.bcount); free(c.bstart); return -2; }

    /* 1. uniform random permutation of the stubs: iid uniform bucket per
     *    stub, stable scatter, Durstenfeld shuffle inside each bucket. */
    gg_parallel(nthreads, cm_count, &c);
    int64_t acc = 0;
    for (int64_t bk = 0; bk < c.NB; ++bk) {
        c.bstart[bk] = acc;
        for (int t = 0; t < nthreads; ++t) {
            int64_t k = c.bcount[(int64_t)t * c.NB + bk];
            c.bcount[(int64_t)t * c.NB + bk] = acc;
            acc += k;
        }
    }
    c.bstart[c.NB] = acc;
    gg_parallel(nthreads, cm_scatter, &c);
    gg_parallel(nthreads, cm_shuffle, &c);
    free(c.bcount); c.bcount = NULL;

    /* 2. consecutive stubs form edges; loops dropped; symmetric entries. */
    c.ecount = (int64_t*)calloc((size_t)n, sizeof(int64_t));
    c.eoff = (int64_t*)malloc((size_t)(n + 1) * sizeof(int64_t));
    c.ecur = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    c.newdeg = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    if (!c.ecount || !c.eoff || !c.ecur || !c.newdeg) return -2;
    gg_parallel(nthreads, cm_edge_count, &c);
    c.eoff[0] = 0;
    c.dmax = 0;
    for (int64_t x = 0; x < n; ++x) {
        c.eoff[x + 1] = c.eoff[x] + c.ecount[x];
        c.ecur[x] = c.eoff[x];
        if (c.ecount[x] > c.dmax) c.dmax = c.ecount[x];
    }
    c.ecol = (int32_t*)malloc((size_t)(c.eoff[n] > 0 ? c.eoff[n] : 1) * sizeof(int32_t));
    if (!c.ecol) return -2;
    gg_parallel(nthreads, cm_edge_fill, &c);
    free(c.shuf); c.shuf = NULL;

    /* 3. collapse multi-edges: sort each row, keep distinct neighbours. */
    c.next_row = 0;
    gg_parallel(nthreads, cm_sort_unique, &c);
    row_ptr[0] = 0;
    for (int64_t x = 0; x < n; ++x) row_ptr[x + 1] = row_ptr[x] + c.newdeg[x];
    c.row_ptr = row_ptr;
    c.col = col;
    gg_parallel(nthreads, cm_copy, &c);
    int64_t nnz = row_ptr[n];
    free(off); free(c.bstart); free(c.ecount); free(c.eoff); free(c.ecur); free(c.newdeg); free(c.ecol);
    return nnz;
}
