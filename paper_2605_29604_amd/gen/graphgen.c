/*
 * Seeded synthetic graph generators (host C).
 *
 * This module produces the *inputs* of the MIS solver: simple undirected graphs
 * in CSR form (row_ptr int64[n+1], col_idx int32[2m], every adjacency list sorted
 * ascending, symmetric, no self-loops, no duplicate edges).  It holds none of the
 * solver's arithmetic (no priorities, no MIS rule), so both the CPU oracle and the
 * GPU library may be fed from it.
 *
 * Workload families (the shapes of the paper's evaluation graphs, Table 1 of the
 * evaluation section: road/mesh graphs, power-law web/social graphs and a
 * Graph500 Kronecker graph):
 *   - Erdos-Renyi G(n, m): m distinct unordered pairs u != v drawn uniformly.
 *   - R-MAT(a, b, c, d) with integer quadrant thresholds on 32-bit draws, drawn
 *     until m distinct non-loop undirected edges exist; optional random vertex
 *     relabelling (Fisher-Yates).  Non power-of-two n: scale = ceil(log2 n),
 *     endpoints >= n rejected.
 *   - 3D 7-point grid sx*sy*sz, v = x + sx*y + sx*sy*z, plus n_long uniformly
 *     random long-range pairs that are neither loops nor already edges.
 *
 * Random numbers: SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014): output i (i >= 1) of the stream seeded with s
 * is F(s + i * 0x9E3779B97F4A7C15), F the published 64-bit finaliser.  Bounded
 * integers use Lemire's multiply-shift on a 32-bit half.  Each family derives
 * its own stream seed from the user seed and a purpose tag.
 *
 * Candidate edge j (j = 0, 1, ...) of a family is a pure function of (seed, j):
 * it uses outputs j*L+1 .. j*L+L of the family stream (L = 1 for Erdos-Renyi and
 * long-range pairs, ceil(scale/2) for R-MAT: each output gives two 32-bit level
 * draws, high half first).  Candidates are generated in parallel and then
 * de-duplicated in draw order inside hash partitions that are independent of
 * each other; the first m distinct valid candidates in draw order are the edges.
 * The output therefore does not depend on the number of host threads.
 *
 * Return values: >= 0 = number of undirected edges written; < 0 = error
 * (-1 bad argument, -2 out of memory, -3 impossible request).
 */
#define _GNU_SOURCE
#include <pthread.h>
#include <sched.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GG_GAMMA 0x9E3779B97F4A7C15ull
#define GG_NPART 64

static uint64_t gg_fin(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
/* output i (1-based) of the SplitMix64 stream seeded with s */
static uint64_t gg_at(uint64_t s, uint64_t i) { return gg_fin(s + i * GG_GAMMA); }

/* uniform integer in [0, bound) from a 32-bit draw, bound <= 2^32 */
static uint32_t gg_bounded32(uint32_t x, uint64_t bound) {
    return (uint32_t)(((uint64_t)x * bound) >> 32);
}

/* stream seed for a purpose tag */
static uint64_t gg_derive(uint64_t seed, uint64_t tag) {
    return gg_at(seed ^ (tag * 0xD1B54A32D192ED03ull), 2);
}

/* ---------------------------------------------------------------- threads */
typedef void (*gg_body)(void* ctx, int64_t begin, int64_t end);
typedef struct { gg_body fn; void* ctx; int64_t total, chunk; int64_t next; pthread_mutex_t mu; } gg_pool;

static void* gg_worker(void* arg) {
    gg_pool* p = (gg_pool*)arg;
    for (;;) {
        pthread_mutex_lock(&p->mu);
        int64_t b = p->next;
        p->next += p->chunk;
        pthread_mutex_unlock(&p->mu);
        if (b >= p->total) break;
        int64_t e = b + p->chunk < p->total ? b + p->chunk : p->total;
        p->fn(p->ctx, b, e);
    }
    return NULL;
}

/* worker threads of a batch generate each of their graphs with one thread */
static __thread int gg_single_thread = 0;

static int gg_threads(void) {
    if (gg_single_thread) return 1;
    const char* env = getenv("GG_THREADS");
    if (env && atoi(env) > 0) return atoi(env);
    cpu_set_t set;
    int n = 1;
    if (sched_getaffinity(0, sizeof(set), &set) == 0) n = CPU_COUNT(&set);
    if (n > 16) n = 16;
    return n < 1 ? 1 : n;
}

/* run fn over [0, total) in chunks; chunk boundaries never change results */
static void gg_parallel(gg_body fn, void* ctx, int64_t total, int64_t chunk) {
    if (total <= 0) return;
    int nt = gg_threads();
    if (chunk < 1) chunk = 1;
    if (nt <= 1 || total <= chunk) { fn(ctx, 0, total); return; }
    gg_pool p = { fn, ctx, total, chunk, 0, PTHREAD_MUTEX_INITIALIZER };
    pthread_t th[64];
    if (nt > 64) nt = 64;
    int started = 0;
    for (int i = 0; i < nt; ++i)
        if (pthread_create(&th[i], NULL, gg_worker, &p) == 0) ++started;
    if (started == 0) gg_worker(&p);
    for (int i = 0; i < started; ++i) pthread_join(th[i], NULL);
}

/* ------------------------------------------- partitioned set of edge keys */
typedef struct { uint64_t* slot; uint64_t mask; int64_t count; } gg_set;

static uint64_t gg_hash(uint64_t k) {
    k ^= k >> 33; k *= 0xFF51AFD7ED558CCDull; k ^= k >> 33; k *= 0xC4CEB9FE1A85EC53ull; k ^= k >> 33;
    return k;
}
static int gg_set_init(gg_set* s, int64_t expect) {
    uint64_t cap = 1024;
    while (cap < (uint64_t)expect * 2 + 16) cap <<= 1;
    s->slot = (uint64_t*)malloc(cap * sizeof(uint64_t));
    if (!s->slot) return -2;
    memset(s->slot, 0xff, cap * sizeof(uint64_t));   /* empty = all ones */
    s->mask = cap - 1;
    s->count = 0;
    return 0;
}
static int gg_set_grow(gg_set* s) {
    gg_set t;
    if (gg_set_init(&t, (int64_t)(s->mask + 1))) return -2;
    for (uint64_t i = 0; i <= s->mask; ++i) {
        uint64_t k = s->slot[i];
        if (k == ~0ull) continue;
        uint64_t j = (gg_hash(k) >> 6) & t.mask;
        while (t.slot[j] != ~0ull) j = (j + 1) & t.mask;
        t.slot[j] = k; t.count++;
    }
    free(s->slot);
    *s = t;
    return 0;
}
/* 1 inserted, 0 present, -2 oom */
static int gg_set_insert(gg_set* s, uint64_t key) {
    if ((uint64_t)(s->count + 1) * 2 > s->mask + 1 && gg_set_grow(s)) return -2;
    uint64_t i = (gg_hash(key) >> 6) & s->mask;
    for (;;) {
        uint64_t cur = s->slot[i];
        if (cur == ~0ull) { s->slot[i] = key; s->count++; return 1; }
        if (cur == key) return 0;
        i = (i + 1) & s->mask;
    }
}
static int gg_part(uint64_t key) { return (int)(gg_hash(key) & (GG_NPART - 1)); }

static uint64_t gg_ekey(uint32_t u, uint32_t v) {
    return u < v ? ((uint64_t)u << 32) | v : ((uint64_t)v << 32) | u;
}
#define GG_REJECT (~0ull)

/* ----------------------------------------------- candidate edge families */
typedef struct {
    int kind;            /* 1 = uniform pairs, 2 = R-MAT */
    uint64_t stream;     /* family stream seed */
    int64_t n;
    int scale, draws;    /* R-MAT: levels and 64-bit outputs per candidate */
    uint64_t t1, t2, t3; /* R-MAT cumulative thresholds */
    /* grid exclusion for long-range pairs (0 = none) */
    int64_t gx, gy, gz;
} gg_family;

static uint64_t gg_candidate(const gg_family* f, uint64_t j) {
    uint32_t u = 0, v = 0;
    if (f->kind == 1) {
        uint64_t x = gg_at(f->stream, j + 1);
        u = gg_bounded32((uint32_t)(x >> 32), (uint64_t)f->n);
        v = gg_bounded32((uint32_t)x, (uint64_t)f->n);
    } else {
        uint64_t base = j * (uint64_t)f->draws;
        int lev = f->scale - 1;
        for (int d = 0; d < f->draws && lev >= 0; ++d) {
            uint64_t x = gg_at(f->stream, base + d + 1);
            for (int h = 0; h < 2 && lev >= 0; ++h, --lev) {
                uint32_t r = h == 0 ? (uint32_t)(x >> 32) : (uint32_t)x;
                /* r < t1: (0,0); < t2: (0,1); < t3: (1,0); else (1,1) */
                uint32_t ub = r >= f->t2;
                uint32_t vb = (uint32_t)((r >= f->t1) & (r < f->t2)) | (uint32_t)(r >= f->t3);
                u |= ub << lev; v |= vb << lev;
            }
        }
        if (u >= (uint64_t)f->n || v >= (uint64_t)f->n) return GG_REJECT;
    }
    if (u == v) return GG_REJECT;
    uint32_t lo = u < v ? u : v, hi = u < v ? v : u;
    if (f->gx > 0) {   /* reject grid edges */
        uint64_t d = hi - lo, sx = (uint64_t)f->gx, sy = (uint64_t)f->gy, sz = (uint64_t)f->gz;
        if (d == 1 && (lo % sx) + 1 < sx) return GG_REJECT;
        if (d == sx && ((lo / sx) % sy) + 1 < sy) return GG_REJECT;
        if (d == sx * sy && (lo / (sx * sy)) + 1 < sz) return GG_REJECT;
    }
    return gg_ekey(u, v);
}

typedef struct {
    const gg_family* f;
    uint64_t first;      /* candidate index of slot 0 */
    uint64_t* key;       /* [count] candidate keys */
    uint8_t* pid;        /* [count] hash partition of the key, GG_NPART = rejected */
    uint8_t* fresh;      /* [count] 1 = first occurrence */
    uint32_t* order;     /* [count] candidate indices grouped by partition, draw order inside */
    int64_t start[GG_NPART + 1];
    gg_set* part;        /* [GG_NPART] */
    int err;
} gg_draws;

static void gg_draws_gen(void* c, int64_t b, int64_t e) {
    gg_draws* B = (gg_draws*)c;
    for (int64_t i = b; i < e; ++i) {
        const uint64_t k = gg_candidate(B->f, B->first + (uint64_t)i);
        B->key[i] = k;
        B->pid[i] = (uint8_t)(k == GG_REJECT ? GG_NPART : gg_part(k));
    }
}
static void gg_draws_dedup(void* c, int64_t b, int64_t e) {
    gg_draws* B = (gg_draws*)c;
    for (int64_t p = b; p < e; ++p) {
        for (int64_t j = B->start[p]; j < B->start[p + 1]; ++j) {
            const uint32_t i = B->order[j];
            int r = gg_set_insert(&B->part[p], B->key[i]);
            if (r < 0) { B->err = -2; return; }
            B->fresh[i] = (uint8_t)r;
        }
    }
}

/* append the first (m - *k_out) distinct valid candidates, in draw order */
static int gg_draw_edges(const gg_family* f, int64_t m, uint32_t* eu, uint32_t* ev,
                         int64_t* k_out, gg_set* part) {
    int64_t k = *k_out;
    uint64_t next = 0;
    while (k < m) {
        int64_t want = m - k;
        int64_t count = want + want / 4 + 4096;
        gg_draws B;
        memset(&B, 0, sizeof B);
        B.f = f; B.first = next; B.part = part;
        B.key = (uint64_t*)malloc((size_t)count * 8);
        B.pid = (uint8_t*)malloc((size_t)count);
        B.fresh = (uint8_t*)calloc((size_t)count, 1);
        B.order = (uint32_t*)malloc((size_t)count * 4);
        if (!B.key || !B.pid || !B.fresh || !B.order) {
            free(B.key); free(B.pid); free(B.fresh); free(B.order);
            return -2;
        }
        gg_parallel(gg_draws_gen, &B, count, 1 << 16);
        /* group candidate indices by partition, keeping draw order inside each */
        int64_t cnt[GG_NPART + 1] = {0};
        for (int64_t i = 0; i < count; ++i) cnt[B.pid[i]]++;
        int64_t fill[GG_NPART];
        B.start[0] = 0;
        for (int p = 0; p < GG_NPART; ++p) { fill[p] = B.start[p]; B.start[p + 1] = B.start[p] + cnt[p]; }
        for (int64_t i = 0; i < count; ++i)
            if (B.pid[i] < GG_NPART) B.order[fill[B.pid[i]]++] = (uint32_t)i;
        gg_parallel(gg_draws_dedup, &B, GG_NPART, 1);
        if (B.err) { free(B.key); free(B.pid); free(B.fresh); free(B.order); return B.err; }
        for (int64_t i = 0; i < count && k < m; ++i) {
            if (!B.fresh[i]) continue;
            eu[k] = (uint32_t)(B.key[i] >> 32);
            ev[k] = (uint32_t)B.key[i];
            ++k;
        }
        next += (uint64_t)count;
        free(B.key); free(B.pid); free(B.fresh); free(B.order);
    }
    *k_out = k;
    return 0;
}

/* ------------------------------------------------------------- CSR build */
typedef struct {
    int64_t n, m; const uint32_t* eu; const uint32_t* ev;
    int64_t* row_ptr; int32_t* col_idx; int64_t* cursor;
} gg_csr_ctx;

static void gg_csr_scatter(void* c, int64_t b, int64_t e) {
    gg_csr_ctx* C = (gg_csr_ctx*)c;
    for (int64_t i = b; i < e; ++i) {
        uint32_t u = C->eu[i], v = C->ev[i];
        int64_t p = __atomic_fetch_add(&C->cursor[u], 1, __ATOMIC_RELAXED);
        C->col_idx[p] = (int32_t)v;
        p = __atomic_fetch_add(&C->cursor[v], 1, __ATOMIC_RELAXED);
        C->col_idx[p] = (int32_t)u;
    }
}
static int gg_cmp_i32(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}
static void gg_csr_sort(void* c, int64_t b, int64_t e) {
    gg_csr_ctx* C = (gg_csr_ctx*)c;
    for (int64_t r = b; r < e; ++r) {
        int32_t* a = C->col_idx + C->row_ptr[r];
        int64_t len = C->row_ptr[r + 1] - C->row_ptr[r];
        if (len <= 32) {
            for (int64_t i = 1; i < len; ++i) {
                int32_t x = a[i]; int64_t j = i - 1;
                while (j >= 0 && a[j] > x) { a[j + 1] = a[j]; --j; }
                a[j + 1] = x;
            }
        } else {
            qsort(a, (size_t)len, 4, gg_cmp_i32);
        }
    }
}

/* CSR from an undirected edge list (each edge once); rows sorted ascending */
static int gg_csr(int64_t n, int64_t m, const uint32_t* eu, const uint32_t* ev,
                  int64_t* row_ptr, int32_t* col_idx) {
    int64_t* cursor = (int64_t*)malloc((size_t)(n + 1) * 8);
    if (!cursor) return -2;
    memset(row_ptr, 0, (size_t)(n + 1) * 8);
    for (int64_t e = 0; e < m; ++e) { row_ptr[eu[e] + 1]++; row_ptr[ev[e] + 1]++; }
    for (int64_t i = 0; i < n; ++i) row_ptr[i + 1] += row_ptr[i];
    memcpy(cursor, row_ptr, (size_t)n * 8);
    gg_csr_ctx C = { n, m, eu, ev, row_ptr, col_idx, cursor };
    gg_parallel(gg_csr_scatter, &C, m, 1 << 16);
    gg_parallel(gg_csr_sort, &C, n, 1 << 12);
    free(cursor);
    return 0;
}

static int gg_parts_init(gg_set* part, int64_t m) {
    for (int p = 0; p < GG_NPART; ++p) {
        if (gg_set_init(&part[p], m / GG_NPART + 64)) {
            for (int q = 0; q < p; ++q) free(part[q].slot);
            return -2;
        }
    }
    return 0;
}
static void gg_parts_free(gg_set* part) {
    for (int p = 0; p < GG_NPART; ++p) free(part[p].slot);
}

static int64_t gg_family_graph(const gg_family* f, int64_t n, int64_t m,
                               int64_t* row_ptr, int32_t* col_idx) {
    uint32_t* eu = (uint32_t*)malloc((size_t)(m ? m : 1) * 4);
    uint32_t* ev = (uint32_t*)malloc((size_t)(m ? m : 1) * 4);
    gg_set part[GG_NPART];
    if (!eu || !ev || gg_parts_init(part, m)) { free(eu); free(ev); return -2; }
    int64_t k = 0;
    int rc = gg_draw_edges(f, m, eu, ev, &k, part);
    gg_parts_free(part);
    if (!rc) rc = gg_csr(n, m, eu, ev, row_ptr, col_idx);
    free(eu); free(ev);
    return rc ? rc : m;
}

/* ---------------------------------------------------------- Erdos-Renyi */
int64_t gg_er(int64_t n, int64_t m, uint64_t seed, int64_t* row_ptr, int32_t* col_idx) {
    if (n < 0 || m < 0 || n > 0x7fffffff || !row_ptr || (m > 0 && !col_idx)) return -1;
    if (m > n * (n - 1) / 2) return -3;
    if (m > n * (n - 1) / 4 + 1024) return -3;   /* rejection sampling would crawl */
    gg_family f;
    memset(&f, 0, sizeof f);
    f.kind = 1; f.stream = gg_derive(seed, 1); f.n = n;
    return gg_family_graph(&f, n, m, row_ptr, col_idx);
}

/* ---------------------------------------------------------------- R-MAT
 * a, b, c are quadrant probabilities scaled to 2^32 (d = the rest); quadrant per
 * level from one 32-bit draw r: r < a -> (0,0); < a+b -> (0,1); < a+b+c -> (1,0);
 * else (1,1); levels fill bits from the most significant down. */
typedef struct { const uint32_t* perm; uint32_t* eu; uint32_t* ev; } gg_relabel_ctx;
static void gg_relabel(void* c, int64_t b, int64_t e) {
    gg_relabel_ctx* R = (gg_relabel_ctx*)c;
    for (int64_t i = b; i < e; ++i) { R->eu[i] = R->perm[R->eu[i]]; R->ev[i] = R->perm[R->ev[i]]; }
}

int64_t gg_rmat(int64_t n, int64_t m, uint64_t a32, uint64_t b32, uint64_t c32,
                int permute, uint64_t seed, int64_t* row_ptr, int32_t* col_idx) {
    if (n < 1 || m < 0 || n > 0x7fffffff || !row_ptr || (m > 0 && !col_idx)) return -1;
    if (a32 + b32 + c32 > (1ull << 32)) return -1;
    if (m > n * (n - 1) / 4 + 1024) return -3;
    gg_family f;
    memset(&f, 0, sizeof f);
    f.kind = 2; f.stream = gg_derive(seed, 2); f.n = n;
    int scale = 0;
    while ((1ll << scale) < n) ++scale;
    f.scale = scale; f.draws = (scale + 1) / 2;
    f.t1 = a32; f.t2 = a32 + b32; f.t3 = a32 + b32 + c32;
    uint32_t* eu = (uint32_t*)malloc((size_t)(m ? m : 1) * 4);
    uint32_t* ev = (uint32_t*)malloc((size_t)(m ? m : 1) * 4);
    gg_set part[GG_NPART];
    if (!eu || !ev || gg_parts_init(part, m)) { free(eu); free(ev); return -2; }
    int64_t k = 0;
    int rc = gg_draw_edges(&f, m, eu, ev, &k, part);
    gg_parts_free(part);
    if (!rc && permute) {
        /* Fisher-Yates relabelling: newid = perm[old] */
        uint32_t* perm = (uint32_t*)malloc((size_t)n * 4);
        if (!perm) rc = -2;
        else {
            uint64_t s = gg_derive(seed, 3);
            for (int64_t i = 0; i < n; ++i) perm[i] = (uint32_t)i;
            for (int64_t i = n - 1, t = 1; i > 0; --i, ++t) {
                uint32_t j = gg_bounded32((uint32_t)(gg_at(s, (uint64_t)t) >> 32), (uint64_t)(i + 1));
                uint32_t tmp = perm[i]; perm[i] = perm[j]; perm[j] = tmp;
            }
            gg_relabel_ctx R = { perm, eu, ev };
            gg_parallel(gg_relabel, &R, m, 1 << 16);
            free(perm);
        }
    }
    if (!rc) rc = gg_csr(n, m, eu, ev, row_ptr, col_idx);
    free(eu); free(ev);
    return rc ? rc : m;
}

/* ------------------------------------------------ 3D grid + long range */
int64_t gg_grid_edges(int64_t sx, int64_t sy, int64_t sz) {
    if (sx < 1 || sy < 1 || sz < 1) return -1;
    return (sx - 1) * sy * sz + sx * (sy - 1) * sz + sx * sy * (sz - 1);
}

int64_t gg_grid(int64_t sx, int64_t sy, int64_t sz, int64_t n_long, uint64_t seed,
                int64_t* row_ptr, int32_t* col_idx) {
    if (sx < 1 || sy < 1 || sz < 1 || n_long < 0 || !row_ptr) return -1;
    int64_t n = sx * sy * sz;
    if (n > 0x7fffffff) return -1;
    int64_t mg = gg_grid_edges(sx, sy, sz);
    int64_t m = mg + n_long;
    if (n_long > (n * (n - 1) / 2 - mg) / 2 + 16) return -3;
    if (m > 0 && !col_idx) return -1;
    uint32_t* eu = (uint32_t*)malloc((size_t)(m ? m : 1) * 4);
    uint32_t* ev = (uint32_t*)malloc((size_t)(m ? m : 1) * 4);
    if (!eu || !ev) { free(eu); free(ev); return -2; }
    int64_t k = 0;
    for (int64_t z = 0; z < sz; ++z)
        for (int64_t y = 0; y < sy; ++y)
            for (int64_t x = 0; x < sx; ++x) {
                uint32_t v = (uint32_t)(x + sx * y + sx * sy * z);
                if (x + 1 < sx) { eu[k] = v; ev[k] = v + 1; ++k; }
                if (y + 1 < sy) { eu[k] = v; ev[k] = (uint32_t)(v + sx); ++k; }
                if (z + 1 < sz) { eu[k] = v; ev[k] = (uint32_t)(v + sx * sy); ++k; }
            }
    int rc = 0;
    if (n_long > 0) {
        gg_family f;
        memset(&f, 0, sizeof f);
        f.kind = 1; f.stream = gg_derive(seed, 4); f.n = n;
        f.gx = sx; f.gy = sy; f.gz = sz;
        gg_set part[GG_NPART];
        if (gg_parts_init(part, n_long)) rc = -2;
        else {
            rc = gg_draw_edges(&f, m, eu, ev, &k, part);
            gg_parts_free(part);
        }
    }
    if (!rc) rc = gg_csr(n, m, eu, ev, row_ptr, col_idx);
    free(eu); free(ev);
    return rc ? rc : m;
}

/* ------------------------------------------------ batches of graphs
 * Disjoint union of `count` graphs, graph g of kind[g] (1 = Erdos-Renyi G(a, b),
 * 2 = R-MAT with n = a, m = b, the given quadrant thresholds and relabelling,
 * 3 = grid a x a x a with b long-range pairs) and seed[g].  voff (count+1) and eoff
 * (count+1, directed entries) are the caller's prefix sums of the vertex counts
 * and of 2 * edges; graph g fills row_ptr[voff[g] .. voff[g+1]-1] and
 * col_idx[eoff[g] .. eoff[g+1]-1] with ids shifted by voff[g], exactly as if it
 * were generated alone and appended.  Graphs with at least `big` edges are made
 * one at a time with every thread; the rest in parallel, one thread each. */
typedef struct {
    const int32_t* kind; const int64_t* a; const int64_t* b; const uint64_t* seed;
    const int64_t* voff; const int64_t* eoff; uint64_t t1, t2, t3;
    int64_t* row_ptr; int32_t* col_idx; int64_t big; int small_pass; int rc;
    pthread_mutex_t mu;
} gg_batch_ctx;

static int gg_batch_one(gg_batch_ctx* B, int64_t g) {
    const int64_t n = B->voff[g + 1] - B->voff[g], e0 = B->eoff[g];
    int64_t* rp = (int64_t*)malloc((size_t)(n + 1) * 8);
    if (!rp) return -2;
    int32_t* ci = B->col_idx + e0;
    int64_t m;
    switch (B->kind[g]) {
        case 1: m = gg_er(B->a[g], B->b[g], B->seed[g], rp, ci); break;
        case 2: m = gg_rmat(B->a[g], B->b[g], B->t1, B->t2 - B->t1, B->t3 - B->t2, 1, B->seed[g], rp, ci); break;
        case 3: m = gg_grid(B->a[g], B->a[g], B->a[g], B->b[g], B->seed[g], rp, ci); break;
        default: m = -1;
    }
    int rc = 0;
    if (m < 0) rc = (int)m;
    else if (2 * m != B->eoff[g + 1] - e0 || rp[n] != 2 * m) rc = -1;
    else {
        const int32_t o = (int32_t)B->voff[g];
        for (int64_t k = 0; k < 2 * m; ++k) ci[k] += o;
        for (int64_t v = 0; v < n; ++v) B->row_ptr[B->voff[g] + v] = e0 + rp[v];
    }
    free(rp);
    return rc;
}

static void gg_batch_body(void* c, int64_t b, int64_t e) {
    gg_batch_ctx* B = (gg_batch_ctx*)c;
    gg_single_thread = 1;
    for (int64_t g = b; g < e; ++g) {
        if (B->eoff[g + 1] - B->eoff[g] >= 2 * B->big) continue;
        int rc = gg_batch_one(B, g);
        if (rc) { pthread_mutex_lock(&B->mu); B->rc = rc; pthread_mutex_unlock(&B->mu); }
    }
    gg_single_thread = 0;
}

int64_t gg_union(int64_t count, const int32_t* kind, const int64_t* a, const int64_t* b, const uint64_t* seed,
                 uint64_t a32, uint64_t b32, uint64_t c32, const int64_t* voff, const int64_t* eoff,
                 int64_t big, int64_t* row_ptr, int32_t* col_idx) {
    if (count < 0 || !kind || !a || !b || !seed || !voff || !eoff || !row_ptr) return -1;
    if (a32 + b32 + c32 > (1ull << 32) || voff[count] > 0x7fffffff) return -1;
    if (eoff[count] > 0 && !col_idx) return -1;
    gg_batch_ctx B;
    memset(&B, 0, sizeof B);
    B.kind = kind; B.a = a; B.b = b; B.seed = seed; B.voff = voff; B.eoff = eoff;
    B.t1 = a32; B.t2 = a32 + b32; B.t3 = a32 + b32 + c32;
    B.row_ptr = row_ptr; B.col_idx = col_idx; B.big = big;
    pthread_mutex_init(&B.mu, NULL);
    for (int64_t g = 0; g < count && !B.rc; ++g)
        if (eoff[g + 1] - eoff[g] >= 2 * big) B.rc = gg_batch_one(&B, g);
    if (!B.rc) gg_parallel(gg_batch_body, &B, count, 1);
    pthread_mutex_destroy(&B.mu);
    if (B.rc) return B.rc;
    row_ptr[voff[count]] = eoff[count];
    return eoff[count] / 2;
}

/* raw SplitMix64 stream: outputs 1..count of the stream seeded with seed */
void gg_splitmix64(uint64_t seed, int64_t count, uint64_t* out) {
    for (int64_t i = 0; i < count; ++i) out[i] = gg_at(seed, (uint64_t)i + 1);
}

/* membership test used by the generator's own tests: is {u, v} drawn as an
 * edge of the CSR?  (binary search in the sorted row) */
int gg_has_edge(const int64_t* row_ptr, const int32_t* col_idx, int32_t u, int32_t v) {
    int64_t lo = row_ptr[u], hi = row_ptr[u + 1];
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (col_idx[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo < row_ptr[u + 1] && col_idx[lo] == v;
}
