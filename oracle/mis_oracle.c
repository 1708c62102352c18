/*
 * CPU oracle for round-synchronous priority MIS -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct host implementation of what the GPU library
 * computes.  Only the test suite, the smoke check and the benchmark's CPU
 * baseline may load it; the GPU library never links or calls it and the two
 * share no source.
 *
 * What it follows (TC-MIS: Maximal Independent Set on Tensor-Cores):
 *   - Algorithm 2 (TC-MIS) and its three phases, Section 3.1 "Base Algorithm":
 *       Phase 1: Max_Np(v) = max over u in N(v) ∩ A of P(u); C(v) = [P(v) > Max_Np(v)]
 *       Phase 2: N_c = A x C (number of candidate neighbours of every vertex)
 *       Phase 3: C(v)=1 -> v joins the MIS and leaves A; C(v)=0 and N_c(v)>0 -> v
 *                leaves A; C(v)=0 and N_c(v)=0 -> v stays in A.
 *   - Priorities fixed once per solve, as in the random-permutation variant of
 *     Luby's algorithm that ECL-MIS builds on (Background section); the updates of
 *     a round are applied only after C is final (heuristic H3's ordering,
 *     Section 3.3).
 *   - The priority itself: Eq. 1 favours low degree with a random perturbation,
 *     "scaled and discretized" to an integer.  Reading used here (the paper gives no
 *     constants): key(v) = q(deg v) << 56 | h(seed, v) << 24 | v, unsigned 64-bit,
 *     higher key wins, with q(d) = floor(255 / (1 + d)) and h the top 32 bits of
 *     output v+1 of the SplitMix64 stream seeded with `seed`.  Requires v < 2^24.
 *
 * Pins (tests run without a GPU): sequential greedy in key order must give the
 * identical set (the round-synchronous fixed-priority process computes the
 * lexicographically-first MIS for that order); independence + maximality
 * verifier; brute-force enumeration on graphs of <= 20 vertices; closed-form
 * special cases; the published SplitMix64 test vector.
 *
 * Status codes: 0 = UNDECIDED, 1 = IN, 2 = OUT.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------- priority */

/* SplitMix64 output i (i >= 1) of the stream seeded with s (Steele, Lea, Flood 2014) */
static uint64_t orc_splitmix(uint64_t s, uint64_t i) {
    uint64_t z = s + i * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

void orc_splitmix_stream(uint64_t seed, int64_t count, uint64_t* out) {
    for (int64_t i = 0; i < count; ++i) out[i] = orc_splitmix(seed, (uint64_t)i + 1);
}

/* discretised degree priority: floor(255 / (1 + deg)) */
uint64_t orc_q(int64_t deg) { return (uint64_t)(255 / (1 + deg)); }

uint64_t orc_key(uint64_t seed, int64_t v, int64_t deg) {
    uint64_t h = orc_splitmix(seed, (uint64_t)v + 1) >> 32;
    return (orc_q(deg) << 56) | (h << 24) | (uint64_t)v;
}

/* keys for every vertex; -1 if n > 2^24 (v does not fit the tie-break field) */
int orc_keys(int64_t n, const int64_t* row_ptr, uint64_t seed, uint64_t* keys) {
    if (n > (1ll << 24)) return -1;
    for (int64_t v = 0; v < n; ++v) keys[v] = orc_key(seed, v, row_ptr[v + 1] - row_ptr[v]);
    return 0;
}

/* The three priority heuristics of Section 3.3, as key rules (rule 0 is orc_keys):
 *   0  degree-aware: q = floor(255 / (1 + deg))
 *   1  H1, purely random priority P(v) = hash(v): q = 0, the key is the hash and id
 *   2  Eq. 1, P(v) = dbar / (dbar + deg(v) - eps(v)), scaled to 255 and discretised.
 *      Reading (the paper gives no constants): dbar is taken with 8 fractional
 *      bits, D = floor(256 nnz / n); eps = e / 256 with e the low 8 bits of the same
 *      SplitMix64 output whose top 32 bits are the hash; then
 *      q = floor(255 * D / (D + 256 deg - e)), at most 255, and 255 when that
 *      denominator is not positive (an isolated vertex: P >= 1).
 * In every rule key(v) = q << 56 | hash << 24 | v, as for rule 0.  The graph here
 * is one graph (a batch applies the rule per graph with its own n and nnz).
 * Returns -1 if n > 2^24, -2 for an unknown rule. */
int orc_keys_rule(int64_t n, const int64_t* row_ptr, uint64_t seed, int rule, uint64_t* keys) {
    if (n > (1ll << 24)) return -1;
    if (rule < 0 || rule > 2) return -2;
    const int64_t nnz = n > 0 ? row_ptr[n] - row_ptr[0] : 0;
    const int64_t D = n > 0 ? (256 * nnz) / n : 0;
    for (int64_t v = 0; v < n; ++v) {
        const int64_t deg = row_ptr[v + 1] - row_ptr[v];
        const uint64_t z = orc_splitmix(seed, (uint64_t)v + 1);
        uint64_t q;
        if (rule == 0) {
            q = orc_q(deg);
        } else if (rule == 1) {
            q = 0;
        } else {
            const int64_t e = (int64_t)(z & 0xFF);
            const int64_t den = D + 256 * deg - e;
            if (den <= 0) {
                q = 255;
            } else {
                const int64_t x = (255 * D) / den;
                q = (uint64_t)(x > 255 ? 255 : x);
            }
        }
        keys[v] = (q << 56) | ((z >> 32) << 24) | (uint64_t)v;
    }
    return 0;
}

/* ------------------------------------------------------------ validation */

/* 0 ok; -5 index out of range / bad row_ptr; -3 self-loop; -4 duplicate; -2 asymmetric.
 * Brute force per edge (rows need not be sorted). */
int orc_validate(int64_t n, const int64_t* row_ptr, const int32_t* col_idx) {
    if (n < 0 || row_ptr[0] != 0) return -5;
    for (int64_t v = 0; v < n; ++v)
        if (row_ptr[v + 1] < row_ptr[v]) return -5;
    for (int64_t v = 0; v < n; ++v) {
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            int64_t u = col_idx[e];
            if (u < 0 || u >= n) return -5;
        }
    }
    for (int64_t v = 0; v < n; ++v) {
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            int64_t u = col_idx[e];
            if (u == v) return -3;
            for (int64_t f = row_ptr[v]; f < e; ++f)
                if (col_idx[f] == u) return -4;
            int found = 0;
            for (int64_t f = row_ptr[u]; f < row_ptr[u + 1]; ++f)
                if (col_idx[f] == v) { found = 1; break; }
            if (!found) return -2;
        }
    }
    return 0;
}

/* ---------------------------------------------- round-synchronous solve */

/*
 * Runs rounds of Algorithm 2 until A is empty or max_rounds (> 0) rounds ran.
 * status[n] (out): final status of every vertex.  trace (optional, 3 per round):
 * |C_r|, number of vertices removed as neighbours of candidates, |A| after the
 * round.  Returns the number of rounds run, or -1 on allocation failure.
 */
int64_t orc_roundsync(int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                      const uint64_t* key, int64_t max_rounds, uint8_t* status,
                      int64_t* trace, int64_t trace_cap) {
    uint8_t* C = (uint8_t*)malloc((size_t)(n ? n : 1));
    int64_t* Nc = (int64_t*)malloc((size_t)(n ? n : 1) * sizeof(int64_t));
    if (!C || !Nc) { free(C); free(Nc); return -1; }
    for (int64_t v = 0; v < n; ++v) status[v] = 0;     /* A <- V */
    int64_t alive = n, rounds = 0;
    while (alive > 0 && (max_rounds <= 0 || rounds < max_rounds)) {
        ++rounds;
        /* Phase 1: neighbour maximum over the alive set and the strict test */
        for (int64_t v = 0; v < n; ++v) {
            C[v] = 0;
            if (status[v] != 0) continue;
            int has = 0;
            uint64_t max_np = 0;
            for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
                int64_t u = col_idx[e];
                if (status[u] != 0) continue;
                if (!has || key[u] > max_np) { max_np = key[u]; has = 1; }
            }
            C[v] = (uint8_t)(!has || key[v] > max_np);  /* empty max is -infinity */
        }
        /* Phase 2: N_c = A x C over the whole adjacency matrix */
        for (int64_t v = 0; v < n; ++v) {
            int64_t s = 0;
            for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) s += C[col_idx[e]];
            Nc[v] = s;
        }
        /* Phase 3: state update of the alive vertices, after C is final */
        int64_t n_in = 0, n_out = 0;
        for (int64_t v = 0; v < n; ++v) {
            if (status[v] != 0) continue;
            if (C[v]) { status[v] = 1; ++n_in; }
            else if (Nc[v] > 0) { status[v] = 2; ++n_out; }
        }
        alive -= n_in + n_out;
        if (trace && rounds <= trace_cap) {
            trace[3 * (rounds - 1) + 0] = n_in;
            trace[3 * (rounds - 1) + 1] = n_out;
            trace[3 * (rounds - 1) + 2] = alive;
        }
    }
    free(C); free(Nc);
    return rounds;
}

/* ------------------------------------------------ sequential greedy (pin) */

static const uint64_t* orc_sort_key;
static int orc_cmp_desc(const void* a, const void* b) {
    uint64_t x = orc_sort_key[*(const int64_t*)a], y = orc_sort_key[*(const int64_t*)b];
    return (x < y) - (x > y);
}

/* scan vertices in decreasing key order; take v iff no neighbour taken.  Returns |I| or -1. */
int64_t orc_greedy(int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                   const uint64_t* key, uint8_t* in_set) {
    int64_t* order = (int64_t*)malloc((size_t)(n ? n : 1) * sizeof(int64_t));
    if (!order) return -1;
    for (int64_t v = 0; v < n; ++v) { order[v] = v; in_set[v] = 0; }
    orc_sort_key = key;
    qsort(order, (size_t)n, sizeof(int64_t), orc_cmp_desc);
    int64_t size = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t v = order[i];
        int blocked = 0;
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e)
            if (in_set[col_idx[e]]) { blocked = 1; break; }
        if (!blocked) { in_set[v] = 1; ++size; }
    }
    free(order);
    return size;
}

/* ------------------------------------------------------------- verifiers */

/* 0 = maximal independent set; 1 = an edge inside the set; 2 = not maximal */
int orc_verify(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, const uint8_t* in_set) {
    for (int64_t v = 0; v < n; ++v) {
        int has_in_nbr = 0;
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            if (in_set[col_idx[e]]) {
                if (in_set[v]) return 1;
                has_in_nbr = 1;
            }
        }
        if (!in_set[v] && !has_in_nbr) return 2;
    }
    return 0;
}

/* lexicographically-first certificate: in(v) <=> no higher-key neighbour is in.
 * Returns 0 if it holds for every vertex, else 1 + the first violating vertex. */
int64_t orc_lfmis_cert(int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                       const uint64_t* key, const uint8_t* in_set) {
    for (int64_t v = 0; v < n; ++v) {
        int dominated = 0;
        for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
            int64_t u = col_idx[e];
            if (key[u] > key[v] && in_set[u]) { dominated = 1; break; }
        }
        if ((in_set[v] != 0) == dominated) return v + 1;
    }
    return 0;
}

/* ------------------------------------- minimum-degree greedy (quality only) */

typedef struct { int64_t deg, v; } orc_hent;
static int orc_hless(orc_hent a, orc_hent b) { return a.deg < b.deg || (a.deg == b.deg && a.v < b.v); }
static void orc_hpush(orc_hent* h, int64_t* sz, orc_hent x) {
    int64_t i = (*sz)++;
    h[i] = x;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (!orc_hless(h[i], h[p])) break;
        orc_hent t = h[i]; h[i] = h[p]; h[p] = t; i = p;
    }
}
static orc_hent orc_hpop(orc_hent* h, int64_t* sz) {
    orc_hent top = h[0];
    h[0] = h[--(*sz)];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, s = i;
        if (l < *sz && orc_hless(h[l], h[s])) s = l;
        if (r < *sz && orc_hless(h[r], h[s])) s = r;
        if (s == i) break;
        orc_hent t = h[i]; h[i] = h[s]; h[s] = t; i = s;
    }
    return top;
}

/* Repeatedly take the undecided vertex of minimum residual degree (ties: smallest
 * id), remove it and its neighbours.  A quality reference, not part of the method.
 * Returns |I| or -1. */
int64_t orc_mindeg_greedy(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, uint8_t* in_set) {
    int64_t cap = n + row_ptr[n] + 1;
    orc_hent* h = (orc_hent*)malloc((size_t)cap * sizeof(orc_hent));
    int64_t* deg = (int64_t*)malloc((size_t)(n ? n : 1) * sizeof(int64_t));
    uint8_t* st = (uint8_t*)calloc((size_t)(n ? n : 1), 1);
    if (!h || !deg || !st) { free(h); free(deg); free(st); return -1; }
    int64_t sz = 0, size = 0;
    for (int64_t v = 0; v < n; ++v) {
        in_set[v] = 0;
        deg[v] = row_ptr[v + 1] - row_ptr[v];
        orc_hent x = { deg[v], v };
        orc_hpush(h, &sz, x);
    }
    while (sz > 0) {
        orc_hent x = orc_hpop(h, &sz);
        if (st[x.v] || x.deg != deg[x.v]) continue;     /* stale entry */
        in_set[x.v] = 1; st[x.v] = 1; ++size;
        for (int64_t e = row_ptr[x.v]; e < row_ptr[x.v + 1]; ++e) {
            int64_t u = col_idx[e];
            if (st[u]) continue;
            st[u] = 2;
            for (int64_t f = row_ptr[u]; f < row_ptr[u + 1]; ++f) {
                int64_t w = col_idx[f];
                if (st[w]) continue;
                deg[w]--;
                orc_hent y = { deg[w], w };
                orc_hpush(h, &sz, y);
            }
        }
    }
    free(h); free(deg); free(st);
    return size;
}
