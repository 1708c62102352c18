/* Host driver for the sanitizer build of the oracle and the input generator: every
 * entry point runs on small graphs (generated, hand-made and invalid ones) and the
 * results are cross-checked, so that AddressSanitizer / UndefinedBehaviorSanitizer
 * see every code path the test suite drives through ctypes.  Prints "ok" or the
 * first failed check. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* oracle */
void orc_splitmix_stream(uint64_t seed, int64_t count, uint64_t* out);
int orc_keys(int64_t n, const int64_t* row_ptr, uint64_t seed, uint64_t* keys);
int orc_keys_rule(int64_t n, const int64_t* row_ptr, uint64_t seed, int rule, uint64_t* keys);
int orc_validate(int64_t n, const int64_t* row_ptr, const int32_t* col_idx);
int64_t orc_roundsync(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, const uint64_t* key,
                      int64_t max_rounds, uint8_t* status, int64_t* trace, int64_t trace_cap);
int64_t orc_greedy(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, const uint64_t* key, uint8_t* in_set);
int orc_verify(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, const uint8_t* in_set);
int64_t orc_lfmis_cert(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, const uint64_t* key,
                       const uint8_t* in_set);
int64_t orc_mindeg_greedy(int64_t n, const int64_t* row_ptr, const int32_t* col_idx, uint8_t* in_set);
/* generator */
int64_t gg_er(int64_t n, int64_t m, uint64_t seed, int64_t* row_ptr, int32_t* col_idx);
int64_t gg_rmat(int64_t n, int64_t m, uint64_t a32, uint64_t b32, uint64_t c32, int permute, uint64_t seed,
                int64_t* row_ptr, int32_t* col_idx);
int64_t gg_grid_edges(int64_t sx, int64_t sy, int64_t sz);
int64_t gg_grid(int64_t sx, int64_t sy, int64_t sz, int64_t n_long, uint64_t seed, int64_t* row_ptr,
                int32_t* col_idx);

#define CHECK(c)                                                   \
    do {                                                           \
        if (!(c)) {                                                \
            printf("failed: %s (line %d)\n", #c, __LINE__);        \
            return 1;                                              \
        }                                                          \
    } while (0)

static int solve_all(int64_t n, const int64_t* rp, const int32_t* ci) {
    uint64_t* key = malloc((size_t)(n ? n : 1) * 8);
    uint8_t* st = malloc((size_t)(n ? n : 1));
    uint8_t* gr = malloc((size_t)(n ? n : 1));
    uint8_t* md = malloc((size_t)(n ? n : 1));
    int64_t* tr = malloc((size_t)(3 * (n + 1)) * 8);
    CHECK(key && st && gr && md && tr);
    CHECK(orc_validate(n, rp, ci) == 0);
    for (int rule = 0; rule < 3; ++rule) {
        CHECK(orc_keys_rule(n, rp, 7, rule, key) == 0);
        const int64_t r = orc_roundsync(n, rp, ci, key, 0, st, tr, n + 1);
        CHECK(r >= 0 && r <= n + 1);
        CHECK(orc_greedy(n, rp, ci, key, gr) >= 0);
        for (int64_t v = 0; v < n; ++v) CHECK((st[v] == 1) == (gr[v] == 1));
        for (int64_t v = 0; v < n; ++v) st[v] = st[v] == 1;
        CHECK(orc_verify(n, rp, ci, st) == 0);
        CHECK(orc_lfmis_cert(n, rp, ci, key, st) == 0);
        if (r > 1) CHECK(orc_roundsync(n, rp, ci, key, r - 1, st, tr, n + 1) == r - 1);
    }
    CHECK(orc_keys(n, rp, 7, key) == 0);
    CHECK(orc_mindeg_greedy(n, rp, ci, md) >= 0);
    CHECK(orc_verify(n, rp, ci, md) == 0);
    free(key); free(st); free(gr); free(md); free(tr);
    return 0;
}

int main(void) {
    uint64_t sm[8];
    orc_splitmix_stream(1234567, 8, sm);
    CHECK(sm[0] != sm[1]);
    /* generated graphs */
    {
        const int64_t n = 3000, m = 12000;
        int64_t* rp = malloc((n + 1) * 8);
        int32_t* ci = malloc(2 * m * 4);
        CHECK(gg_er(n, m, 5, rp, ci) == m);
        CHECK(solve_all(n, rp, ci) == 0);
        const uint64_t a32 = (uint64_t)(0.57 * 4294967296.0), b32 = (uint64_t)(0.19 * 4294967296.0);
        free(rp); free(ci);
        const int64_t nr = 4096, mr = 8 * 4096;
        rp = malloc((nr + 1) * 8);
        ci = malloc(2 * mr * 4);
        CHECK(gg_rmat(nr, mr, a32, b32, b32, 1, 3, rp, ci) == mr);
        CHECK(solve_all(nr, rp, ci) == 0);
        free(rp); free(ci);
        const int64_t s = 12, mg = gg_grid_edges(s, s, s), nl = mg / 100;
        rp = malloc((s * s * s + 1) * 8);
        ci = malloc(2 * (mg + nl) * 4);
        CHECK(gg_grid(s, s, s, nl, 9, rp, ci) == mg + nl);
        CHECK(solve_all(s * s * s, rp, ci) == 0);
        free(rp); free(ci);
    }
    /* hand-made: empty, single vertex, star */
    {
        int64_t rp0[1] = {0};
        int32_t ci0[1] = {0};
        CHECK(solve_all(0, rp0, ci0) == 0);
        int64_t rp1[2] = {0, 0};
        CHECK(solve_all(1, rp1, ci0) == 0);
        int64_t rps[7] = {0, 5, 6, 7, 8, 9, 10};
        int32_t cis[10] = {1, 2, 3, 4, 5, 0, 0, 0, 0, 0};
        CHECK(solve_all(6, rps, cis) == 0);
    }
    /* invalid graphs: the validator reports, nothing reads out of bounds */
    {
        int64_t rp[3] = {0, 1, 2};
        int32_t loop[2] = {0, 0}, range[2] = {1, 7}, asym[1] = {1};
        CHECK(orc_validate(2, rp, loop) == -3);
        CHECK(orc_validate(2, rp, range) == -5);
        int64_t rpa[3] = {0, 1, 1};
        CHECK(orc_validate(2, rpa, asym) == -2);
        int64_t rpd[3] = {0, 2, 4};
        int32_t dup[4] = {1, 1, 0, 0};
        CHECK(orc_validate(2, rpd, dup) == -4);
        uint64_t k[2];
        CHECK(orc_keys_rule(2, rp, 1, 5, k) == -2);
    }
    printf("ok\n");
    return 0;
}
