/* Host driver for the sanitizer build of the library: every host-side argument
 * check of the C ABI (no device work: each call below fails, or only sizes, on the
 * host), so that AddressSanitizer / UndefinedBehaviorSanitizer see the option
 * resolution, the layout arithmetic and the error paths.  Prints "ok" or the first
 * failed check. */
#include <stdio.h>
#include <string.h>

#include "../../include/tcmis.h"

#define CHECK(c)                                                   \
    do {                                                           \
        if (!(c)) {                                                \
            printf("failed: %s (line %d)\n", #c, __LINE__);        \
            return 1;                                              \
        }                                                          \
    } while (0)

int main(void) {
    mis_build_opts o;
    mis_default_opts(&o);
    mis_csr csr = {1000, 8000, (const int64_t*)256, (const int32_t*)256};
    size_t bytes = 0, prev = 0;
    const int paths[4] = {MIS_PATH_AUTO, MIS_PATH_TILE, MIS_PATH_CSR, MIS_PATH_HYBRID};
    for (int p = 0; p < 4; ++p) {
        for (int tile = 0; tile <= 32; tile += 16) {
            mis_default_opts(&o);
            o.path = paths[p];
            o.tile = tile;
            const int rc = mis_build_bytes(&csr, &o, &bytes);
            CHECK(rc == MIS_OK || rc == MIS_EINVAL);
            if (rc == MIS_OK) CHECK(bytes > 0);
        }
    }
    mis_default_opts(&o);
    o.dyn_slack = 8;
    CHECK(mis_build_bytes(&csr, &o, &bytes) == MIS_OK && bytes > prev);
    o.dense_min = 9;
    CHECK(mis_build_bytes(&csr, &o, &bytes) == MIS_EINVAL);
    /* out-of-range options */
    const int bad_field[9] = {0, 1, 2, 3, 4, 5, 6, 7, 8};
    for (int f = 0; f < 9; ++f) {
        mis_default_opts(&o);
        switch (bad_field[f]) {
            case 0: o.path = 9; break;
            case 1: o.tile = 8; break;
            case 2: o.reorder = 11; break;
            case 3: o.orient = 3; break;
            case 4: o.poll_rounds = -1; break;
            case 5: o.launch = 7; break;
            case 6: o.dense_min = -5; break;
            case 7: o.key_rule = 4; break;
            default: o.dyn_slack = -2; break;
        }
        CHECK(mis_build_bytes(&csr, &o, &bytes) == MIS_EINVAL);
        CHECK(strlen(mis_last_error()) > 0);
    }
    /* graphs the paths cannot hold */
    mis_csr wide = {10, (int64_t)1 << 31, (const int64_t*)256, (const int32_t*)256};
    mis_default_opts(&o);
    o.path = MIS_PATH_CSR;
    CHECK(mis_build_bytes(&wide, &o, &bytes) == MIS_EINVAL);
    o.path = MIS_PATH_HYBRID;
    CHECK(mis_build_bytes(&wide, &o, &bytes) == MIS_OK);
    mis_csr big = {((int64_t)1 << 24) + 1, 0, (const int64_t*)256, 0};
    CHECK(mis_build_bytes(&big, NULL, &bytes) == MIS_EINVAL);
    /* builds that fail before any device work */
    mis_graph* g = (mis_graph*)1;
    CHECK(mis_build_tiles(&csr, NULL, (void*)256, 16, NULL, &g) == MIS_EINVAL && g == NULL);
    CHECK(mis_build_tiles(&csr, NULL, (void*)(256 + 64), (size_t)1 << 40, NULL, &g) == MIS_EINVAL);
    CHECK(mis_build_tiles(NULL, NULL, (void*)256, 16, NULL, &g) == MIS_EINVAL);
    int64_t off[4] = {0, 300, 200, 1000};
    CHECK(mis_build_batch_bytes(&csr, 3, off, NULL, &bytes) == MIS_EINVAL);
    off[2] = 600;
    CHECK(mis_build_batch_bytes(&csr, 3, off, NULL, &bytes) == MIS_OK);
    mis_default_opts(&o);
    o.dyn_slack = 4;
    CHECK(mis_build_batch_bytes(&csr, 3, off, &o, &bytes) == MIS_EINVAL);
    /* calls on null handles */
    CHECK(mis_solve(NULL, NULL, 0, NULL, 0, NULL, NULL) == MIS_EINVAL);
    CHECK(mis_solve_union(NULL, NULL, NULL, NULL, NULL, NULL) == MIS_EINVAL);
    CHECK(mis_solve_batch(NULL, 1, NULL, NULL, 0, NULL, NULL, NULL, NULL) == MIS_EINVAL);
    CHECK(mis_solve_batch_scratch_bytes(NULL, 1, &bytes) == MIS_EINVAL);
    CHECK(mis_solve_scratch_bytes(NULL, &bytes) == MIS_EINVAL);
    CHECK(mis_session_step(NULL, NULL) == MIS_EINVAL);
    CHECK(mis_graph_bytes(NULL, NULL) == MIS_EINVAL);
    float ms[4];
    int32_t cnt = 0;
    CHECK(mis_build_times(NULL, ms, 4, &cnt) == MIS_EINVAL);
    CHECK(mis_update_edges(NULL, NULL, NULL, 0, NULL, NULL, NULL) == MIS_EINVAL);
    mis_free_tiles(NULL);
    /* the no-allocation entry point refuses what it cannot hold, on the host */
    mis_csr huge = {(int64_t)1 << 22, (int64_t)1 << 25, (const int64_t*)256, (const int32_t*)256};
    CHECK(mis_solve_noalloc(&huge, NULL, (uint8_t*)256, NULL, NULL, NULL) == MIS_EINVAL);
    mis_default_opts(&o);
    o.reorder = MIS_REORDER_RCM;
    o.path = MIS_PATH_TILE;
    CHECK(mis_solve_noalloc(&csr, &o, (uint8_t*)256, NULL, NULL, NULL) == MIS_EINVAL);
    CHECK(mis_noalloc_max_bytes() > 0);
    /* autotune sizing and session argument checks */
    CHECK(mis_autotune_bytes(&csr, 0, NULL, NULL, &bytes) == MIS_OK && bytes > 0);
    CHECK(mis_autotune_bytes(NULL, 0, NULL, NULL, &bytes) == MIS_EINVAL);
    mis_session_config cfg;
    memset(&cfg, 0, sizeof(cfg));
    mis_default_opts(&cfg.opts);
    mis_session* s = NULL;
    CHECK(mis_session_create(&cfg, &s) == MIS_EINVAL && s == NULL);
    cfg.arena = (void*)256;
    cfg.arena_bytes = 1 << 20;
    cfg.max_live = 0;
    CHECK(mis_session_create(&cfg, &s) == MIS_EINVAL);
    cfg.max_live = 2;
    cfg.opts.launch = MIS_LAUNCH_PERSISTENT;
    CHECK(mis_session_create(&cfg, &s) == MIS_EINVAL);
    int32_t n_done = 0;
    CHECK(mis_session_progress(NULL, 0, NULL, 0, &n_done) == MIS_EINVAL);
    CHECK(mis_session_query(NULL, NULL, NULL, NULL) == MIS_EINVAL);
    mis_session_destroy(NULL);
    for (int c = -12; c <= 1; ++c) CHECK(mis_status_string(c) != NULL);
    CHECK(strncmp(mis_version(), "tcmis", 5) == 0);
    mis_release_host_buffers();
    printf("ok\n");
    return 0;
}
