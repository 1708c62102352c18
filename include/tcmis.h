/*
 * tcmis.h -- C ABI of the MI355X (gfx950) priority-MIS library.
 *
 * The library computes the maximal independent set that round-synchronous,
 * fixed-priority selection produces (TC-MIS, Algorithm 2, Section 3.1): in every
 * round each undecided vertex whose priority beats all undecided neighbours
 * becomes a candidate (Phase 1); the candidate-neighbour count N_c = A x C is
 * formed (Phase 2); candidates join the set and vertices with N_c > 0 leave it
 * (Phase 3).  For a fixed strict total order of priorities the result is unique
 * (it equals the sequential greedy in decreasing priority order), so results are
 * bit-exact across paths, tile sizes, reorderings and launch shapes.
 *
 * Conventions for every entry point:
 *   - Pointers marked DEVICE are HIP device pointers on the current device;
 *     pointers marked HOST are ordinary host memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work is
 *     enqueued on it; calls that must read results back say that they
 *     synchronise it.
 *   - Return value: MIS_OK (0) or a negative mis_status.  Argument errors are
 *     detected on the host before any device work is enqueued.  After an error
 *     mis_last_error() returns a thread-local message with details.
 *   - A solve keeps its round state either in a caller's scratch (mis_solve with
 *     scratch != NULL: any number of such solves of one handle may run
 *     concurrently, on different streams or threads, each with its own scratch)
 *     or in the handle's own round state (scratch == NULL: one such solve at a
 *     time per handle).  The structure is read-only to solves, except that the
 *     hybrid path's round 1 writes the higher-priority neighbour rows of the
 *     vertices it leaves undecided into the handle: every solve of a handle
 *     writes the same values there, so concurrent solves stay correct.
 *     mis_update_edges changes a handle and must not overlap any solve of it.
 */
#ifndef TCMIS_H
#define TCMIS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MIS_OK = 0,
    MIS_EINVAL = -1,      /* bad argument (null pointer, negative size, bad option) */
    MIS_ENOTSYM = -2,     /* validate: adjacency not symmetric */
    MIS_ESELFLOOP = -3,   /* validate: self-loop (a vertex could never be a candidate) */
    MIS_EDUP = -4,        /* validate: duplicate or unsorted adjacency entries */
    MIS_ERANGE = -5,      /* validate: column index out of [0, n) or bad row_ptr */
    MIS_ENOMEM = -6,      /* host allocation failed */
    MIS_EBUSY = -7,       /* session: no free slot or arena region right now (retry later) */
    MIS_EHIP = -8,        /* a HIP runtime call failed */
    MIS_EINTERNAL = -9    /* round limit exceeded or broken invariant */
} mis_status;

/* Path through the round kernels. */
enum {
    MIS_PATH_AUTO = 0,    /* hybrid path (mis_autotune picks per graph) */
    MIS_PATH_TILE = 1,    /* every edge in T x T bit tiles: LDS-staged candidate phase + int8 MFMA
                             exclusion, on a reordered vertex set */
    MIS_PATH_CSR = 2,     /* scalar CSR path (the plain GPU method) */
    MIS_PATH_HYBRID = 3   /* per 16-row block of the input order: the edges to higher-priority
                             neighbours as 16 x 16 bit tiles on int8 MFMA where the block is dense
                             (opts.dense_min), as sorted entry lists otherwise; both phases read
                             alive / in-set bitmaps (Section 3.2, memory footprint trade-offs) */
};

/* Vertex order used to lay out tiles (results are always in input ids). */
enum {
    MIS_REORDER_AUTO = 0,
    MIS_REORDER_NONE = 1,    /* input order (natural order of meshes) */
    MIS_REORDER_DEGREE = 2,  /* decreasing degree class floor(255 / (1 + deg)), ties by id */
    MIS_REORDER_KEY = 3,     /* decreasing priority key: tile column < row <=> higher key */
    MIS_REORDER_RCM = 4      /* reverse Cuthill-McKee (host), banded meshes */
};

/* Priority rule of the default keys (Section 3.3; all are 64-bit keys
 * q << 56 | h << 24 | v with h the top 32 bits of output v+1 of the SplitMix64
 * stream seeded with opts.seed, v the (graph-local) id; higher key wins). */
enum {
    MIS_KEY_DEGREE = 0,   /* q = floor(255 / (1 + deg v)): the degree-aware priority (H2/H3 order) */
    MIS_KEY_HASH = 1,     /* q = 0: the purely random priority P(v) = hash(v) (H1) */
    MIS_KEY_EQ1 = 2       /* q = min(255, floor(255 D / (D + 256 deg v - e))) with D = floor(256 nnz / n)
                             (the average degree, 8 fractional bits) and e the low 8 bits of the
                             same SplitMix64 output (the perturbation, in 1/256): Eq. 1,
                             d / (d + deg v - eps), scaled and discretised; q = 255 where the
                             denominator is not positive.  In a batch, n and nnz are the graph's own */
};

/* How the rounds are launched (results are identical). */
enum {
    MIS_LAUNCH_AUTO = 0,      /* direct on a handle's first solve; from its second solve on a
                                 hipGraph (captured then, once) when capture works */
    MIS_LAUNCH_DIRECT = 1,    /* one kernel launch per phase (2 CSR, 3 tiles), enqueued back to back */
    MIS_LAUNCH_GRAPH = 2,     /* poll_rounds rounds captured once as a hipGraph and replayed */
    MIS_LAUNCH_PERSISTENT = 3 /* poll_rounds rounds per cooperative launch, grid barriers between
                                 phases (workgroups stay resident; every barrier wait is bounded and
                                 a timeout is reported as MIS_EINTERNAL) */
};

/* Input graph: undirected, simple, symmetric CSR, rows sorted ascending. */
typedef struct {
    int64_t n;                /* vertices, 0 <= n < 2^31 */
    int64_t nnz;              /* directed entries = 2 |E| = row_ptr[n]; < 2^31 on the tile and CSR
                                 paths, < 2^40 on the hybrid path */
    const int64_t* row_ptr;   /* DEVICE int64[n+1] */
    const int32_t* col_idx;   /* DEVICE int32[nnz] */
} mis_csr;

typedef struct {
    int32_t path;             /* MIS_PATH_* */
    int32_t tile;             /* 0 = auto, 16 or 32 */
    int32_t reorder;          /* MIS_REORDER_* */
    int32_t orient;           /* -1 = auto, 0 = full symmetric tiles, candidate phase compares
                                 LDS-staged neighbour keys; 1 = tiles keep only edges to
                                 higher-priority neighbours (candidate phase needs no keys) */
    int32_t validate;         /* 1 = check symmetry/loops/duplicates/range on the device */
    int32_t poll_rounds;      /* rounds enqueued between termination polls (0 = default 4) */
    int32_t launch;           /* MIS_LAUNCH_* */
    int32_t blocks_per_cu;    /* workgroups per compute unit of the persistent round kernels
                                 (0 = default 8, at most 32) */
    int32_t dense_min;        /* hybrid path: a 16-row block whose higher-priority edges average at
                                 least this many per nonzero 16 x 16 tile (and fit 64 tiles) is
                                 stored as bit tiles, every other block as entry lists.
                                 0 = default (16; a 36-byte tile costs no more bytes than 9
                                 4-byte indices, but blocks near that break-even run faster
                                 as lists), -1 = entry lists only */
    int32_t key_rule;         /* default priority rule when keys == NULL (MIS_KEY_*; Section 3.3) */
    int32_t timing;           /* 1 = record HIP events between the build's stages on the build
                                 stream (read them with mis_build_times) */
    int32_t dyn_slack;        /* hybrid path, one graph, dense_min -1: > 0 makes the handle
                                 dynamic (mis_update_edges): both orientations kept in rows of
                                 its own with this many free slots per row and orientation;
                                 0 = static handle */
    uint64_t seed;            /* priority seed (default key rule) */
    const uint64_t* keys;     /* optional DEVICE uint64[n], pairwise distinct priorities
                                 (higher wins); NULL = default key rule, needs n <= 2^24 */
} mis_build_opts;

/* Fills opts with defaults: auto path/tile/reorder/orient, validate 0, seed 1. */
void mis_default_opts(mis_build_opts* opts);

/* Per-solve statistics (HOST struct).  Fields marked "in" are read by mis_solve;
 * all others are written. */
typedef struct {
    int32_t rounds;           /* rounds until every vertex was decided (or max_rounds) */
    int32_t path;             /* path used */
    int32_t tile;             /* tile size used (0 on the CSR path) */
    int32_t reorder;          /* reorder used */
    int32_t orient;           /* orientation used */
    int32_t timing;           /* in: 1 = time every kernel with HIP events on `stream` */
    int64_t n_in;             /* size of the independent set */
    int64_t tiles;            /* nonzero tiles (0 on the CSR path) */
    int64_t tile_bytes;       /* bytes of the tile stream: tiles * (T*T/8 bitmap + 4 index) */
    int64_t alg_bytes;        /* algorithmic bytes: sum over rounds of units[k] * bytes per unit */
    int64_t units[8];         /* work units summed over rounds.  CSR path: adjacency entries read
                                 by the candidate kernel (12 B each: index + neighbour key),
                                 vertices it examined (28 B), entries read by the exclusion
                                 kernel (8 B: index + neighbour state), vertices it examined
                                 (24 B), units[4..7] = 0.  Tile path: 4-byte index and
                                 row-mask words the candidate kernel read (4 B), bytes of
                                 bitmaps and neighbour keys it read (1 B), 4-byte words the
                                 exclusion kernel read (4 B), tiles it multiplied on the matrix
                                 cores (T*T/8 B), row-blocks the finalize kernel updated (24 B:
                                 three row masks read and written), chunk list entries it
                                 wrote (8 B), units[6..7] = 0.  Hybrid path: entries the
                                 candidate kernel read (8 B: index + the bitmap word it
                                 selects), rows it examined (16 B: list slot, row start, count),
                                 the same two for the exclusion kernel, tiles multiplied on the
                                 matrix cores by the candidate and by the exclusion kernel
                                 (36 B: bitmap + column block), dense row-blocks each examined
                                 (24 B: list slot, block slot, tile range, two bitmap words). */
    float kernel_ms[3];       /* timing = 1: total ms of the candidate / exclusion / finalize
                                 kernels (the CSR path has no finalize kernel) */
    int32_t launches;         /* timing = 1: rounds enqueued (each launches every kernel once) */
    int32_t trace_cap;        /* in: rounds the trace buffer holds (0 = no trace) */
    int32_t graph;            /* 1 if full batches of rounds ran as a replayed hipGraph, 2 if as
                                 persistent cooperative launches */
    int32_t pad3_;
    int64_t* trace;           /* in: optional HOST int64[3*trace_cap]; out: per round |C_r|,
                                 vertices removed as neighbours of candidates, alive after */
} mis_stats;

typedef struct mis_graph mis_graph;   /* opaque host handle; device memory is the caller's workspace */

/*
 * Device workspace bytes that mis_build_tiles needs for this graph and these
 * options (host-only arithmetic on n, nnz and the options; no device access).
 * The figure is an upper bound (tile counts are bounded by the entry count), and
 * it is the handle's whole device footprint: tiles, keys, per-round state,
 * build temporaries.
 */
int mis_build_bytes(const mis_csr* csr, const mis_build_opts* opts, size_t* bytes);

/*
 * Builds the solver structure of a graph inside a caller-provided workspace:
 * priority keys (the degree-aware priority of Eq. 1, discretised), the vertex
 * reordering and the nonzero T x T bit tiles with a row-block index (Section 3.2:
 * only nonzero tiles are stored, in a compressed block format), or the
 * degree-binned vertex lists of the CSR path.
 *   csr       : the graph (DEVICE arrays; must stay alive and unchanged while the
 *               handle is used -- the CSR and hybrid paths read it during solves).
 *   opts      : NULL = defaults.
 *   workspace : DEVICE memory of at least mis_build_bytes bytes, 256-byte aligned,
 *               owned by the caller; it must outlive the handle and must not be
 *               touched while work of the handle is in flight.
 *   out       : receives the handle (host memory owned by the library).
 * All device work is enqueued on `stream`; nothing is allocated on the device and
 * the stream is not synchronised, except with validate = 1 (the error flags are
 * read back) or reorder = MIS_REORDER_RCM (the order is computed on the host).
 * Errors: MIS_EINVAL (also: workspace too small or misaligned),
 * MIS_ENOTSYM/ESELFLOOP/EDUP/ERANGE (validate = 1), MIS_EHIP.
 */
int mis_build_tiles(const mis_csr* csr, const mis_build_opts* opts, void* workspace, size_t workspace_bytes,
                    void* stream, mis_graph** out);

/* Workspace bytes the handle uses (as mis_build_bytes reported for it). */
int mis_graph_bytes(const mis_graph* g, size_t* bytes);

/*
 * Device bytes of one solve's round state for this handle (control block, trace
 * ring, counters, per-vertex status bitmaps or words, next-round work lists), the
 * scratch that mis_solve takes.  Host-only.  Errors: MIS_EINVAL (null argument).
 */
int mis_solve_scratch_bytes(const mis_graph* g, size_t* bytes);

/*
 * Runs the rounds of Algorithm 2 (Section 3.1: Phase 1 candidates, Phase 2
 * N_c = A x C, Phase 3 updates, until no vertex is undecided) over a built handle
 * and writes in_set[v] = 1 if vertex v (input id) is in the independent set, else 0.
 *   in_set        : DEVICE uint8[n], caller-owned.
 *   max_rounds    : > 0 stops after that many rounds (vertices still undecided are
 *                   written as 0; stats->rounds tells how many ran); 0 = run to
 *                   completion.
 *   scratch       : DEVICE, 256-byte aligned, at least mis_solve_scratch_bytes
 *                   bytes, caller-owned; holds this solve's round state, so that
 *                   the handle is only read and concurrent solves of one handle
 *                   with different scratch buffers are allowed.  NULL = the round
 *                   state inside the handle's workspace (then one solve at a time
 *                   per handle, and repeated solves may replay a captured graph of
 *                   the round loop, launch = AUTO or GRAPH).
 *   scratch_bytes : its size (ignored when scratch is NULL).
 *   stats         : optional HOST.
 * Enqueues `poll_rounds` rounds at a time and synchronises `stream` after each
 * batch to read the alive counter; returns when every vertex is decided.
 * Errors: MIS_EINVAL (null handle or output, negative max_rounds, scratch too small
 * or misaligned), MIS_EINTERNAL (round limit, device-side check), MIS_EHIP.
 */
int mis_solve(mis_graph* g, uint8_t* in_set, int32_t max_rounds, void* scratch, size_t scratch_bytes,
              mis_stats* stats, void* stream);

/*
 * Batches: `count` independent graphs solved together as one block-diagonal graph.
 *   csr     : the disjoint union of the graphs (DEVICE arrays): graph g owns vertices
 *             offsets[g] .. offsets[g+1]-1 and has no edge to another graph.
 *   offsets : HOST int64[count+1], offsets[0] = 0, offsets[count] = csr->n.
 * Priorities use graph-local ids (vertex v of graph g gets the key of vertex
 * v - offsets[g] in g alone), so graph g's result is identical to solving it alone,
 * and so is its number of rounds.  Every round kernel covers all graphs of the batch
 * in one launch.  With validate = 1 an edge between two graphs is rejected
 * (MIS_EINVAL).  Workspace, streams and errors as for mis_build_tiles.
 */
int mis_build_batch_bytes(const mis_csr* csr, int32_t count, const int64_t* offsets, const mis_build_opts* opts,
                          size_t* bytes);
int mis_build_batch(const mis_csr* csr, int32_t count, const int64_t* offsets, const mis_build_opts* opts,
                    void* workspace, size_t workspace_bytes, void* stream, mis_graph** out);

/*
 * Solves a batch built with mis_build_batch (the rounds of Algorithm 2 over the
 * block-diagonal union; Section 3.1).  in_set: DEVICE uint8[csr->n] (graph g's
 * answer is in_set[offsets[g] .. offsets[g+1]-1]).  stats: optional HOST, for the
 * whole batch (rounds = the largest per-graph round count).  graph_rounds (HOST
 * int32[count]) and graph_in (HOST int64[count]), optional: each graph's own number
 * of rounds and set size.  Uses the handle's own round state.  Synchronises `stream`.
 * Errors: MIS_EINVAL (null handle, or one not built by mis_build_batch), MIS_EHIP,
 * MIS_EINTERNAL.
 */
int mis_solve_union(mis_graph* batch, uint8_t* in_set, mis_stats* stats, int32_t* graph_rounds, int64_t* graph_in,
                    void* stream);

/*
 * Solves independently built handles together, without concatenating or rebuilding
 * anything: the rounds of Algorithm 2 (Section 3.1) run for all graphs at once, every
 * round kernel one launch whose workgroups are split into per-graph shares over each
 * handle's own (read-only) structure, with every graph's round state in `scratch`.
 * Graphs share no edge, so each graph's result and number of rounds equal its solve
 * alone.
 *   graphs        : HOST array of `count` single-graph handles built by
 *                   mis_build_tiles with the hybrid path (they may differ in size,
 *                   options and dense-block threshold).
 *   in_sets       : HOST array of `count` DEVICE uint8 outputs, in_sets[i] of
 *                   graphs[i]'s n bytes (input ids).
 *   scratch       : DEVICE, 256-byte aligned, at least mis_solve_batch_scratch_bytes
 *                   for these handles, caller-owned.
 *   stats         : optional HOST, for the whole batch (rounds = the largest
 *                   per-graph round count, n_in = the total set size).
 *   graph_rounds  : optional HOST int32[count]; graph_in: optional HOST int64[count].
 * Rounds are enqueued poll_rounds (the largest of the handles') at a time; the
 * stream is synchronised after each batch of rounds.  The handles are only read, so
 * they may be solved elsewhere at the same time with other scratch.
 * Errors: MIS_EINVAL (a null or non-hybrid or batch handle, a null output, scratch
 * too small or misaligned), MIS_EINTERNAL (round limit, device-side check), MIS_EHIP.
 */
int mis_solve_batch_scratch_bytes(mis_graph* const* graphs, int32_t count, size_t* bytes);
int mis_solve_batch(mis_graph* const* graphs, int32_t count, uint8_t* const* in_sets, void* scratch,
                    size_t scratch_bytes, mis_stats* stats, int32_t* graph_rounds, int64_t* graph_in, void* stream);

/*
 * Autotuning of implementation choices that leave the result unchanged (path,
 * tile size, vertex order, the hybrid path's dense-block threshold, grid size of the
 * round kernels).  Measures the degree profile of the graph (or batch: count/offsets
 * as for mis_build_batch, count = 0 for one graph) on the device, rounds it to a
 * bucket, and on the first graph of a bucket builds and solves every candidate --
 * the CSR path; the hybrid path with dense_min -1 (entry lists only), 4, 9 or 16;
 * the tile path with tile 16 or 32 in key, degree or input order (and RCM order,
 * at one grid size, when the maximum degree is at most four times the average) --
 * at 4/8/16 workgroups per CU, twice in the workspace, timing the second run of
 * build + solve with HIP events.  The fastest candidate is cached per bucket
 * (process-wide, thread-safe) and written to *out as complete build options (base's
 * seed, keys, validate, poll_rounds and launch are kept).  A nonzero path, tile,
 * blocks_per_cu or dense_min in `base` fixes that choice.
 *   workspace : DEVICE, 256-byte aligned, at least mis_autotune_bytes bytes; its
 *               contents are scratch.  from_cache (HOST, optional): 1 if no trial ran.
 * Synchronises `stream`.  Every candidate computes the same set; only time differs.
 * Errors: MIS_EINVAL, MIS_EHIP, MIS_EINTERNAL (no candidate could run).
 */
int mis_autotune_bytes(const mis_csr* csr, int32_t count, const int64_t* offsets, const mis_build_opts* base,
                       size_t* bytes);
int mis_autotune(const mis_csr* csr, int32_t count, const int64_t* offsets, const mis_build_opts* base,
                 void* workspace, size_t workspace_bytes, void* stream, mis_build_opts* out, int32_t* from_cache);
/* Forgets every tuned bucket. */
void mis_autotune_clear(void);

/*
 * Serving session: continuous batching of independent MIS requests on one GPU.
 * Requests are admitted while others run, as long as a slot and a region of the
 * caller's device arena are free (admission by HBM footprint: the request's CSR copy,
 * its solver structure from mis_build_bytes and its output).  Every live request
 * has its own stream; mis_session_progress enqueues its rounds rounds_per_step at a
 * time without waiting on any one request, so the rounds of all live requests
 * overlap on the device, and a request admitted between two progress calls starts
 * at once instead of waiting for the others to finish.  A request's result is
 * identical to solving it alone (its kernels read only its own state).
 * A session is driven by one host thread at a time.
 */
typedef struct mis_session mis_session;

typedef struct {
    void* arena;              /* DEVICE, 256-byte aligned, caller-owned; every per-request
                                 device byte comes from here (no device allocation) */
    size_t arena_bytes;
    int32_t max_live;         /* requests on the device at once, 1..256 */
    int32_t rounds_per_step;  /* rounds enqueued per request between polls (0 = 4) */
    mis_build_opts opts;      /* build options of requests admitted without their own
                                 (launch must not be MIS_LAUNCH_PERSISTENT) */
} mis_session_config;

typedef struct {
    uint64_t tag;             /* the caller's tag from mis_session_admit */
    int32_t status;           /* MIS_OK, or MIS_EINTERNAL if the round bound was exceeded or a
                                 device-side check raised an error flag (the output is then
                                 not a valid result) */
    int32_t rounds;           /* rounds the request took */
    int64_t n;                /* vertices */
    int64_t n_in;             /* size of its independent set */
    double admit_s, done_s;   /* seconds since session creation: admission, retirement */
} mis_done;

/* Creates a session (streams, events, pinned host mirrors; no device memory). */
int mis_session_create(const mis_session_config* cfg, mis_session** out);

/*
 * Admits one request: copies its CSR to the arena if csr_on_host (HOST arrays that
 * must stay valid until the request retires; pinned memory keeps the copy
 * asynchronous), builds its solver structure, and enqueues its first rounds.
 *   opts  : NULL = the session's options (poll_rounds is the session's rounds_per_step)
 *   d_out : DEVICE uint8[n] for the result, or NULL to place it in the arena
 *   h_out : HOST uint8[n] that receives the result when the request retires, or NULL
 *           (at least one of d_out / h_out).
 * Returns MIS_EBUSY, with nothing enqueued, when no slot or no arena region of the
 * request's footprint is free (retry after mis_session_progress retires requests),
 * and MIS_EINVAL when the footprint exceeds the whole arena or opts asks for
 * MIS_LAUNCH_PERSISTENT (cooperative grids of concurrent requests could not all be
 * resident).  Validation options
 * (validate = 1, reorder = MIS_REORDER_RCM) synchronise the request's stream.
 */
int mis_session_admit(mis_session* s, const mis_csr* csr, int32_t csr_on_host, const mis_build_opts* opts,
                      uint8_t* d_out, uint8_t* h_out, uint64_t tag);

/*
 * Advances every live request whose last enqueued work has finished (next rounds,
 * or output), and retires finished requests into done[0 .. *n_done-1] (HOST, at
 * most cap), freeing their slot and arena region.  wait = 0 returns at once;
 * wait = 1 returns once at least one request retired or none is live.
 */
int mis_session_progress(mis_session* s, int32_t wait, mis_done* done, int32_t cap, int32_t* n_done);

/*
 * The two halves of mis_session_progress, for callers that drive them separately.
 * mis_session_step advances, without waiting, every live request whose last enqueued
 * rounds have finished: its next rounds_per_step rounds (the rounds stay on the
 * device between steps), or its output once no vertex is undecided; *advanced
 * (HOST, optional) receives how many it advanced.  mis_session_poll retires
 * requests whose output has landed into done[0 .. *n_done-1] (HOST, at most cap),
 * freeing their slot and arena region; it enqueues nothing.  wait = 1 returns once
 * at least one request retired or no request is waiting for its output.
 * Errors: MIS_EINVAL, MIS_EHIP.
 */
int mis_session_step(mis_session* s, int32_t* advanced);
int mis_session_poll(mis_session* s, int32_t wait, mis_done* done, int32_t cap, int32_t* n_done);

/* Live requests, arena bytes in use and the largest free arena region (HOST, each optional). */
int mis_session_query(const mis_session* s, int32_t* live, size_t* bytes_in_use, size_t* largest_free);

/* Waits for the session's device work, then releases it (the arena stays the caller's). */
void mis_session_destroy(mis_session* s);

/*
 * Durations (HOST float[cap], milliseconds, from HIP events on the build stream) of
 * the build stages of a handle built with opts.timing = 1; *count receives the
 * number of stages.  Stages (after validation, which is not timed): keys, then
 *   hybrid path: dense blocks (every block's test and the bitmaps, or only the
 *                empty slot map when the sample of blocks the key stage takes found
 *                too few), then empty stages; a dynamic handle (dyn_slack > 0):
 *                orientation row search (with clearing the counts), orientation,
 *                then empty stages; an empty graph has the keys stage only;
 *   tile path:   vertex order, tiles;
 *   CSR path:    vertex lists.
 * Synchronises the last event.  Errors: MIS_EINVAL (no timing), MIS_EHIP.
 */
int mis_build_times(const mis_graph* g, float* ms, int32_t cap, int32_t* count);

/*
 * Build + solve in one call that allocates nothing: for callers that cannot allocate
 * (code under stream capture, tight serving loops, harnesses that forbid
 * allocation).  It computes what mis_build_tiles + mis_solve compute for the same
 * graph and options, with the solver structure and round state in a device array
 * of mis_noalloc_max_bytes() bytes (64 MiB) that the library holds on every GPU it
 * runs on until the process ends.  It calls no device or host allocation routine:
 * no workspace argument, no pooled pinned buffers (the round loop polls into host
 * stack memory), no captured graph (rounds are launched directly).
 *   csr, opts : as for mis_build_tiles (opts NULL = defaults); the CSR stays the
 *               caller's.  Refused with MIS_EINVAL: reorder = MIS_REORDER_RCM (host
 *               buffers), timing = 1 (events), launch graph or persistent, and any
 *               graph whose structure (mis_build_bytes) exceeds the array.
 *   in_set    : DEVICE uint8[n], as for mis_solve.
 *   rounds, n_in : HOST, optional: rounds run and the set's size.
 * Synchronises `stream`.  All calls on one GPU share its array (the last call's
 * contents stay there; every call rebuilds what it reads), so calls that may
 * overlap on one GPU -- from several threads, or on streams not ordered with each
 * other -- race and must be serialised by the caller.
 * Errors: as mis_build_tiles and mis_solve.
 */
int mis_solve_noalloc(const mis_csr* csr, const mis_build_opts* opts, uint8_t* in_set, int32_t* rounds, int64_t* n_in,
                      void* stream);

/* Bytes of the per-GPU array behind mis_solve_noalloc. */
size_t mis_noalloc_max_bytes(void);

/*
 * Edge insertions and deletions on a dynamic handle (hybrid path, built with
 * dyn_slack > 0), and the repair of its set (Section 5's dynamic setting).
 * Priorities stay those of the build, so the result is the set the
 * round-synchronous rule gives on the edited graph with the build's keys; only the
 * lower-priority ends of the edited edges and the vertices below a vertex whose
 * status changes are decided again.
 *   edges  : DEVICE int32[2*count], edge i = {edges[2i], edges[2i+1]} (either order)
 *   ops    : DEVICE int8[count], 1 = insert (the edge must be absent), 0 = delete
 *            (the edge must be present); an edge appears at most once per batch
 *   in_set : DEVICE uint8[n]; in: the handle's current result (from mis_solve or the
 *            previous update), out: the result on the edited graph
 *   stats  : optional HOST: rounds of the repair, n_in, units[0] = entries read
 * Deletes apply before inserts.  The handle's rows change in place, and a later
 * mis_solve solves the edited graph from scratch.  When the edits leave more than
 * n/256 vertices to re-decide, or one of them with more than 4,096 higher-priority
 * neighbours (a hub's row would be scanned in every repair round), the set is
 * recomputed by a full solve of the edited handle instead (the same result; stats
 * then describe that solve).  Synchronises `stream`.
 * Errors: MIS_EINVAL (not a dynamic handle; an edit out of range, a self-loop or a
 * missing edge), MIS_ENOMEM (a row ran out of slots: the handle no longer holds
 * that edge -- rebuild with a larger dyn_slack), MIS_EHIP.
 */
int mis_update_edges(mis_graph* g, const int32_t* edges, const int8_t* ops, int64_t count, uint8_t* in_set,
                     mis_stats* stats, void* stream);

/* Releases the handle (host memory only; the workspace stays the caller's). */
void mis_free_tiles(mis_graph* g);

/*
 * Frees the pinned host buffers that idle solves keep for their round-loop polls
 * (solves take one from a process-wide pool and give it back).  Optional: call it
 * before the HIP runtime is shut down, e.g. at the end of a program; no library
 * code frees host or device memory from a static destructor.  Solves running on
 * other threads keep their buffers; a later solve allocates a new one.
 */
void mis_release_host_buffers(void);

/* Static text for a status code. */
const char* mis_status_string(int status);

/* Thread-local detail of the last error on this thread ("" if none). */
const char* mis_last_error(void);

/* Library version string. */
const char* mis_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TCMIS_H */
