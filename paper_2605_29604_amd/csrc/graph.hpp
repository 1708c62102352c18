// The opaque handle behind mis_graph, its device workspace layout and the
// device-side round control block.
#pragma once
#include <cstddef>
#include <atomic>
#include <type_traits>
#include <vector>

#include "common.hpp"

namespace tcmis {

constexpr int kLightDeg = 32;       // CSR path: thread per vertex up to this degree, wave above
constexpr int kTraceCap = 4096;     // device trace ring (rounds); the host drains it at every poll
constexpr int kUnits = 8;           // work-unit counters per round (TraceRec::u)
constexpr int kStripes = 128;       // round counters are spread over this many cache lines (a multiple of 64)
constexpr int kStripeWords = 16;    // int64 words per stripe (one 128-byte line)
// hybrid: entries per tile from which a 16-row block takes bit tiles by default.  A
// 36-byte 16x16 tile costs no more bytes than 9 entry indices, but each dense block
// costs its wave a chain of dependent steps per round, so blocks near that break-even
// (a 7-point mesh in natural order: about 9.4) run faster as entry lists.
constexpr int kDenseMinDefault = 16;

// Device control block of the round loop.  Round r's kernels take r as an
// argument and count into the round-parity half of the counter stripes (each
// workgroup adds into stripe blockIdx % kStripes, so no single line takes every
// atomic); round r is closed (stripes summed into the trace ring and cleared,
// `alive` and `round` advanced) by the first wave of round r+1's first kernel, or
// by the one-wave close kernel the host enqueues before it reads the block.  No
// workgroup ever waits for another, and no fence is needed: every
// cross-workgroup hand-over crosses a kernel boundary.
struct Ctrl {
    int32_t round;          // rounds closed
    int32_t rbase;          // rounds enqueued before the current batch (round = rbase + index in batch)
    uint32_t error;         // invariant violation flags
    int32_t pad0;
    int64_t alive;          // undecided vertices after `round` rounds
    int64_t n_in;           // vertices in the set so far
    int64_t n_act[2][4];    // active work items per list buffer (CSR: [light, heavy]; tile: [chunks,
                            // row-blocks]; hybrid: [light rows, heavy rows, dense row-blocks])
    unsigned long long bar; // grid-barrier arrivals of persistent launches (only grows)
};
// Counter words of a stripe: |C|, removed neighbours, work units u0..u5.

// A tile chunk: at most 64 consecutive tiles of one row-block, packed as
// t0 (bits 33..63) | len - 1 (bits 27..32) | row-block (bits 0..26).
__host__ __device__ inline uint64_t chunk_word(int64_t t0, int64_t len, int64_t I) {
    return ((uint64_t)t0 << 33) | ((uint64_t)(len - 1) << 27) | (uint64_t)I;
}
// an unused slot of a chunk list (no chunk has all bits set: tile indices stay below 2^31 - 1)
constexpr uint64_t kChunkHole = ~0ull;

// Per-round trace record in the device ring.
//   c, x, alive : |C_r|, vertices removed as neighbours of candidates, undecided after r
//   u[0..7]     : work units.  CSR path: adjacency entries read by the candidate
//                 kernel, vertices it examined, entries read by the exclusion kernel,
//                 vertices it examined (u4..u7 = 0).  Tile path: 4-byte index and
//                 mask words the candidate kernel read, bytes of bitmaps and keys it
//                 read, 4-byte words the exclusion kernel read, tiles it multiplied on
//                 the matrix cores, row-blocks the finalize kernel updated, chunk list
//                 entries it wrote (u6 = u7 = 0).  Hybrid path: entries read and rows
//                 examined by the candidate kernel, the same for the exclusion kernel,
//                 tiles multiplied by the candidate and by the exclusion kernel, dense
//                 row-blocks examined by each.
struct TraceRec {
    int64_t c, x, alive, round;
    int64_t u[kUnits];
};

// Sizes the build produces on the device (never read back during the build).
struct alignas(8) Meta {
    int32_t ntiles;         // nonzero tiles
    int32_t nvalid;         // adjacency entries kept in tiles
    int64_t nchunks;        // tile path: chunks of the round-1 list
    int32_t n_light;        // CSR path: vertices with degree <= kLightDeg
    int32_t pad;
    // hybrid path
    int32_t n_dense;        // dense row-blocks (bit tiles)
    int32_t n_dtiles;       // their tiles (the build reserves both in one 64-bit atomic)
    int32_t n_dcand;        // dense candidates among the sampled row-blocks
    int32_t n_done;         // workgroups of the dense-block build that finished
};
static_assert(offsetof(Meta, n_dense) % 8 == 0 && offsetof(Meta, n_dtiles) == offsetof(Meta, n_dense) + 4,
              "n_dense and n_dtiles form one 8-byte word");

}  // namespace tcmis

// A row-block's round state on the tile path, kept together so that one 8-byte load
// reads both masks of a column block (bit r = row r of the block).
struct RowState {
    uint32_t alive;     // undecided rows
    uint32_t blocked;   // rows with an undecided higher-priority neighbour (this round)
};

// Everything a build or a solve reads: the configuration, the structure's arrays in
// the build workspace and the arrays of one solve's round state.  Plain data: a
// solve with a caller's scratch runs on a copy whose round-state pointers point into
// that scratch (layout_state), so the structure is only ever read by a solve.
struct GraphCore {
    // input (caller-owned device CSR)
    int64_t n = 0, nnz = 0;
    const int64_t* row_ptr = nullptr;
    const int32_t* col_idx = nullptr;

    // chosen configuration
    int path = MIS_PATH_CSR, tile = 0, reorder = MIS_REORDER_NONE, orient = 0;
    int poll_rounds = 4;
    int launch = MIS_LAUNCH_AUTO;
    bool user_keys = false;           // priorities supplied by the caller

    bool btiming = false;             // build-stage events (opts.timing = 1)
    int grid_blocks = 2048;           // persistent grid of the round kernels
    int cus = 256;                    // compute units of the device the handle was built on
    int64_t enq_rounds = 0;           // rounds enqueued since the solve began (host side)
    int coop_blocks = 0;              // grid of the cooperative round kernels (sized at build)

    // workspace (caller-owned device memory): the structure, then the handle's own
    // round state (state_off .. ws_bytes)
    char* ws = nullptr;
    size_t ws_bytes = 0;
    size_t state_off = 0;

    // round state (per solve): control block, a copy of the build's sizes and the trace
    // ring side by side (one copy brings all three back), the counter stripes
    tcmis::Ctrl* ctrl = nullptr;
    tcmis::Meta* smeta = nullptr;     // copy of *meta taken when a solve starts
    tcmis::TraceRec* trace = nullptr;
    int64_t* stripes = nullptr;       // [2][kStripes][kStripeWords] round counters

    tcmis::Meta* meta = nullptr;      // sizes the build produced (structure)
    char* scan_tmp = nullptr;         // scan scratch (int64 elements)
    char* sort_tmp = nullptr;         // radix sort scratch

    uint64_t* key = nullptr;          // priorities, input ids

    // batch (mis_build_batch): graph g owns input vertices goff[g] .. goff[g+1]-1
    int32_t count = 0;
    int64_t* goff = nullptr;          // [count+1] device copy of the offsets
    int32_t* g_rounds = nullptr;      // [count] per-graph rounds (mis_solve_batch)
    int64_t* g_in = nullptr;          // [count] per-graph set sizes

    // ---- CSR path
    int32_t* light = nullptr;         // vertices with degree <= kLightDeg (initial active list)
    int32_t* heavy = nullptr;
    int32_t* act[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    uint32_t* st = nullptr;           // per-vertex decision word: 0 or (round << 2 | code)
    uint64_t* ak = nullptr;           // alive ? key : 0
    int32_t* flag32 = nullptr;        // [n] build temporary

    // ---- tile path (new vertex order)
    int64_t nI = 0;                   // row-blocks of `tile` rows
    int64_t tile_cap = 0;             // capacity in tiles (upper bound)
    int64_t chunk_cap = 0;            // capacity of a chunk list
    int32_t* new_id = nullptr;        // input id -> new id
    int32_t* order = nullptr;         // new id -> input id
    uint64_t* sk = nullptr;           // [n] x2 order sort keys
    uint64_t* sk2 = nullptr;
    uint32_t* pl = nullptr;           // [n] x2 order sort payload
    uint32_t* pl2 = nullptr;
    int32_t* ndeg = nullptr;          // [n+1] degrees in new order -> new row pointer
    int32_t* brow = nullptr;          // [nnz/2048+2] first new row of each entry workgroup
    uint64_t* ent = nullptr;          // [nnz] x2 tile entries
    uint64_t* ent2 = nullptr;
    int32_t* hsums = nullptr;         // [nnz/2048+2] tile heads per chunk -> first tile of the chunk
    int32_t* ecnt = nullptr;          // [nnz/4096+1] kept entries per entry workgroup
    int64_t* rb_ptr = nullptr;        // [nI+1] tile range of each row-block
    int64_t* rb_chunk = nullptr;      // [nI+1] first round-1 chunk of each row-block
    int32_t* tile_col = nullptr;      // [tile_cap] column block J
    int32_t* tile_start = nullptr;    // [tile_cap] first sorted entry of each tile
    uint32_t* tile_bits = nullptr;    // [tile_cap * tile*tile/32] row masks (T=16: two rows per word)
    uint64_t* key_p = nullptr;        // [nI*tile] keys in new order, padding 0 (orient = 0)
    uint32_t* hrows = nullptr;        // [nI] rows with at least one tile entry
    uint64_t* chunks_all = nullptr;   // [chunk_cap] every row-block's chunks, row-block order
    uint64_t* chunks_r1 = nullptr;    // [nI + chunk_cap] round 1's list: row-block I's first chunk at
                                      // [I], its later chunks at nI + their index, kChunkHole elsewhere
    uint64_t* chunks[2] = {nullptr, nullptr};   // [chunk_cap] next round's chunks
    int32_t* rbl[2] = {nullptr, nullptr};       // [nI] next round's active row-blocks
    RowState* rs = nullptr;           // [nI] undecided rows and this round's blocked rows
    uint32_t* hit = nullptr;          // [nI] rows with a candidate neighbour (this round)
    uint32_t* inmask = nullptr;       // [nI] rows in the set
    int32_t* dround = nullptr;        // [nI*tile] round in which each row was decided (hybrid: [n])

    // ---- hybrid path (input order; row-block I = vertices 16I .. 16I+15)
    int dense_min = 0;                // entries per tile from which a row-block takes bit tiles (0: never)
    uint64_t seed = 1;                // default key rule's seed
    uint8_t* q8 = nullptr;            // [n] degree class floor(255 / (1 + deg)) of every vertex
    int32_t* hbrow = nullptr;         // [nnz/kHybE + 2] first row of each orientation workgroup
    int32_t* hbase = nullptr;         // [n] orientation scratch (workgroups whose rows exceed LDS)
    int32_t* hoff = nullptr;          // [n] orientation scratch
    int32_t* hcol = nullptr;          // [nnz] oriented entries: row v's are hcol[rp[v] .. rp[v] + hcnt[v])
    int32_t* hcnt = nullptr;          // [n] higher-priority neighbours of each vertex
    int32_t* dsamp = nullptr;         // [kGateSamples] the dense-block sample's candidate flags
    int32_t* dslot = nullptr;         // [nI] list slot of each dense row-block (-1: entry lists)
    int32_t* drb = nullptr;           // [nI] dense row-blocks by list slot
    int32_t* dptr = nullptr;          // [nI+1] first tile of each list slot (slot + 1: the end)
    int32_t* dcol = nullptr;          // [tile cap] column block of each dense tile
    uint32_t* dbits = nullptr;        // [tile cap * 8] 16x16 bitmaps (word w: rows 2w, 2w+1)
    uint32_t* hA = nullptr;           // [nw] undecided vertices (bitmap)
    uint32_t* hS = nullptr;           // [nw] vertices in the set (bitmap)
    int32_t* hblk = nullptr;          // [n] static handles, round 1: the first higher-priority
                                      // neighbour phase 1 met (vertices that have one)
    int32_t* hdact[2] = {nullptr, nullptr};   // dense blocks still undecided, by round parity
    const int64_t* hrp = nullptr;     // row starts of hcol (the input row pointer, or drp)

    // ---- dynamic handles (hybrid path, dyn_slack > 0): both orientations in rows of
    // their own with room for inserted edges; deleted entries read -1
    int dyn_slack = 0;
    int64_t* drp = nullptr;           // [n+1] row starts: exclusive scan of deg + slack
    int32_t* lcol = nullptr;          // [drp[n]] lower-priority neighbours
    int32_t* lcnt = nullptr;          // [n] slots used in lcol rows
    int32_t* hloff = nullptr;         // [n] orientation scratch
    uint32_t* rS = nullptr;           // [nw] repair: in the set
    uint32_t* rP = nullptr;           // [nw] repair: pending (status to recompute)
    uint32_t* rC = nullptr;           // [nw] repair: this round's candidates
    int32_t* rlist[2] = {nullptr, nullptr};   // [n] pending vertices by round parity
    int32_t* rflip = nullptr;         // [n] vertices whose status changed this round
    int32_t* rdec = nullptr;          // [n] this round's decisions
    int64_t* rcnt = nullptr;          // repair counters (see dyn.hip)
    int64_t* hflag = nullptr;         // [n] build temporary (row capacities)
};

struct mis_graph : GraphCore {
    // captured round loop (launch = graph) over the handle's own round state:
    // poll_rounds rounds and the close kernel
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    bool graph_failed = false;
    std::atomic<int64_t> solves{0};   // solves over the handle's own state (auto launch captures from the 2nd)

    std::vector<hipEvent_t> bev;      // build-stage events, recorded on the build stream

    mis_graph() = default;
    mis_graph(const mis_graph&) = delete;
    mis_graph& operator=(const mis_graph&) = delete;
    ~mis_graph() {
        if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        for (hipEvent_t e : bev) (void)hipEventDestroy(e);
    }
};

namespace tcmis {
// Records a build-stage boundary on s when the handle was built with timing.
void build_mark(mis_graph* g, hipStream_t s);

// Assigns every workspace array of g: the structure, then the handle's own round
// state (base == nullptr: only computes the size).
size_t layout(GraphCore* g, char* base);
// Assigns the arrays of one solve's round state from base (nullptr: size only);
// without the trace ring when with_trace is false.
size_t layout_state(GraphCore* g, char* base, bool with_trace = true);

// Pieces of the round loop, enqueued on `s` without synchronising it:
// solve_begin resets the round state, solve_rounds enqueues k more rounds (as the
// captured hipGraph when k == poll_rounds and graph launch is allowed) and
// solve_output writes the in/out vector in input ids.
int solve_begin(GraphCore* g, hipStream_t s);

// Option checks and defaults (host-only), the handle's configuration, and the build
// into a workspace of `need` bytes (layout() of the configured handle).
int resolve_opts(const mis_csr* csr, const mis_build_opts* opts, mis_build_opts* o, int32_t count,
                 const int64_t* offsets);
void configure_graph(GraphCore* g, const mis_csr* csr, const mis_build_opts& o, int32_t count);
int build_into(mis_graph* g, const mis_csr* csr, const mis_build_opts& o, int32_t count, const int64_t* offsets,
               char* ws, size_t need, hipStream_t s);
int solve_rounds(GraphCore* g, int64_t k, bool allow_graph, hipStream_t s, mis_graph* owner = nullptr);
int solve_output(GraphCore* g, uint8_t* in_set, hipStream_t s, bool if_done = false);
}  // namespace tcmis
