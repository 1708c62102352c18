// The opaque handle behind mis_graph, its device workspace layout and the
// device-side round control block.
#pragma once
#include <type_traits>
#include <vector>

#include "common.hpp"

namespace tcmis {

constexpr int kLightDeg = 32;       // CSR path: thread per vertex up to this degree, wave above
constexpr int kTraceCap = 4096;     // device trace ring (rounds); the host drains it at every poll
constexpr int kSegTiles = 512;      // tile path: at most this many tiles per work segment

// Device control block of the round loop.  Round r's kernels take r as an
// argument and count into cnt[r & 1]; round r is closed (counters moved to the
// trace ring, `alive` and `round` advanced) by the first thread of round r+1's
// candidate kernel, or by the one-thread close kernel the host enqueues before it
// reads the block.  No workgroup ever waits for another, and no fence is needed:
// every cross-workgroup hand-over crosses a kernel boundary.
struct Ctrl {
    int32_t round;          // rounds closed
    int32_t rbase;          // rounds enqueued before the current batch (round = rbase + index in batch)
    uint32_t error;         // invariant violation flags
    int32_t pad0;
    int64_t alive;          // undecided vertices after `round` rounds
    int64_t n_in;           // vertices in the set so far
    int64_t n_act[2][2];    // active work items per list buffer (CSR: [light, heavy]; tile: [segments, -])
    int64_t cnt[2][6];      // per round parity: |C|, removed neighbours, work units u0..u3
};

// Per-round trace record in the device ring.
//   c, x, alive : |C_r|, vertices removed as neighbours of candidates, undecided after r
//   u[0..3]     : work units.  CSR path: adjacency entries read by the candidate
//                 kernel, vertices it examined, entries read by the exclusion kernel,
//                 vertices it examined.  Tile path: tiles read by the candidate kernel,
//                 neighbour keys it staged, tiles whose candidate segment the exclusion
//                 kernel examined, tiles it multiplied on the matrix cores.
struct TraceRec {
    int64_t c, x, alive, round;
    int64_t u[4];
};

// Sizes the build produces on the device (never read back during the build).
struct Meta {
    int32_t ntiles;         // nonzero tiles
    int32_t nvalid;         // adjacency entries kept in tiles
    int64_t nseg;           // work segments
    int32_t n_light;        // CSR path: vertices with degree <= kLightDeg
    int32_t pad;
};

}  // namespace tcmis

struct mis_graph {
    // input (caller-owned device CSR)
    int64_t n = 0, nnz = 0;
    const int64_t* row_ptr = nullptr;
    const int32_t* col_idx = nullptr;

    // chosen configuration
    int path = MIS_PATH_CSR, tile = 0, reorder = MIS_REORDER_NONE, orient = 0;
    int poll_rounds = 4;
    int launch = MIS_LAUNCH_AUTO;
    bool user_keys = false;           // priorities supplied by the caller

    // captured round loop (launch = graph): poll_rounds rounds and the close kernel
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    bool graph_failed = false;

    ~mis_graph() {
        if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
    }
    int grid_blocks = 2048;           // persistent grid of the round kernels

    // workspace (caller-owned device memory)
    char* ws = nullptr;
    size_t ws_bytes = 0;

    tcmis::Ctrl* ctrl = nullptr;
    tcmis::Meta* meta = nullptr;
    tcmis::TraceRec* trace = nullptr;
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
    int64_t seg_cap = 0;              // capacity in segments
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
    int32_t* tile_col = nullptr;      // [tile_cap] column block J
    int32_t* tile_row = nullptr;      // [tile_cap] row block I
    int32_t* tile_start = nullptr;    // [tile_cap] first sorted entry of each tile
    uint32_t* tile_bits = nullptr;    // [tile_cap * tile*tile/32] row masks (T=16: two rows per word)
    uint64_t* key_p = nullptr;        // [nI*tile] keys in new order, padding 0 (orient = 0)
    int64_t* segc = nullptr;          // [nI] segments per row-block -> first segment
    int32_t* seg_rb = nullptr;        // [seg_cap] row-block of a segment
    int64_t* seg_t0 = nullptr;        // [seg_cap] first tile
    int64_t* seg_t1 = nullptr;        // [seg_cap] one past the last tile
    int32_t* rb_seg0 = nullptr;       // [nI] first segment of a row-block
    int32_t* rb_nseg = nullptr;       // [nI]
    int32_t* seg_all = nullptr;       // [seg_cap] 0, 1, 2, ... (round-1 active list)
    int32_t* seglist[2] = {nullptr, nullptr};
    uint32_t* alive0 = nullptr;       // [nI] rows that exist (initial alive mask)
    uint32_t* alive = nullptr;        // [nI] undecided rows
    uint64_t* cand = nullptr;         // [nI] (round << 32) | candidate mask
    uint32_t* inmask = nullptr;       // [nI] rows in the set
    int32_t* dround = nullptr;        // [nI*tile] round in which each row was decided
    uint64_t* part = nullptr;         // [2*nI] (segments done << 32 | partial mask) of multi-segment row-blocks
};

namespace tcmis {
// Assigns every workspace array of g (base == nullptr: only computes the size).
size_t layout(mis_graph* g, char* base);

// Pieces of the round loop, enqueued on `s` without synchronising it:
// solve_begin resets the round state, solve_rounds enqueues k more rounds (as the
// captured hipGraph when k == poll_rounds and graph launch is allowed) and
// solve_output writes the in/out vector in input ids.
int solve_begin(mis_graph* g, hipStream_t s);
int solve_rounds(mis_graph* g, int64_t k, bool allow_graph, hipStream_t s);
int solve_output(mis_graph* g, uint8_t* in_set, hipStream_t s);
}  // namespace tcmis
