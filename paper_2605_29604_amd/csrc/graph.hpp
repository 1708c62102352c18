// The opaque handle behind mis_graph and the device-side round control block.
#pragma once
#include <vector>

#include "common.hpp"

namespace tcmis {

constexpr int kLightDeg = 32;       // CSR path: thread per vertex up to this degree, wave above
constexpr int kTraceCap = 4096;     // device trace ring (rounds); the host drains it at every poll
constexpr int kSegTiles = 512;      // tile path: at most this many tiles per work segment

// Device control block of the round loop.  Every round kernel reads `round` and
// `alive` at entry; only the last workgroup of the round's final kernel writes them
// (after every other workgroup has finished), so the round loop can be enqueued or
// captured without host involvement.
struct Ctrl {
    int32_t round;          // rounds completed
    int32_t pad0;
    int64_t alive;          // undecided vertices after `round` rounds
    int64_t cnt_c;          // candidates of the round in progress
    int64_t cnt_x;          // removed neighbours of candidates in the round in progress
    int64_t n_act[2][2];    // active work items per list buffer (CSR: [light, heavy]; tile: [segments, -])
    uint32_t blocks_done;   // last-workgroup detection
    uint32_t error;         // invariant violation flags
    int64_t n_in;           // vertices in the set so far
    int64_t u[4];           // work units of the round in progress (see TraceRec)
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

}  // namespace tcmis

struct mis_graph {
    // input (caller-owned device CSR)
    int64_t n = 0, nnz = 0;
    const int64_t* row_ptr = nullptr;
    const int32_t* col_idx = nullptr;
    int device = 0;

    // chosen configuration
    int path = MIS_PATH_CSR, tile = 0, reorder = MIS_REORDER_NONE, orient = 0;
    int poll_rounds = 4;
    int grid_blocks = 2048;           // persistent grid of the round kernels

    // priorities (input ids)
    uint64_t* key = nullptr;

    // ---- CSR path
    int64_t n_light = 0, n_heavy = 0;
    int32_t* light = nullptr;         // vertices with degree <= kLightDeg (initial active list)
    int32_t* heavy = nullptr;
    int32_t* act[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    uint32_t* st = nullptr;           // per-vertex decision word: 0 or (round << 2 | code)
    uint64_t* ak = nullptr;           // alive ? key : 0

    // ---- tile path (new vertex order)
    int64_t nI = 0;                   // row-blocks of `tile` rows
    int32_t* new_id = nullptr;        // input id -> new id
    int64_t ntiles = 0;
    int64_t* rb_ptr = nullptr;        // [nI+1] tile range of each row-block
    int32_t* tile_col = nullptr;      // [ntiles] column block J
    uint32_t* tile_bits = nullptr;    // [ntiles * tile*tile/32] row masks (T=16: two rows per word)
    uint64_t* key_p = nullptr;        // [nI*tile] keys in new order, padding 0 (orient = 0)
    int64_t nseg = 0;
    int32_t* seg_rb = nullptr;        // [nseg] row-block of a segment
    int64_t* seg_t0 = nullptr;        // [nseg] first tile
    int64_t* seg_t1 = nullptr;        // [nseg] one past the last tile
    int32_t* rb_seg0 = nullptr;       // [nI] first segment of a row-block
    int32_t* rb_nseg = nullptr;       // [nI]
    uint32_t* alive0 = nullptr;       // [nI] rows that exist (initial alive mask)
    uint32_t* alive = nullptr;        // [nI] undecided rows
    uint64_t* cand = nullptr;         // [nI] (round << 32) | candidate mask
    uint32_t* inmask = nullptr;       // [nI] rows in the set
    uint32_t* acc = nullptr;          // [2*nI] partial masks of multi-segment row-blocks
    uint32_t* done = nullptr;         // [2*nI] finished segments of multi-segment row-blocks
    int32_t* seglist[2] = {nullptr, nullptr};
    int32_t* seg_all = nullptr;       // [nseg] 0..nseg-1 (initial active list)

    // ---- round control
    tcmis::Ctrl* ctrl = nullptr;      // device
    tcmis::Ctrl* h_ctrl = nullptr;    // pinned host mirror
    tcmis::TraceRec* trace = nullptr; // device ring [kTraceCap]
    tcmis::TraceRec* h_trace = nullptr;  // pinned host copy

    size_t bytes = 0;                 // device bytes owned
    std::vector<void*> owned;         // device allocations to free
};
