// Tile path: the rounds of Algorithm 2 over nonzero T x T bit tiles (T = 16, 32).
//
// Layout (new vertex order, row-block I = rows I*T .. I*T+T-1):
//   rb_ptr[I] .. rb_ptr[I+1]  tiles of row-block I, column block tile_col[t]
//   tile_bits                 T=16: 8 words per tile, word w = rows 2w (low 16 bits)
//                             and 2w+1 (high 16 bits); T=32: 32 words, one per row
//   alive[I]                  undecided rows of row-block I (bit r)
//   cand[I]                   (round << 32) | rows of I that are candidates in `round`
// Work is split into segments of at most kSegTiles tiles of one row-block; a
// row-block with several segments combines their partial masks with one atomic OR
// each, and the segment that finishes last completes the row-block.
//
// Candidate kernel (Phase 1, Section 3.1; Phase 1 of the paper runs on the vector
// units): for each tile of an active row-block the wave loads the row masks, ANDs
// them with the alive mask of the tile's column block and
//   orient = 0: stages the keys of the alive columns in LDS and compares each row's
//               key against the keys of its set, alive columns;
//   orient = 1: the tiles hold only edges to higher-priority neighbours, so any set,
//               alive bit blocks the row (no keys are read).
// Rows blocked anywhere are combined with a ballot; candidates = alive & ~blocked.
//
// Exclusion kernel (Phases 2 and 3, Section 3.2): N_c = A x C on the matrix cores
// as an int8 x int8 -> int32 product (exact: every count is <= the degree).  Bit
// tiles are expanded to 0/1 bytes in registers.  T=16: v_mfma_i32_16x16x64_i8
// takes four tiles of a row-block at once along K (A: lane = row, k-group = tile;
// B: the same four candidate segments, identical in all 16 columns).  T=32:
// v_mfma_i32_32x32x32_i8 takes one tile.  Tiles whose candidate segment is empty
// are skipped (the paper's early exit), and a row-block stops as soon as every
// alive non-candidate row has a candidate neighbour.  Phase 3 is fused: the wave
// that completes a row-block writes its new alive mask, its members and, if rows
// remain, its segments to the next round's active list.
#include "round.hpp"

namespace tcmis {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

struct TileArgs {
    const int32_t* seg_rb;
    const int64_t* seg_t0;
    const int64_t* seg_t1;
    const int32_t* rb_seg0;
    const int32_t* rb_nseg;
    const int32_t* tile_col;
    const uint32_t* bits;
    const uint64_t* key_p;
    uint32_t* alive;
    uint64_t* cand;
    uint32_t* inmask;
    uint32_t* acc;      // [2*nI]: candidate-phase and exclusion-phase partial masks
    uint32_t* done;     // [2*nI]
    const int32_t* seg_all;
    int32_t* seglist[2];
    int64_t nseg;
    int64_t nI;
    Ctrl* ctrl;
    TraceRec* trace;
};

template <int T>
__device__ inline uint32_t row_mask(const uint32_t* bits, int64_t t, int row) {
    if (T == 16) return (bits[t * 8 + (row >> 1)] >> ((row & 1) << 4)) & 0xFFFFu;
    return bits[t * 32 + row];
}

// rows (bit r) with any lane of that row set, from a 64-lane ballot laid out as
// lane = g*T + r
template <int T>
__device__ inline uint32_t fold_rows(uint64_t b) {
    if (T == 16) return (uint32_t)((b | (b >> 16) | (b >> 32) | (b >> 48)) & 0xFFFFull);
    return (uint32_t)((b | (b >> 32)) & 0xFFFFFFFFull);
}

__device__ inline void active_list(const TileArgs& a, int r, const int32_t** list, int64_t* n) {
    if (r == 1) { *list = a.seg_all; *n = a.nseg; }
    else { *list = a.seglist[(r - 1) & 1]; *n = a.ctrl->n_act[(r - 1) & 1][0]; }
}

// 16 bits -> 16 bytes of 0/1 (byte i = bit i)
__device__ inline v4i expand16(uint32_t x) {
    v4i o;
    o[0] = (int)(((x & 0xFu) * 0x00204081u) & 0x01010101u);
    o[1] = (int)((((x >> 4) & 0xFu) * 0x00204081u) & 0x01010101u);
    o[2] = (int)((((x >> 8) & 0xFu) * 0x00204081u) & 0x01010101u);
    o[3] = (int)((((x >> 12) & 0xFu) * 0x00204081u) & 0x01010101u);
    return o;
}

// Completes a row-block's mask: single-segment row-blocks use the wave's own mask;
// otherwise the last of the row-block's segments gets the OR of all partials.
// Returns true (in lane 0) when the caller must finalise the row-block with *total.
__device__ inline bool combine(uint32_t* acc, uint32_t* done, int64_t I, int nseg, uint32_t part, uint32_t* total) {
    if (nseg == 1) { *total = part; return true; }
    if (part) atomicOr(&acc[I], part);
    __threadfence();
    const uint32_t prev = atomicAdd(&done[I], 1u);
    if (prev != (uint32_t)nseg - 1) return false;
    __threadfence();
    *total = atomicExch(&acc[I], 0u);
    atomicExch(&done[I], 0u);
    return true;
}

template <int T, int ORIENT>
__global__ void __launch_bounds__(kBlock) k_tile_cand(TileArgs a) {
    constexpr int G = kWave / T;   // tiles per pass
    __shared__ uint64_t kst[kBlock / kWave][kWave];
    if (a.ctrl->alive == 0) return;
    const int r = a.ctrl->round + 1;
    const int32_t* list;
    int64_t nact;
    active_list(a, r, &list, &nact);
    if (blockIdx.x == 0 && threadIdx.x == 0) a.ctrl->n_act[r & 1][0] = 0;
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    const int g = lane / T, row = lane % T;
    uint64_t* kw = kst[wid];
    const int64_t nwaves = (int64_t)gridDim.x * (kBlock / kWave);
    int64_t n_cand = 0, tiles = 0, keys = 0;
    for (int64_t w = (int64_t)blockIdx.x * (kBlock / kWave) + wid; w < nact; w += nwaves) {
        const int s = list[w];
        const int64_t I = a.seg_rb[s];
        const int64_t t0 = a.seg_t0[s], t1 = a.seg_t1[s];
        const uint32_t al = a.alive[I];
        const uint64_t kr = ORIENT ? 0 : a.key_p[I * T + row];
        bool blk = false;
        uint32_t blocked = 0;
        for (int64_t tb = t0; tb < t1; tb += G) {
            const int64_t t = tb + g;
            const bool valid = t < t1;
            const int64_t J = valid ? a.tile_col[t] : 0;
            const uint32_t aJ = valid ? a.alive[J] : 0u;
            uint32_t m = valid ? (row_mask<T>(a.bits, t, row) & aJ) : 0u;
            if (ORIENT) {
                blk |= m != 0;
            } else {
                // stage the keys of the alive columns of this lane's tile
                const bool need = (aJ >> row) & 1u;
                kw[lane] = need ? a.key_p[J * T + row] : 0ull;
                keys += need;
                wave_sync_lds();
                while (m && !blk) {
                    const int c = __builtin_ctz(m);
                    m &= m - 1;
                    blk = kw[g * T + c] > kr;
                }
                wave_sync_lds();
            }
            tiles += valid && row == 0;
            blocked = fold_rows<T>(ballot(blk));
            if ((blocked & al) == al) break;
        }
        blocked = fold_rows<T>(ballot(blk));
        if (lane == 0) {
            uint32_t total;
            if (combine(a.acc, a.done, I, a.rb_nseg[I], blocked, &total)) {
                const uint32_t c = al & ~total;
                a.cand[I] = ((uint64_t)(uint32_t)r << 32) | c;
                n_cand += __popc(c);
            }
        }
    }
    wave_add(&a.ctrl->cnt_c, n_cand);
    wave_add(&a.ctrl->u[0], tiles);
    wave_add(&a.ctrl->u[1], keys);
}

template <int T>
__device__ inline uint32_t cand_of(const uint64_t* cand, int64_t J, int r) {
    const uint64_t w = cand[J];
    return (uint32_t)(w >> 32) == (uint32_t)r ? (uint32_t)w : 0u;
}

// rows with N_c > 0 from the accumulator (all B columns are equal, so any column works)
__device__ inline uint32_t hits16(const v4i& acc) {
    uint32_t h = 0;
    #pragma unroll
    for (int j = 0; j < 4; ++j) {
        // lane l holds D[4*(l/16) + j][l%16]; lanes 0, 16, 32, 48 give rows j, 4+j, 8+j, 12+j
        const uint64_t b = ballot(acc[j] > 0);
        h |= (uint32_t)((b >> 0) & 1) << j;
        h |= (uint32_t)((b >> 16) & 1) << (4 + j);
        h |= (uint32_t)((b >> 32) & 1) << (8 + j);
        h |= (uint32_t)((b >> 48) & 1) << (12 + j);
    }
    return h;
}

__device__ inline uint32_t hits32(const v16i& acc) {
    uint32_t h = 0;
    #pragma unroll
    for (int j = 0; j < 16; ++j) {
        // lane l holds D[8*(j/4) + 4*(l/32) + j%4][l%32]; lanes 0 and 32
        const uint64_t b = ballot(acc[j] > 0);
        const int r0 = 8 * (j / 4) + (j % 4);
        h |= (uint32_t)((b >> 0) & 1) << r0;
        h |= (uint32_t)((b >> 32) & 1) << (r0 + 4);
    }
    return h;
}

template <int T, int ORIENT>
__global__ void __launch_bounds__(kBlock) k_tile_excl(TileArgs a) {
    __shared__ int32_t lbuf[kBlock / kWave][kWave];
    if (a.ctrl->alive == 0) return;
    const int r = a.ctrl->round + 1;
    const int32_t* list;
    int64_t nact;
    active_list(a, r, &list, &nact);
    int32_t* next = a.seglist[r & 1];
    int64_t* next_cnt = &a.ctrl->n_act[r & 1][0];
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    int32_t* buf = lbuf[wid];
    int pend = 0;
    const int64_t nwaves = (int64_t)gridDim.x * (kBlock / kWave);
    int64_t n_out = 0, scanned = 0, mult = 0;
    for (int64_t w = (int64_t)blockIdx.x * (kBlock / kWave) + wid; w < nact; w += nwaves) {
        const int s = list[w];
        const int64_t I = a.seg_rb[s];
        const int64_t t0 = a.seg_t0[s], t1 = a.seg_t1[s];
        const uint32_t al = a.alive[I];
        const uint32_t cI = cand_of<T>(a.cand, I, r);
        const uint32_t rest = al & ~cI;     // undecided non-candidates
        uint32_t hit = 0;
        if (rest) {
            if (T == 16) {
                const int g = lane >> 4, row = lane & 15;
                v4i acc = {0, 0, 0, 0};
                int since = 0;
                for (int64_t tb = t0; tb < t1; tb += 4) {
                    const int64_t t = tb + g;
                    const bool valid = t < t1;
                    const int64_t J = valid ? a.tile_col[t] : 0;
                    const uint32_t cJ = valid ? cand_of<T>(a.cand, J, r) : 0u;
                    scanned += valid && row == 0;
                    if (!ballot(cJ != 0)) continue;      // no candidate in any of the 4 segments
                    const uint32_t m = cJ ? row_mask<16>(a.bits, t, row) : 0u;
                    mult += cJ != 0 && row == 0;
                    acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(expand16(m), expand16(cJ), acc, 0, 0, 0);
                    if (++since == 4) {
                        since = 0;
                        hit = hits16(acc);
                        if ((hit & rest) == rest) break;
                    }
                }
                hit = hits16(acc);
            } else {
                const int h = lane >> 5, row = lane & 31;
                v16i acc = {};
                int since = 0;
                for (int64_t t = t0; t < t1; ++t) {
                    const int64_t J = a.tile_col[t];
                    const uint32_t cJ = cand_of<T>(a.cand, J, r);
                    scanned += lane == 0;
                    if (!cJ) continue;
                    const uint32_t m = row_mask<32>(a.bits, t, row);
                    mult += lane == 0;
                    acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(expand16(m >> (16 * h)), expand16(cJ >> (16 * h)), acc,
                                                               0, 0, 0);
                    if (++since == 4) {
                        since = 0;
                        hit = hits32(acc);
                        if ((hit & rest) == rest) break;
                    }
                }
                hit = hits32(acc);
            }
        }
        bool keep_rb = false;
        int nseg_I = 0;
        if (lane == 0) {
            uint32_t total;
            nseg_I = a.rb_nseg[I];
            if (combine(a.acc + a.nI, a.done + a.nI, I, nseg_I, hit & rest, &total)) {
                const uint32_t out = rest & total;
                const uint32_t na = rest & ~total;
                a.alive[I] = na;
                if (cI) a.inmask[I] |= cI;
                n_out += __popc(out);
                keep_rb = na != 0;
            }
        }
        // next round's active list: single-segment row-blocks through the wave
        // buffer, longer ones directly
        nseg_I = __shfl(nseg_I, 0, kWave);
        keep_rb = __shfl((int)keep_rb, 0, kWave) != 0;
        if (keep_rb && nseg_I > 1) {
            if (lane == 0) {
                const unsigned long long p = atomicAdd((unsigned long long*)next_cnt, (unsigned long long)nseg_I);
                const int s0 = a.rb_seg0[I];
                for (int k = 0; k < nseg_I; ++k) next[p + k] = s0 + k;
            }
        } else {
            lbuf_push(buf, pend, next, next_cnt, keep_rb && lane == 0, s);
        }
    }
    lbuf_flush(buf, pend, next, next_cnt);
    wave_add(&a.ctrl->cnt_x, n_out);
    wave_add(&a.ctrl->u[2], scanned);
    wave_add(&a.ctrl->u[3], mult);
    finish_round(a.ctrl, a.trace, r);
}

__global__ void k_tile_output(const int32_t* new_id, const uint32_t* inmask, int64_t n, int tshift, uint8_t* in_set) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = new_id[v];
        in_set[v] = (uint8_t)((inmask[p >> tshift] >> (p & ((1 << tshift) - 1))) & 1u);
    }
}

TileArgs make_args(mis_graph* g) {
    TileArgs a;
    a.seg_rb = g->seg_rb; a.seg_t0 = g->seg_t0; a.seg_t1 = g->seg_t1;
    a.rb_seg0 = g->rb_seg0; a.rb_nseg = g->rb_nseg;
    a.tile_col = g->tile_col; a.bits = g->tile_bits; a.key_p = g->key_p;
    a.alive = g->alive; a.cand = g->cand; a.inmask = g->inmask; a.acc = g->acc; a.done = g->done;
    a.seg_all = g->seg_all; a.seglist[0] = g->seglist[0]; a.seglist[1] = g->seglist[1];
    a.nseg = g->nseg; a.nI = g->nI;
    a.ctrl = g->ctrl; a.trace = g->trace;
    return a;
}

template <int T, int ORIENT>
void launch_phase(mis_graph* g, int phase, hipStream_t s) {
    TileArgs a = make_args(g);
    if (phase == 0) hipLaunchKernelGGL((k_tile_cand<T, ORIENT>), dim3(g->grid_blocks), dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((k_tile_excl<T, ORIENT>), dim3(g->grid_blocks), dim3(kBlock), 0, s, a);
}

}  // namespace

int tile_init(mis_graph* g, hipStream_t s) {
    const size_t nI = (size_t)g->nI;
    TC_HIP(hipMemcpyAsync(g->alive, g->alive0, nI * 4, hipMemcpyDeviceToDevice, s));
    TC_HIP(hipMemsetAsync(g->cand, 0, nI * 8, s));
    TC_HIP(hipMemsetAsync(g->inmask, 0, nI * 4, s));
    TC_HIP(hipMemsetAsync(g->acc, 0, nI * 2 * 4, s));
    TC_HIP(hipMemsetAsync(g->done, 0, nI * 2 * 4, s));
    return MIS_OK;
}

// phase 0 = candidate kernel, 1 = exclusion kernel (which closes the round)
int tile_enqueue_phase(mis_graph* g, int phase, hipStream_t s) {
    if (g->tile == 16) {
        if (g->orient) launch_phase<16, 1>(g, phase, s); else launch_phase<16, 0>(g, phase, s);
    } else {
        if (g->orient) launch_phase<32, 1>(g, phase, s); else launch_phase<32, 0>(g, phase, s);
    }
    TC_HIP(hipGetLastError());
    return MIS_OK;
}

int tile_output(mis_graph* g, uint8_t* in_set, hipStream_t s) {
    if (g->n > 0)
        hipLaunchKernelGGL(k_tile_output, dim3(stream_grid(g->n)), dim3(kBlock), 0, s, g->new_id, g->inmask, g->n,
                           g->tile == 16 ? 4 : 5, in_set);
    TC_HIP(hipGetLastError());
    return MIS_OK;
}

}  // namespace tcmis
