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
// A wave takes one segment at a time and streams its tiles 64 lanes wide: each
// lane owns one tile (T=16) or a quarter tile (T=32: rows 8k..8k+7) and loads 32
// contiguous bytes of bitmap, so a wave keeps 64 tiles of independent loads in
// flight.  Bitmaps are only read for tiles whose column block can matter (alive
// rows for Phase 1, candidate rows for Phase 2).
//
// Candidate kernel (Phase 1, Section 3.1): a row is blocked when it has a set bit
// in a column that is alive and
//   orient = 1: unconditionally (the tiles hold only edges to higher-priority
//               neighbours, so no keys are read);
//   orient = 0: whose key beats the row's key (the row keys of the segment's
//               row-block are staged in LDS once per segment, neighbour keys are
//               gathered per set alive bit).
// Blocked rows are OR-reduced across the wave; candidates = alive & ~blocked.
//
// Exclusion kernel (Phases 2 and 3, Section 3.2): N_c = A x C on the matrix cores
// as an int8 x int8 -> int32 product (exact: every count is <= the degree).  The
// tiles of an iteration whose candidate segment is non-empty (the paper's early
// exit skips the rest) are compacted into LDS, then fed to
// v_mfma_i32_16x16x64_i8 four tiles at a time (A: lane = row, k-group = tile; B:
// the four candidate segments, equal in all 16 columns) or to
// v_mfma_i32_32x32x32_i8 one 32x32 tile at a time.  Bits are expanded to 0/1
// bytes in registers.  A row-block stops as soon as every alive non-candidate row
// has a candidate neighbour.  Phase 3 is fused: the wave that completes a
// row-block writes its new alive mask, its members and, if rows remain, its
// segments to the next round's active list.
#include "round.hpp"

namespace tcmis {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kWpb = kBlock / kWave;   // waves per block

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
    uint64_t* part;     // [2*nI]: candidate-phase and exclusion-phase (count << 32 | mask) words
    const int32_t* seg_all;
    int32_t* seglist[2];
    int32_t* dround;
    const Meta* meta;
    int64_t nI;
    Ctrl* ctrl;
    TraceRec* trace;
};

template <int T>
struct Geo {
    static constexpr int kLpt = T == 16 ? 1 : 4;      // lanes per tile
    static constexpr int kTpi = kWave / kLpt;          // tiles per wave iteration
    static constexpr int kWpt = T * T / 32;            // bitmap words per tile
};

// the 8 bitmap words a lane owns: tile t, quarter k
template <int T>
__device__ inline void load8(const uint32_t* bits, int64_t t, int k, uint32_t w[8]) {
    const uint4* p = reinterpret_cast<const uint4*>(bits + t * Geo<T>::kWpt + 8 * k);
    const uint4 a = p[0], b = p[1];
    w[0] = a.x; w[1] = a.y; w[2] = a.z; w[3] = a.w;
    w[4] = b.x; w[5] = b.y; w[6] = b.z; w[7] = b.w;
}

// rows (bit r of the row-block) among the lane's words with a set bit in colmask
template <int T>
__device__ inline uint32_t rows_hit(const uint32_t w[8], uint32_t colmask, int k) {
    uint32_t r = 0;
    if (T == 16) {
        const uint32_t cm = colmask | (colmask << 16);
        #pragma unroll
        for (int j = 0; j < 8; ++j) {
            const uint32_t x = w[j] & cm;
            r |= (uint32_t)((x & 0xFFFFu) != 0) << (2 * j);
            r |= (uint32_t)((x >> 16) != 0) << (2 * j + 1);
        }
    } else {
        #pragma unroll
        for (int j = 0; j < 8; ++j) r |= (uint32_t)((w[j] & colmask) != 0) << j;
        r <<= 8 * k;
    }
    return r;
}

__device__ inline uint32_t wave_or(uint32_t x) {
    for (int off = kWave / 2; off > 0; off >>= 1) x |= (uint32_t)__shfl_xor((int)x, off, kWave);
    return x;
}

__device__ inline void active_list(const TileArgs& a, int r, const int32_t** list, int64_t* n) {
    if (r == 1) { *list = a.seg_all; *n = a.meta->nseg; }
    else { *list = a.seglist[(r - 1) & 1]; *n = a.ctrl->n_act[(r - 1) & 1][0]; }
}

__device__ inline uint32_t cand_of(const uint64_t* cand, int64_t J, int r) {
    const uint64_t w = cand[J];
    return (uint32_t)(w >> 32) == (uint32_t)r ? (uint32_t)w : 0u;
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
// otherwise each segment folds its partial mask and a completion count into one
// 64-bit word (count << 32 | mask) with compare-and-swap, and the segment that
// brings the count to nseg receives the OR of all partials and resets the word.
// One atomic word carries both, so no fence is needed between them.
__device__ inline bool combine(uint64_t* part, int64_t I, int nseg, uint32_t mine, uint32_t* total) {
    if (nseg == 1) { *total = mine; return true; }
    unsigned long long* w = (unsigned long long*)&part[I];
    unsigned long long old = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), seen;
    do {
        seen = old;
        const unsigned long long nw = ((seen >> 32) + 1) << 32 | ((uint32_t)seen | mine);
        old = atomicCAS(w, seen, nw);
    } while (old != seen);
    if ((int64_t)(seen >> 32) + 1 != nseg) return false;
    *total = (uint32_t)seen | mine;
    atomicExch(w, 0ull);
    return true;
}

template <int T, int ORIENT>
__global__ void __launch_bounds__(kBlock) k_tile_cand(TileArgs a, int ri) {
    const int r = a.ctrl->rbase + ri;   // round number (the batch base is on the device)
    using G = Geo<T>;
    __shared__ uint64_t rkeys[kWpb][32];
    open_round(a.ctrl, a.trace, r);
    const int32_t* list;
    int64_t nact;
    active_list(a, r, &list, &nact);
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    const int sub = lane / G::kLpt, k = lane % G::kLpt;
    uint64_t* rk = rkeys[wid];
    const int64_t nwaves = (int64_t)gridDim.x * kWpb;
    int64_t n_cand = 0, tiles = 0, keys = 0;
    for (int64_t w = (int64_t)blockIdx.x * kWpb + wid; w < nact; w += nwaves) {
        const int s = list[w];
        const int64_t I = a.seg_rb[s];
        const int64_t t0 = a.seg_t0[s], t1 = a.seg_t1[s];
        const uint32_t al = a.alive[I];
        if (!ORIENT) {
            wave_sync_lds();
            if (lane < T) rk[lane] = a.key_p[I * T + lane];
            wave_sync_lds();
        }
        uint32_t blocked = 0;
        for (int64_t tb = t0; tb < t1; tb += G::kTpi) {
            const int64_t t = tb + sub;
            const bool valid = t < t1;
            const int64_t J = valid ? a.tile_col[t] : 0;
            const uint32_t aJ = valid ? a.alive[J] : 0u;
            tiles += valid && k == 0;
            if (aJ) {
                uint32_t wd[8];
                load8<T>(a.bits, t, k, wd);
                if (ORIENT) {
                    blocked |= rows_hit<T>(wd, aJ, k);
                } else {
                    #pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        uint32_t x = wd[j] & (T == 16 ? (aJ | (aJ << 16)) : aJ);
                        while (x) {
                            const int b = __builtin_ctz(x);
                            x &= x - 1;
                            const int row = T == 16 ? 2 * j + (b >> 4) : 8 * k + j;
                            const int col = T == 16 ? (b & 15) : b;
                            if ((blocked >> row) & 1u) continue;
                            ++keys;
                            if (a.key_p[J * T + col] > rk[row]) blocked |= 1u << row;
                        }
                    }
                }
            }
            if ((wave_or(blocked) & al) == al) break;
        }
        blocked = wave_or(blocked);
        if (lane == 0) {
            uint32_t total;
            if (combine(a.part, I, a.rb_nseg[I], blocked, &total)) {
                const uint32_t c = al & ~total;
                a.cand[I] = ((uint64_t)(uint32_t)r << 32) | c;
                n_cand += __popc(c);
            }
        }
    }
    int64_t* cnt = a.ctrl->cnt[r & 1];
    wave_add(&cnt[0], n_cand);
    wave_add(&cnt[2], tiles);
    wave_add(&cnt[3], keys);
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

template <int T>
struct Acc;
template <>
struct Acc<16> { typedef v4i type; };
template <>
struct Acc<32> { typedef v16i type; };

template <int T, int ORIENT>
__global__ void __launch_bounds__(kBlock) k_tile_excl(TileArgs a, int ri) {
    const int r = a.ctrl->rbase + ri;   // round number (the batch base is on the device)
    using G = Geo<T>;
    __shared__ uint32_t sbits[kWpb][G::kTpi * G::kWpt];
    __shared__ uint32_t scand[kWpb][G::kTpi];
    __shared__ int32_t lbuf[kWpb][kWave];
    const int32_t* list;
    int64_t nact;
    active_list(a, r, &list, &nact);
    int32_t* next = a.seglist[r & 1];
    int64_t* next_cnt = &a.ctrl->n_act[r & 1][0];
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    const int sub = lane / G::kLpt, k = lane % G::kLpt;
    uint32_t* sb = sbits[wid];
    uint32_t* sc = scand[wid];
    int32_t* buf = lbuf[wid];
    int pend = 0;
    const int64_t nwaves = (int64_t)gridDim.x * kWpb;
    int64_t n_out = 0, scanned = 0, mult = 0;
    for (int64_t w = (int64_t)blockIdx.x * kWpb + wid; w < nact; w += nwaves) {
        const int s = list[w];
        const int64_t I = a.seg_rb[s];
        const int64_t t0 = a.seg_t0[s], t1 = a.seg_t1[s];
        const uint32_t al = a.alive[I];
        const uint32_t cI = cand_of(a.cand, I, r);
        const uint32_t rest = al & ~cI;     // undecided non-candidates
        uint32_t hit = 0;
        if (rest) {
            typename Acc<T>::type acc = {};
            for (int64_t tb = t0; tb < t1; tb += G::kTpi) {
                const int64_t t = tb + sub;
                const bool valid = t < t1;
                const int64_t J = valid ? a.tile_col[t] : 0;
                const uint32_t cJ = valid ? cand_of(a.cand, J, r) : 0u;
                scanned += valid && k == 0;
                const uint64_t heads = ballot(cJ != 0 && k == 0);
                if (!heads) continue;
                // compact the tiles with candidates into LDS
                wave_sync_lds();
                if (cJ) {
                    const int slot = __popcll(heads & ((1ull << (lane - k)) - 1ull));
                    uint32_t wd[8];
                    load8<T>(a.bits, t, k, wd);
                    uint4* dst = reinterpret_cast<uint4*>(sb + slot * G::kWpt + 8 * k);
                    dst[0] = make_uint4(wd[0], wd[1], wd[2], wd[3]);
                    dst[1] = make_uint4(wd[4], wd[5], wd[6], wd[7]);
                    if (k == 0) sc[slot] = cJ;
                }
                wave_sync_lds();
                const int ntc = __popcll(heads);
                mult += lane == 0 ? ntc : 0;
                if constexpr (T == 16) {
                    const int g = lane >> 4, row = lane & 15;
                    for (int base = 0; base < ntc; base += 4) {
                        const int sl = base + g;
                        const bool v = sl < ntc;
                        const uint32_t m = v ? (sb[sl * 8 + (row >> 1)] >> ((row & 1) << 4)) & 0xFFFFu : 0u;
                        const uint32_t c = v ? sc[sl] : 0u;
                        acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(expand16(m), expand16(c), acc, 0, 0, 0);
                    }
                    hit = hits16(acc);
                } else {
                    const int h = lane >> 5, row = lane & 31;
                    for (int sl = 0; sl < ntc; ++sl) {
                        const uint32_t m = sb[sl * 32 + row];
                        const uint32_t c = sc[sl];
                        acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(expand16(m >> (16 * h)), expand16(c >> (16 * h)),
                                                                   acc, 0, 0, 0);
                    }
                    hit = hits32(acc);
                }
                if ((hit & rest) == rest) break;
            }
        }
        bool keep_rb = false;
        int nseg_I = 0;
        uint32_t decided = 0;
        if (lane == 0) {
            uint32_t total;
            nseg_I = a.rb_nseg[I];
            if (combine(a.part + a.nI, I, nseg_I, hit & rest, &total)) {
                const uint32_t out = rest & total;
                const uint32_t na = rest & ~total;
                a.alive[I] = na;
                if (cI) a.inmask[I] |= cI;
                n_out += __popc(out);
                keep_rb = na != 0;
                decided = cI | out;
            }
        }
        // rows decided this round record the round; the next round's active list
        // takes single-segment row-blocks through the wave buffer, longer ones directly
        nseg_I = __shfl(nseg_I, 0, kWave);
        keep_rb = __shfl((int)keep_rb, 0, kWave) != 0;
        decided = (uint32_t)__shfl((int)decided, 0, kWave);
        if (lane < T && ((decided >> lane) & 1u)) a.dround[I * T + lane] = r;
        if (keep_rb && nseg_I > 1) {
            if (lane == 0) {
                const unsigned long long p = atomicAdd((unsigned long long*)next_cnt, (unsigned long long)nseg_I);
                const int s0 = a.rb_seg0[I];
                for (int q = 0; q < nseg_I; ++q) next[p + q] = s0 + q;
            }
        } else {
            lbuf_push(buf, pend, next, next_cnt, keep_rb && lane == 0, s);
        }
    }
    lbuf_flush(buf, pend, next, next_cnt);
    int64_t* cnt = a.ctrl->cnt[r & 1];
    wave_add(&cnt[1], n_out);
    wave_add(&cnt[4], scanned);
    wave_add(&cnt[5], mult);
}

__global__ void k_tile_output(const int32_t* new_id, const uint32_t* inmask, int64_t n, int tshift, uint8_t* in_set) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = new_id[v];
        in_set[v] = (uint8_t)((inmask[p >> tshift] >> (p & ((1 << tshift) - 1))) & 1u);
    }
}

__global__ void k_tile_init(const uint32_t* alive0, uint32_t* alive, uint64_t* cand, uint32_t* inmask, uint64_t* part,
                            int64_t nI) {
    for (int64_t I = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; I < nI; I += (int64_t)gridDim.x * blockDim.x) {
        alive[I] = alive0[I];
        cand[I] = 0;
        inmask[I] = 0;
        part[I] = 0;
        part[nI + I] = 0;
    }
}

TileArgs make_args(mis_graph* g) {
    TileArgs a;
    a.seg_rb = g->seg_rb; a.seg_t0 = g->seg_t0; a.seg_t1 = g->seg_t1;
    a.rb_seg0 = g->rb_seg0; a.rb_nseg = g->rb_nseg;
    a.tile_col = g->tile_col; a.bits = g->tile_bits; a.key_p = g->key_p;
    a.alive = g->alive; a.cand = g->cand; a.inmask = g->inmask; a.part = g->part;
    a.seg_all = g->seg_all; a.seglist[0] = g->seglist[0]; a.seglist[1] = g->seglist[1];
    a.dround = g->dround;
    a.meta = g->meta; a.nI = g->nI;
    a.ctrl = g->ctrl; a.trace = g->trace;
    return a;
}

template <int T, int ORIENT>
void launch_phase(mis_graph* g, int phase, int r, hipStream_t s) {
    TileArgs a = make_args(g);
    if (phase == 0) hipLaunchKernelGGL((k_tile_cand<T, ORIENT>), dim3(g->grid_blocks), dim3(kBlock), 0, s, a, r);
    else hipLaunchKernelGGL((k_tile_excl<T, ORIENT>), dim3(g->grid_blocks), dim3(kBlock), 0, s, a, r);
}

}  // namespace

int tile_init(mis_graph* g, hipStream_t s) {
    if (g->nI > 0)
        hipLaunchKernelGGL(k_tile_init, dim3(stream_grid(g->nI)), dim3(kBlock), 0, s, g->alive0, g->alive, g->cand,
                           g->inmask, g->part, g->nI);
    TC_HIP(hipGetLastError());
    return MIS_OK;
}

// phase 0 = candidate kernel, 1 = exclusion kernel (which closes the round)
int tile_enqueue_phase(mis_graph* g, int phase, int r, hipStream_t s) {
    if (g->tile == 16) {
        if (g->orient) launch_phase<16, 1>(g, phase, r, s); else launch_phase<16, 0>(g, phase, r, s);
    } else {
        if (g->orient) launch_phase<32, 1>(g, phase, r, s); else launch_phase<32, 0>(g, phase, r, s);
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
