// Tile path: the rounds of Algorithm 2 over nonzero T x T bit tiles (T = 16, 32).
//
// Layout (new vertex order, row-block I = rows I*T .. I*T+T-1):
//   tile slots                tile_col[t] column block, tile_bits bitmap; a row-block's
//                             tiles are described by its chunks, chunks_all[rb_chunk[I]
//                             .. rb_chunk[I+1]) (round 1 lists them all)
//   tile_bits                 T=16: 8 words per tile, word w = rows 2w (low 16 bits)
//                             and 2w+1 (high 16 bits); T=32: 32 words, one per row
//   rs[I] = {alive, blocked}  undecided rows of row-block I (bit r) and this round's
//                             Phase-1 mask, side by side so that one 8-byte load
//                             reads a column block's candidates
//   hit[I]                    this round's Phase-2 mask; blocked and hit are built
//                             with atomic ORs and cleared by the finalize kernel
//
// Each round is three kernels over a list of tile chunks: at most 64 tiles (T=16)
// or 16 tiles (T=32) of one row-block, described by one word (first tile, length,
// row-block).  Round 1 takes every row-block's chunks (listed once by the build),
// later rounds the chunks of row-blocks that still have undecided rows.  A wave
// takes a contiguous share of the list, so it meets a row-block's chunks one after
// another: once the row-block has nothing left to learn in the phase, its further
// chunks are skipped without touching memory.
//
//   candidate (Phase 1, Section 3.1)  blocked[I] |= rows with a set bit in an
//       undecided column; with key orientation the tiles keep only edges to
//       higher-priority neighbours, so no key is read, and in round 1 (everything
//       undecided) the blocked rows are the rows with any entry, recorded by the
//       build, so round 1 has no candidate pass over the tiles.  Without
//       orientation the neighbour's key must beat the row's key.
//   exclusion (Phase 2, Section 3.2)  N_c = A x C on the matrix cores as an int8 x
//       int8 -> int32 product (exact: every count is <= the degree).  The chunk's
//       tiles whose column block holds a candidate (C = alive & ~blocked) are
//       compacted into LDS and fed to v_mfma_i32_16x16x64_i8 four tiles at a time
//       (A: lane = row, K = the four tiles' columns; B: the four candidate vectors,
//       equal in every column) or to v_mfma_i32_32x32x32_i8 one 32x32 tile at a
//       time; bits are expanded to 0/1 bytes in registers.
//   finalize (Phase 3)  per listed row-block: candidates join the set, hit
//       non-candidates leave it, the rest stay; blocked/hit are cleared and the
//       row-block's chunks are appended to the next round's list.
//
// Every lane works on one tile (T=16) or a quarter tile (T=32: rows 8k..8k+7), so a
// wave keeps 64 independent tile loads in flight; a chunk's row masks are OR-reduced
// across the wave and applied with one atomic.
#include "round.hpp"

namespace tcmis {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kWpb = kBlock / kWave;   // waves per block

struct TileArgs {
    const int64_t* rb_chunk;
    const int32_t* tile_col;
    const uint32_t* bits;
    const uint64_t* key_p;
    const uint32_t* hrows;
    RowState* rs;
    uint32_t* hit;
    uint32_t* inmask;
    int32_t* dround;
    const uint64_t* chunks_all;
    const uint64_t* chunks_r1;
    uint64_t* chunks[2];
    int32_t* rbl[2];
    const Meta* meta;
    int64_t n;
    int64_t nI;
    Ctrl* ctrl;
    int64_t* stripes;
    TraceRec* trace;
};

template <int T>
struct Geo {
    static constexpr int kLpt = T == 16 ? 1 : 4;      // lanes per tile
    static constexpr int kTpi = kWave / kLpt;          // tiles per chunk
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

// Round r's chunk list: round 1 takes every row-block's chunks, first chunks ahead
// of later ones, with holes (built once); later rounds the list the previous
// finalize wrote.
__device__ inline void round_chunks(const TileArgs& a, int r, const uint64_t** list, int64_t* n) {
    if (r == 1) { *list = a.chunks_r1; *n = a.nI + a.meta->nchunks; }
    else { *list = a.chunks[(r - 1) & 1]; *n = a.ctrl->n_act[(r - 1) & 1][0]; }
}

// Waves take runs of kChunkRun consecutive chunks, runs dealt out cyclically: a run
// keeps a row-block's chunks together, so once the row-block has nothing left to
// learn the rest of the run is skipped from registers, while the cyclic deal spreads
// the row-blocks that must be scanned to the end over all waves.
constexpr int kChunkRun = 8;

struct Chunk {
    int64_t t0, I;
    int len;
};

__device__ inline Chunk decode(uint64_t w) {
    Chunk c;
    c.t0 = (int64_t)(w >> 33);
    c.len = (int)((w >> 27) & 63u) + 1;
    c.I = (int64_t)(w & ((1ull << 27) - 1));
    return c;
}

// lane j's 64-bit value, as a wave-uniform (scalar) value; j must be uniform
__device__ inline uint64_t lane_word(uint64_t x, int j) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, j);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), j);
    return ((uint64_t)hi << 32) | lo;
}

// A wave-uniform word through the scalar cache, which takes no vector address
// processing (the limit of the round kernels, whose tile loads and column-block
// gathers keep the address units busy).  Only for row-block masks that no wave
// writes during the pass, in the one-phase kernels: the scalar cache is refreshed
// at each launch but not at the grid barriers of the persistent kernel.
template <bool kScalar>
__device__ inline uint32_t mask_load(const uint32_t* p) {
    if constexpr (kScalar) return *(const __attribute__((address_space(4))) uint32_t*)p;
    else return *p;
}

// keeps the loads issued so far where they are (no wait is implied): a load whose
// only use sits behind a branch would otherwise be moved into the branch, after the
// loads it was meant to overlap
__device__ inline void keep_issued() { asm volatile("" ::: "memory"); }

__device__ inline uint32_t wave_or(uint32_t x) {
    for (int off = kWave / 2; off > 0; off >>= 1) x |= (uint32_t)__shfl_xor((int)x, off, kWave);
    return x;
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

template <int T, int ORIENT, bool kScalar>
__device__ void tile_cand(const TileArgs& a, int r) {
    using G = Geo<T>;
    open_round(a.ctrl, a.stripes, a.trace, r);
    if (ORIENT && r == 1) return;       // blocked = rows with any entry, set at solve start
    __shared__ uint64_t rkeys[kWpb][T];   // orient = 0: the chunk's row keys
    const uint64_t* list;
    int64_t nch;
    round_chunks(a, r, &list, &nch);
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    const int sub = lane / G::kLpt, k = lane % G::kLpt;
    uint64_t* rk = rkeys[wid];
    int64_t words = 0, bytes = 0;
    int64_t prev_I = -1;
    uint32_t prev_open = 0;
    const int64_t nwaves = (int64_t)gridDim.x * kWpb;
    const int64_t w0 = (int64_t)blockIdx.x * kWpb + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    for (int64_t cb = w0 * kChunkRun; cb < nch; cb += nwaves * kChunkRun) {
      // the wave's next run of chunk descriptors in one load
      const int64_t c1 = min(nch, cb + kChunkRun);
      const uint64_t dl = cb + lane < c1 ? list[cb + lane] : 0;
      const int nb = (int)(c1 - cb);
      words += lane == 0 ? 2 * nb : 0;
      for (int jc = 0; jc < nb; ++jc) {
        const uint64_t cw = lane_word(dl, jc);
        if (cw == kChunkHole) continue;   // an unused slot of the round-1 list
        const Chunk ch = decode(cw);
        // a row-block whose undecided rows are all blocked stays so for the rest of
        // this kernel (blocked only grows): skip its further chunks without a load
        if (ch.I == prev_I && prev_open == 0) continue;
        // lanes past the chunk's end repeat its last tile (no branch around the load)
        const bool v = sub < ch.len;
        const int64_t t = ch.t0 + min(sub, ch.len - 1);
        const uint32_t J = (uint32_t)a.tile_col[t];   // in flight with the row-block masks
        keep_issued();
        // undecided rows not yet blocked: alive is fixed during the pass, blocked is
        // read through the vector path, where other waves' ORs show up sooner
        uint32_t open = mask_load<kScalar>(&a.rs[ch.I].alive) & ~a.rs[ch.I].blocked;
        words += lane == 0 ? 2 : 0;
        if (open) {
            if (!ORIENT && ch.I != prev_I) {   // stage the row-block's keys once
                wave_sync_lds();
                if (lane < T) rk[lane] = a.key_p[ch.I * T + lane];
                bytes += lane == 0 ? 8 * T : 0;
                wave_sync_lds();
            }
            uint32_t m = 0;
            const uint32_t aJ = v ? a.rs[J].alive : 0u;
            words += k == 0 && v ? 2 : 0;
            {
                if (aJ) {
                    uint32_t wd[8];
                    load8<T>(a.bits, t, k, wd);
                    bytes += 32;
                    if (ORIENT) {
                        m = rows_hit<T>(wd, aJ, k) & open;
                    } else {
                        #pragma unroll
                        for (int j = 0; j < 8; ++j) {
                            uint32_t x = wd[j] & (T == 16 ? (aJ | (aJ << 16)) : aJ);
                            while (x) {
                                const int b = __builtin_ctz(x);
                                x &= x - 1;
                                const int row = T == 16 ? 2 * j + (b >> 4) : 8 * k + j;
                                const int col = T == 16 ? (b & 15) : b;
                                if (!((open >> row) & 1u) || ((m >> row) & 1u)) continue;
                                bytes += 8;
                                if (a.key_p[(int64_t)J * T + col] > rk[row]) m |= 1u << row;
                            }
                        }
                    }
                }
            }
            m = wave_or(m);
            if (m && lane == 0) atomicOr(&a.rs[ch.I].blocked, m);
            open &= ~m;
        }
        prev_I = ch.I;
        prev_open = open;
      }
    }
    int64_t x[2] = {words, bytes};
    block_count(a.stripes, r, {2, 3}, x);
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

template <int T, bool kScalar>
__device__ void tile_excl(const TileArgs& a, int r) {
    using G = Geo<T>;
    __shared__ uint32_t sbits[kWpb][G::kTpi * G::kWpt];
    __shared__ uint32_t scand[kWpb][G::kTpi];
    const uint64_t* list;
    int64_t nch;
    round_chunks(a, r, &list, &nch);
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    const int sub = lane / G::kLpt, k = lane % G::kLpt;
    uint32_t* sb = sbits[wid];
    uint32_t* sc = scand[wid];
    int64_t words = 0, mult = 0;
    int64_t prev_I = -1;
    uint32_t prev_rest = 0;
    const int64_t nwaves = (int64_t)gridDim.x * kWpb;
    const int64_t w0 = (int64_t)blockIdx.x * kWpb + __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    for (int64_t cb = w0 * kChunkRun; cb < nch; cb += nwaves * kChunkRun) {
      // the wave's next run of chunk descriptors in one load
      const int64_t c1 = min(nch, cb + kChunkRun);
      const uint64_t dl = cb + lane < c1 ? list[cb + lane] : 0;
      const int nb = (int)(c1 - cb);
      words += lane == 0 ? 2 * nb : 0;
      for (int jc = 0; jc < nb; ++jc) {
        const uint64_t cw = lane_word(dl, jc);
        if (cw == kChunkHole) continue;   // an unused slot of the round-1 list
        const Chunk ch = decode(cw);
        // a row-block whose undecided non-candidates all have a candidate neighbour
        // stays so for the rest of this kernel (hit only grows): skip its chunks
        if (ch.I == prev_I && prev_rest == 0) continue;
        // lanes past the chunk's end repeat its last tile (no branch around the load)
        const bool v = sub < ch.len;
        const int64_t t = ch.t0 + min(sub, ch.len - 1);
        const uint32_t J = (uint32_t)a.tile_col[t];   // in flight with the row-block masks
        keep_issued();
        // alive and blocked are fixed during the pass; hit is read through the vector
        // path, where other waves' ORs show up sooner
        uint32_t rest = mask_load<kScalar>(&a.rs[ch.I].alive) & mask_load<kScalar>(&a.rs[ch.I].blocked) &
                        ~a.hit[ch.I];
        words += lane == 0 ? 3 : 0;
        if (rest) {
            const uint2 sJ = *reinterpret_cast<const uint2*>(&a.rs[J]);
            const uint32_t cJ = v ? sJ.x & ~sJ.y : 0u;   // candidates of the column block
            words += k == 0 && v ? 3 : 0;
            const uint64_t heads = ballot(cJ != 0 && k == 0);
            if (heads) {
                // compact the tiles that meet a candidate into LDS
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
                uint32_t hit;
                if constexpr (T == 16) {
                    // four tiles per product: A = lane's row of tile g along K, B = tile g's
                    // candidate vector in every column; the sum over all groups is N_c
                    const int g = lane >> 4, row = lane & 15;
                    v4i acc = {0, 0, 0, 0};
                    for (int base = 0; base < ntc; base += 4) {
                        const int sl = base + g;
                        const bool v = sl < ntc;
                        const uint32_t m = v ? (sb[sl * 8 + (row >> 1)] >> ((row & 1) << 4)) & 0xFFFFu : 0u;
                        const uint32_t cv = v ? sc[sl] : 0u;
                        acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(expand16(m), expand16(cv), acc, 0, 0, 0);
                    }
                    hit = hits16(acc);
                } else {
                    const int h = lane >> 5, row = lane & 31;
                    v16i acc = {};
                    for (int sl = 0; sl < ntc; ++sl) {
                        const uint32_t m = sb[sl * 32 + row];
                        const uint32_t cv = sc[sl];
                        acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(expand16(m >> (16 * h)), expand16(cv >> (16 * h)),
                                                                   acc, 0, 0, 0);
                    }
                    hit = hits32(acc);
                }
                hit &= rest;
                if (hit && lane == 0) atomicOr(&a.hit[ch.I], hit);
                rest &= ~hit;
            }
        }
        prev_I = ch.I;
        prev_rest = rest;
      }
    }
    int64_t x[2] = {words, mult};
    block_count(a.stripes, r, {4, 5}, x);
}

// Phase 3 for the row-blocks of round r (round 1: all), one lane per row-block.
template <int T>
__device__ void tile_fin(const TileArgs& a, int r) {
    __shared__ int64_t spre[kWpb][kWave + 1];
    __shared__ int64_t st0[kWpb][kWave];
    __shared__ int64_t wres[2][kWpb];   // per wave: chunks and row-blocks to append, then their first slots
    const int64_t nrb = r == 1 ? a.nI : a.ctrl->n_act[(r - 1) & 1][1];
    const int32_t* list = a.rbl[(r - 1) & 1];
    uint64_t* next_ch = a.chunks[r & 1];
    int32_t* next_rb = a.rbl[r & 1];
    int64_t* next_cnt = a.ctrl->n_act[r & 1];
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    int64_t* pre = spre[wid];
    int64_t* s0 = st0[wid];
    int64_t n_cand = 0, n_out = 0, rbs = 0, written = 0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    // block-uniform trip count: the workgroup reserves list space once per pass
    for (int64_t bb = (int64_t)blockIdx.x * kBlock; bb < nrb; bb += stride) {
        const int64_t idx = bb + wid * kWave + lane;
        bool keep = false;
        int64_t I = -1, t0 = 0, t1 = 0;
        if (idx < nrb) {
            I = r == 1 ? idx : list[idx];
            const RowState st = a.rs[I];
            const uint32_t al = st.alive;
            if (al) {
                const uint32_t b = st.blocked, h = a.hit[I];
                const uint32_t c = al & ~b, out = al & b & h, na = al & b & ~h;
                a.rs[I] = RowState{na, 0u};
                if (c) a.inmask[I] |= c;
                a.hit[I] = 0;
                uint32_t dec = a.dround ? c | out : 0u;   // per-row rounds: batches only
                while (dec) {
                    const int row = __builtin_ctz(dec);
                    dec &= dec - 1;
                    a.dround[I * T + row] = r;
                }
                n_cand += __popc(c);
                n_out += __popc(out);
                ++rbs;
                if (na) {
                    keep = true;
                    t0 = a.rb_chunk[I];
                    t1 = a.rb_chunk[I + 1];
                }
            }
        }
        // the row-block and its chunks go to the next round's lists; the workgroup
        // reserves space with one atomic per list and each wave writes its chunks
        // cooperatively
        const uint64_t kb = ballot(keep);
        const int64_t nc = keep ? t1 - t0 : 0;   // the row-block's round-1 chunks
        int64_t incl = nc;
        #pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const int64_t o = __shfl_up(incl, off, kWave);
            if (lane >= off) incl += o;
        }
        const int64_t total = __shfl(incl, kWave - 1, kWave);
        if (lane == 0) {
            wres[0][wid] = total;
            wres[1][wid] = __popcll(kb);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t c = 0, n = 0;
            for (int w = 0; w < kWpb; ++w) {
                c += wres[0][w];
                n += wres[1][w];
            }
            unsigned long long c0 = 0, n0 = 0;
            if (c) c0 = atomicAdd((unsigned long long*)&next_cnt[0], (unsigned long long)c);
            if (n) n0 = atomicAdd((unsigned long long*)&next_cnt[1], (unsigned long long)n);
            for (int w = 0; w < kWpb; ++w) {
                const int64_t cw = wres[0][w], nw = wres[1][w];
                wres[0][w] = (int64_t)c0;
                wres[1][w] = (int64_t)n0;
                c0 += cw;
                n0 += nw;
            }
        }
        __syncthreads();
        const int64_t cb = wres[0][wid], rb = wres[1][wid];
        __syncthreads();   // wres is rewritten by the next pass
        if (!kb) continue;
        if (keep) next_rb[rb + __popcll(kb & lanes_below())] = (int32_t)I;
        wave_sync_lds();
        pre[lane + 1] = incl;
        if (lane == 0) pre[0] = 0;
        s0[lane] = t0;
        wave_sync_lds();
        for (int64_t q = lane; q < total; q += kWave) {
            int lo = 0, hi = kWave - 1;   // owner: last lane with pre[owner] <= q
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (pre[mid] <= q) lo = mid; else hi = mid - 1;
            }
            next_ch[cb + q] = a.chunks_all[s0[lo] + (q - pre[lo])];
        }
        written += lane == 0 ? total : 0;
        wave_sync_lds();
    }
    int64_t x[4] = {n_cand, n_out, rbs, written};
    block_count(a.stripes, r, {0, 1, 6, 7}, x);
}

// One kernel per phase; round r = the batch base on the device + ri.
template <int T, int ORIENT>
__global__ void __launch_bounds__(kBlock) k_tile_cand(TileArgs a, int ri) { tile_cand<T, ORIENT, true>(a, a.ctrl->rbase + ri); }
template <int T>
__global__ void __launch_bounds__(kBlock) k_tile_excl(TileArgs a, int ri) { tile_excl<T, true>(a, a.ctrl->rbase + ri); }
template <int T>
__global__ void __launch_bounds__(kBlock) k_tile_fin(TileArgs a, int ri) { tile_fin<T>(a, a.ctrl->rbase + ri); }

// Persistent variant: k rounds in one cooperative launch, a grid barrier after
// every phase; the last round is closed and the base advanced at the end.
template <int T, int ORIENT>
__global__ void __launch_bounds__(kBlock) k_tile_rounds(TileArgs a, int k) {
    const int rb = a.ctrl->rbase;
    for (int ri = 1; ri <= k; ++ri) {
        tile_cand<T, ORIENT, false>(a, rb + ri);
        grid_barrier(a.ctrl);
        tile_excl<T, false>(a, rb + ri);
        grid_barrier(a.ctrl);
        tile_fin<T>(a, rb + ri);
        grid_barrier(a.ctrl);
    }
    finish_rounds(a.ctrl, a.stripes, a.trace, rb, k);
}

__device__ inline uint32_t in_bit(const uint32_t* inmask, int64_t p, int tshift) {
    return (inmask[p >> tshift] >> (p & ((1 << tshift) - 1))) & 1u;
}

// With `gate`, the result is written only once every vertex is decided (the kernel
// is enqueued after each batch of rounds, so a finished solve needs no further host
// round trip).
__global__ void k_tile_output(const Ctrl* gate, const int32_t* new_id, const uint32_t* inmask, int64_t n, int tshift,
                              uint8_t* in_set) {
    if (gate && gate->alive != 0) return;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        in_set[v] = (uint8_t)in_bit(inmask, new_id[v], tshift);
}

// four vertices per thread: one 16-byte load of new ids, one 4-byte store (in_set
// 4-byte aligned); the last n % 4 vertices by the first thread
__global__ void k_tile_output4(const Ctrl* gate, const int32_t* new_id, const uint32_t* inmask, int64_t n, int tshift,
                               uint8_t* in_set) {
    if (gate && gate->alive != 0) return;
    const int64_t nq = n >> 2;
    const int64_t t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (int64_t i = t0; i < nq; i += (int64_t)gridDim.x * blockDim.x) {
        const int4 p = reinterpret_cast<const int4*>(new_id)[i];
        reinterpret_cast<uint32_t*>(in_set)[i] = in_bit(inmask, p.x, tshift) | in_bit(inmask, p.y, tshift) << 8 |
                                                 in_bit(inmask, p.z, tshift) << 16 | in_bit(inmask, p.w, tshift) << 24;
    }
    if (t0 == 0)
        for (int64_t v = nq << 2; v < n; ++v) in_set[v] = (uint8_t)in_bit(inmask, new_id[v], tshift);
}

// round state before round 1: every existing row undecided; with key orientation
// round 1's blocked rows are the rows with any entry
__global__ void k_tile_init(const uint32_t* hrows, RowState* rs, uint32_t* hit, uint32_t* inmask, int64_t n, int64_t nI,
                            int T, int orient) {
    for (int64_t I = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; I < nI; I += (int64_t)gridDim.x * blockDim.x) {
        const int64_t rows = min((int64_t)T, n - I * T);
        rs[I] = RowState{rows >= 32 ? 0xFFFFFFFFu : ((1u << rows) - 1u), orient ? hrows[I] : 0u};
        hit[I] = 0;
        inmask[I] = 0;
    }
}

TileArgs make_args(GraphCore* g) {
    TileArgs a;
    a.rb_chunk = g->rb_chunk;
    a.tile_col = g->tile_col;
    a.bits = g->tile_bits;
    a.key_p = g->key_p;
    a.hrows = g->hrows;
    a.rs = g->rs;
    a.hit = g->hit;
    a.inmask = g->inmask;
    a.dround = g->count > 0 ? g->dround : nullptr;
    a.chunks_all = g->chunks_all;
    a.chunks_r1 = g->chunks_r1;
    a.chunks[0] = g->chunks[0];
    a.chunks[1] = g->chunks[1];
    a.rbl[0] = g->rbl[0];
    a.rbl[1] = g->rbl[1];
    a.meta = g->meta;
    a.n = g->n;
    a.nI = g->nI;
    a.ctrl = g->ctrl;
    a.stripes = g->stripes;
    a.trace = g->trace;
    return a;
}

template <int T, int ORIENT>
void launch_phase(GraphCore* g, int phase, int r, hipStream_t s) {
    TileArgs a = make_args(g);
    if (phase == 0) hipLaunchKernelGGL((k_tile_cand<T, ORIENT>), dim3(g->grid_blocks), dim3(kBlock), 0, s, a, r);
    else if (phase == 1) hipLaunchKernelGGL((k_tile_excl<T>), dim3(g->grid_blocks), dim3(kBlock), 0, s, a, r);
    else hipLaunchKernelGGL((k_tile_fin<T>), dim3(g->grid_blocks), dim3(kBlock), 0, s, a, r);
}

template <int T, int ORIENT>
int launch_rounds(GraphCore* g, int k, hipStream_t s) {
    TileArgs a = make_args(g);
    return launch_cooperative((const void*)k_tile_rounds<T, ORIENT>, g, &a, k, s);
}

}  // namespace

// k rounds as one cooperative launch (see k_tile_rounds)
int tile_enqueue_rounds(GraphCore* g, int k, hipStream_t s) {
    if (g->tile == 16) return g->orient ? launch_rounds<16, 1>(g, k, s) : launch_rounds<16, 0>(g, k, s);
    return g->orient ? launch_rounds<32, 1>(g, k, s) : launch_rounds<32, 0>(g, k, s);
}

int tile_init(GraphCore* g, hipStream_t s) {
    if (g->nI > 0)
        hipLaunchKernelGGL(k_tile_init, dim3(stream_grid(g->nI)), dim3(kBlock), 0, s, g->hrows, g->rs, g->hit,
                           g->inmask, g->n, g->nI, g->tile, g->orient);
    TC_HIP(hipGetLastError());
    return MIS_OK;
}

// phase 0 = candidate kernel, 1 = exclusion kernel, 2 = finalize kernel
int tile_enqueue_phase(GraphCore* g, int phase, int r, hipStream_t s) {
    if (g->tile == 16) {
        if (g->orient) launch_phase<16, 1>(g, phase, r, s); else launch_phase<16, 0>(g, phase, r, s);
    } else {
        if (g->orient) launch_phase<32, 1>(g, phase, r, s); else launch_phase<32, 0>(g, phase, r, s);
    }
    TC_HIP(hipGetLastError());
    return MIS_OK;
}

int tile_output(GraphCore* g, uint8_t* in_set, bool if_done, hipStream_t s) {
    const int tshift = g->tile == 16 ? 4 : 5;
    const Ctrl* gate = if_done ? g->ctrl : nullptr;
    if (g->n > 0 && ((uintptr_t)in_set & 3) == 0)   // new_id is a 256-byte aligned workspace array
        hipLaunchKernelGGL(k_tile_output4, dim3(stream_grid(ceil_div(g->n, 4))), dim3(kBlock), 0, s, gate, g->new_id,
                           g->inmask, g->n, tshift, in_set);
    else if (g->n > 0)
        hipLaunchKernelGGL(k_tile_output, dim3(stream_grid(g->n)), dim3(kBlock), 0, s, gate, g->new_id, g->inmask,
                           g->n, tshift, in_set);
    TC_HIP(hipGetLastError());
    return MIS_OK;
}

}  // namespace tcmis
