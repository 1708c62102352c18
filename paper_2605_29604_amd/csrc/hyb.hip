// Hybrid path: the rounds of Algorithm 2 over the edges to higher-priority
// neighbours, stored per 16-row block of the input order either as nonzero 16 x 16
// bit tiles (Section 3.2) or as entry lists (Section 3.2, "Memory Footprint and
// Representation Trade-offs": a tile only pays where it holds enough edges).
//
// Why only higher-priority neighbours.  A candidate neighbour of an undecided
// vertex always out-ranks it (a candidate beats every undecided neighbour), and
// Phase 1 only asks whether an undecided neighbour out-ranks the vertex.  So after
// round 1 both phases read only H(v) = { u in N(v) : key(u) > key(v) } and neither
// reads a key:
//   Phase 1  C(v) = alive(v) and no u in H(v) is alive
//   Phase 2  v leaves the undecided set if some u in H(v) joined the set this round
// With the in-set bitmap S, "joined this round" is simply S(u): a neighbour that
// joined in an earlier round would already have removed v.
//
// Build of a static handle (no reordering, no sort, no pass that compares every
// edge):
//   1. keys and the one-byte degree class q(v) of every vertex; the same kernel's
//      waves take a sample of 1024 16-row blocks (k_keys, dense.hpp);
//   2. dense blocks (optional; only the empty slot map unless 1% of the sample
//      qualified): a wave per block ORs a signature bit of each entry's column
//      block; a block with at least dense_min entries per estimated tile is a
//      candidate, whose entries the wave orients (priority comparisons), sorts in
//      LDS and counts in tiles; a block whose higher-priority entries average at
//      least dense_min per tile (at most 64 tiles) is written as bitmaps.
// Round 1 then reads the caller's CSR directly: Phase 1 compares each vertex's
// neighbours with it until one out-ranks it, in steps of 4, 12 and 16 entries (the
// degree class decides most pairs from the 1-byte table, a tie rebuilds the
// neighbour's hash in registers) and keeps the neighbour that blocked it; Phase 2
// tests that neighbour's S bit, else scans for a candidate neighbour; only the
// vertices still undecided after round 1 are oriented (their H rows written to
// hcol[rp[v] ..]).  On the R-MAT workload that is about a tenth of the entries a
// full orientation reads.
//
// A dynamic handle (edges inserted and deleted later) orients every edge at build
// time instead (k_orient: both orientations, with slack per row), and its round 1
// starts from the counts of higher-priority neighbours.
//
// Round r >= 2 (two kernels, a thread per 32-bit word of the alive bitmap):
//   P1  alive rows: scan H(v) for an alive neighbour (early exit); dense blocks:
//       blocked rows = H x alive on the matrix cores (int8 x int8 -> int32, exact);
//       candidates set their S bit.
//   P2  alive rows: S(v) -> IN; else scan H(v) for an S neighbour -> OUT; dense
//       blocks: N_c = H x S on the matrix cores.  Decided vertices clear their
//       alive bit; undecided dense blocks go to the next round's list.
// P1 only reads alive and writes S; P2 only reads S and writes alive; every hand-over
// crosses a kernel boundary (or a grid barrier in the persistent kernel).
#include "dense.hpp"
#include "round.hpp"

namespace tcmis {

namespace {

constexpr int kHE = 2048;                 // adjacency entries per orientation workgroup
constexpr int kHWin = 512;                // rows a workgroup stages in LDS
constexpr int kHSteps = 9;                // 2^kHSteps = kHWin
constexpr int kHLight = 32;               // rows with at most this many entries take one lane
constexpr int kP2Words = 8;               // bitmap words a wave takes in round 1's exclusion phase
constexpr int kGrp = 16;                  // entries per step of a later round's scan of an H row
constexpr int kOGrp = 8;                  // entries per step when a round-1 lane writes an H row
constexpr int kWpb = kBlock / kWave;

typedef int v4i __attribute__((ext_vector_type(4)));

__device__ inline uint32_t bit_of(const uint32_t* m, int64_t v) { return (m[v >> 5] >> (v & 31)) & 1u; }

// the 16 bits of column block J (vertices 16J .. 16J+15) of a bitmap
__device__ inline uint32_t half_of(const uint32_t* m, int64_t J) { return (m[J >> 1] >> ((J & 1) << 4)) & 0xFFFFu; }

// Adjacent lanes holding the same word index w (w < 0: none) combine their masks; the
// first lane of each run applies one atomic: AND with ~m (kClear) or OR with m.
template <bool kClear>
__device__ inline void run_apply(int64_t w, uint32_t m, uint32_t* dst) {
    const int lane = lane_id();
    #pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t mo = (uint32_t)__shfl_down((int)m, off, kWave);
        const int64_t wo = __shfl_down(w, off, kWave);
        if (lane + off < kWave && wo == w) m |= mo;
    }
    const int64_t wp = __shfl_up(w, 1, kWave);
    if ((lane == 0 || wp != w) && w >= 0 && m) {
        if (kClear) atomicAnd(&dst[w], ~m);
        else atomicOr(&dst[w], m);
    }
}

// ---------------------------------------------------------------- build

// First row of every orientation workgroup's entry range (the last slot: the row of
// the last entry), one thread per row: row v owns the workgroups whose first entry
// b * kHE falls inside it.
__global__ void k_orient_rows(const int64_t* rp, int64_t n, int64_t nnz, int64_t nblocks, int32_t* brow) {
    GRID_STRIDE(v, n) {
        const int64_t e0 = rp[v], e1 = rp[v + 1];
        if (e1 <= e0) continue;
        for (int64_t b = (e0 + kHE - 1) / kHE; b * kHE < e1; ++b) brow[b] = (int32_t)v;
        if (e0 <= nnz - 1 && nnz - 1 < e1) brow[nblocks] = (int32_t)v;
    }
}

// does column u out-rank row v?  kUserKeys: compare the keys; else the default key
// rule: the degree class decides unless it ties, then the hash of the graph-local
// id, then the id (kv is row v's whole key, so its class, hash and local id are known)
// the default rule between two vertices of the same degree class
__device__ inline bool tie_higher(int64_t u, int64_t v, uint64_t kv, uint64_t seed) {
    const int64_t lv = (int64_t)(kv & 0xFFFFFFull);
    const int64_t lu = u - (v - lv);   // same graph: same offset
    const uint32_t hu = (uint32_t)(splitmix_at(seed, (uint64_t)lu + 1) >> 32);
    const uint32_t hv = (uint32_t)(kv >> 24);
    return hu != hv ? hu > hv : lu > lv;
}

template <bool kUserKeys>
__device__ inline bool higher(int64_t u, int64_t v, uint64_t kv, const uint64_t* key, const uint8_t* q8, uint64_t seed) {
    if (kUserKeys) return key[u] > kv;
    const uint32_t qu = q8[u], qv = (uint32_t)(kv >> 56);
    if (qu != qv) return qu > qv;
    return tie_higher(u, v, kv, seed);
}

// Where the orientation writes: the higher-priority entries of row v go to
// hcol[hrp[v] + ...] (hrp = the dynamic layout's row starts), the lower-priority ones
// to lcol[hrp[v] + ...].
struct OrientOut {
    const int64_t* hrp;
    int32_t* hcol;
    int32_t* hcnt;
    int32_t* lcol;
    int32_t* lcnt;
    int32_t* g_base;    // [n] scratch of workgroups whose rows exceed LDS
    int32_t* g_off;
    int32_t* g_loff;
};

// Row bounds of a workgroup's rows relative to its range start: from LDS when they
// were staged there (wst[i] = start of row u0+i, wst[w] = end of row u1; the first
// start may be negative), else from the input row pointer.
template <bool kLds>
struct Rows {
    const int64_t* rp;
    int64_t u0, base;
    const int32_t* wst;
    __device__ int64_t start(int li) const { return kLds ? (int64_t)wst[li] : rp[u0 + li] - base; }
    __device__ int64_t stop(int li) const { return kLds ? (int64_t)wst[li + 1] : rp[u0 + li + 1] - base; }
};

// Orientation.  Workgroup b takes entries [b*kHE, (b+1)*kHE), thread t the eight
// consecutive entries b*kHE + 8t .. 8t+7 (two 16-byte column loads).  The thread
// finds the row of its first entry with a fixed-step search over the staged row
// starts and walks forward for the other seven, then issues its eight degree-class
// gathers.  The kept entries of a row piece are ranked by a workgroup prefix count
// in entry order; a row wholly inside the range is written from its row start, a
// piece of a longer row from the offset its atomic add returned.
template <bool kUserKeys, bool kLds>
__device__ void orient_body(const int64_t* rp, const int32_t* ci, const uint64_t* key, const uint8_t* q8,
                            uint64_t seed, int64_t nnz, int64_t u0, int64_t u1, const OrientOut& o, const int32_t* wst,
                            const uint64_t* wkey, int32_t* wbase, int32_t* woff, int32_t* wloff) {
    constexpr int kPer = kHE / kBlock;   // 8 consecutive entries per thread
    __shared__ int32_t wsum[kWpb];
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    const int64_t base = (int64_t)blockIdx.x * kHE;
    const int64_t end = min(nnz, base + kHE);
    const int64_t erel = end - base;     // entries of the range
    const int w = (int)(u1 - u0 + 1);
    const Rows<kLds> R{rp, u0, base, wst};
    const int64_t t0 = (int64_t)threadIdx.x * kPer;   // first entry of the thread, relative
    // columns: two 16-byte loads when the thread's eight entries are all in range and aligned
    int32_t cu[kPer];
    const int32_t* src = ci + base + t0;
    if (t0 + kPer <= erel && (((uintptr_t)src) & 15) == 0) {
        const v4i a = __builtin_nontemporal_load(reinterpret_cast<const v4i*>(src));
        const v4i b = __builtin_nontemporal_load(reinterpret_cast<const v4i*>(src) + 1);
        #pragma unroll
        for (int j = 0; j < 4; ++j) {
            cu[j] = a[j];
            cu[4 + j] = b[j];
        }
    } else {
        #pragma unroll
        for (int j = 0; j < kPer; ++j) cu[j] = ci[base + min(t0 + j, erel - 1)];
    }
    // the row of each entry
    int li[kPer];
    {
        const int64_t e0 = min(t0, erel - 1);
        int lo = 0;
        if (kLds) {
            #pragma unroll
            for (int k = kHSteps - 1; k >= 0; --k) {
                const int c = lo + (1 << k);
                const int32_t wc = wst[min(c, w - 1)];
                lo = ((c <= w - 1) & (wc <= e0)) ? c : lo;
            }
        } else {
            int64_t a = u0, b = u1;
            while (a < b) {
                const int64_t mid = (a + b + 1) >> 1;
                if (rp[mid] <= base + e0) a = mid; else b = mid - 1;
            }
            lo = (int)(a - u0);
        }
        #pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int64_t e = min(t0 + j, erel - 1);
            while (lo + 1 < w && R.start(lo + 1) <= e) ++lo;
            li[j] = lo;
        }
    }
    uint32_t keep = 0;   // bit j: entry j is kept
    #pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int64_t v = u0 + li[j];
        const uint64_t kv = kLds ? wkey[li[j]] : key[v];
        if (t0 + j < erel && higher<kUserKeys>(cu[j], v, kv, key, q8, seed)) keep |= 1u << j;
    }
    // exclusive prefix count of kept entries at the thread's first entry (entry order)
    const int cnt = __popc(keep);
    int incl = cnt;
    #pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int x = __shfl_up(incl, off, kWave);
        if (lane >= off) incl += x;
    }
    if (lane == kWave - 1) wsum[wid] = incl;
    __syncthreads();
    int pre0 = incl - cnt;
    for (int q = 0; q < wid; ++q) pre0 += wsum[q];
    auto pre = [&](int j) { return pre0 + __popc(keep & ((1u << j) - 1u)); };
    // a row piece's first entry records the prefix there
    #pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int64_t e = t0 + j;
        if (e < erel && e == max(R.start(li[j]), (int64_t)0)) {
            if (kLds) wbase[li[j]] = pre(j); else o.g_base[u0 + li[j]] = pre(j);
        }
    }
    __syncthreads();
    // a row piece's last entry: its kept count; a whole row stores it, a piece adds it
    // (and the same for the lower-priority entries of a dynamic handle)
    #pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int64_t e = t0 + j;
        if (e >= erel) continue;
        const int64_t r0 = R.start(li[j]), r1 = R.stop(li[j]);
        if (e != min(r1, erel) - 1) continue;
        const int64_t v = u0 + li[j];
        const int32_t b0 = kLds ? wbase[li[j]] : o.g_base[v];
        const int32_t c = pre(j) + (int32_t)((keep >> j) & 1u) - b0;
        const int32_t lc = (int32_t)(e + 1 - max(r0, (int64_t)0)) - c;
        const bool whole = r0 >= 0 && r1 <= erel;
        int32_t off = 0, loff = 0;
        if (whole) o.hcnt[v] = c;
        else if (c > 0) off = atomicAdd(&o.hcnt[v], c);
        if (o.lcol) {
            if (whole) o.lcnt[v] = lc;
            else if (lc > 0) loff = atomicAdd(&o.lcnt[v], lc);
        }
        if (kLds) { woff[li[j]] = off; wloff[li[j]] = loff; }
        else { o.g_off[v] = off; if (o.lcol) o.g_loff[v] = loff; }
    }
    __syncthreads();
    #pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int64_t e = t0 + j;
        const bool kept = (keep >> j) & 1u;
        if (!kept && (!o.lcol || e >= erel)) continue;
        const int64_t v = u0 + li[j];
        const int32_t b0 = kLds ? wbase[li[j]] : o.g_base[v];
        // the row's first slot: the input row start, or the dynamic layout's own
        const int64_t rs = o.hrp == rp ? (li[j] == 0 ? rp[u0] : base + R.start(li[j])) : o.hrp[v];
        if (kept) {
            const int32_t off = kLds ? woff[li[j]] : o.g_off[v];
            o.hcol[rs + off + (pre(j) - b0)] = cu[j];
        } else {
            const int32_t loff = kLds ? wloff[li[j]] : o.g_loff[v];
            const int32_t rank = (int32_t)(e - max(R.start(li[j]), (int64_t)0)) - (pre(j) - b0);
            o.lcol[rs + loff + rank] = cu[j];
        }
    }
}

template <bool kUserKeys>
__global__ void __launch_bounds__(kBlock) k_orient(const int64_t* rp, const int32_t* ci, const uint64_t* key,
                                                   const uint8_t* q8, uint64_t seed, int64_t nnz,
                                                   const int32_t* brow, OrientOut o) {
    __shared__ int32_t wst[kHWin + 1];  // row starts relative to the range (the first: <= 0), then the
                                        // last row's end (beyond the range: kHE + 1)
    __shared__ uint64_t wkey[kHWin];    // row keys
    __shared__ int32_t wbase[kHWin];    // prefix at each row piece's first entry
    __shared__ int32_t woff[kHWin];     // offset of each row piece inside its row
    __shared__ int32_t wloff[kHWin];    // the same for the lower-priority entries (dynamic handles)
    const int64_t base = (int64_t)blockIdx.x * kHE;
    const int64_t u0 = brow[blockIdx.x], u1 = brow[blockIdx.x + 1];
    const int64_t w = u1 - u0 + 1;
    if (w <= kHWin) {   // uniform over the workgroup
        for (int64_t i = threadIdx.x; i <= w; i += kBlock) {
            const int64_t r = rp[u0 + i] - base;   // i = w: the end of row u1
            // past the range: kHE + 1 (a row running past the range is not whole)
            wst[i] = (int32_t)(i == 0 ? max<int64_t>(r, INT32_MIN) : min<int64_t>(r, kHE + 1));
            if (i < w) wkey[i] = key[u0 + i];
        }
        __syncthreads();
        orient_body<kUserKeys, true>(rp, ci, key, q8, seed, nnz, u0, u1, o, wst, wkey, wbase, woff, wloff);
    } else {
        orient_body<kUserKeys, false>(rp, ci, key, q8, seed, nnz, u0, u1, o, wst, wkey, wbase, woff, wloff);
    }
}

// ---- dense blocks (the candidate test and the sample are in dense.hpp)

// the sample when the keys came from the caller (the key kernel takes it otherwise)
__global__ void __launch_bounds__(kBlock) k_dense_sample(const int64_t* rp, const int32_t* ci, int64_t n,
                                                         int64_t stride, int samples, int dense_min, int32_t* samp) {
    dense_sample(rp, ci, n, stride, samples, dense_min, samp, ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave,
                 (int64_t)gridDim.x * kWpb);
}

// Gathers block I's higher-priority entries (priority comparisons with their rows,
// lanes taking entries in turn) into sk as (column << 4 | row) keys and sorts them
// (bitonic, padded with ~0); returns their number, or 0 if there are none or more
// than kDenseCap.  Every lane of the wave calls it.
template <bool kUserKeys>
__device__ inline int dense_collect(const int64_t* rp, const int32_t* ci, const uint64_t* key, const uint8_t* q8,
                                    uint64_t seed, int64_t n, int64_t I, uint64_t* sk, int32_t* sr, uint64_t* skv,
                                    int32_t* scount) {
    const int lane = lane_id();
    const int64_t v0 = 16 * I;
    const int64_t base = rp[v0];
    wave_sync_lds();
    if (lane <= 16) sr[lane] = (int32_t)(rp[min<int64_t>(v0 + lane, n)] - base);
    if (lane < 16 && v0 + lane < n) skv[lane] = key[v0 + lane];
    if (lane == 0) *scount = 0;
    wave_sync_lds();
    const int32_t tot = sr[16];
    for (int32_t k = lane; k < tot; k += kWave) {
        int r = 0;
        while (sr[r + 1] <= k) ++r;
        const int32_t u = ci[base + k];
        if (higher<kUserKeys>(u, v0 + r, skv[r], key, q8, seed)) {
            const int32_t pos = atomicAdd(scount, 1);
            if (pos < kDenseCap) sk[pos] = ((uint64_t)(uint32_t)u << 4) | (uint64_t)r;
        }
    }
    wave_sync_lds();
    const int32_t total = *scount;
    if (total == 0 || total > kDenseCap) return 0;
    int P = 64;
    while (P < total) P <<= 1;
    for (int k = total + lane; k < P; k += kWave) sk[k] = ~0ull;
    wave_sync_lds();
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int k = lane; k < P; k += kWave) {
                const int j = k ^ stride;
                if (j > k) {
                    const uint64_t x = sk[k], y = sk[j];
                    const bool up = (k & size) == 0;
                    if ((x > y) == up) { sk[k] = y; sk[j] = x; }
                }
            }
            wave_sync_lds();
        }
    }
    return total;
}

// tiles among the sorted keys: runs of one column block (key >> 8)
__device__ inline int dense_tiles(const uint64_t* sk, int total) {
    int nt = 0;
    for (int k0 = 0; k0 < total; k0 += kWave) {
        const int k = k0 + lane_id();
        nt += __popcll(ballot(k < total && (k == 0 || (sk[k] >> 8) != (sk[k - 1] >> 8))));
    }
    return nt;
}

// The dense blocks, a chunk of kDenseChunk consecutive row-blocks per workgroup, one
// wave per block: the candidate test (block_candidate), the exact test (the block's
// higher-priority entries sorted in LDS: at most kDenseTiles tiles and at least
// dense_min entries per tile), list slots and tile ranges reserved with one 64-bit
// atomic per workgroup that found any (the list order is the order of those atomics;
// nothing depends on it), the tiles' bitmaps and column blocks, and dslot for every
// block of the chunk (-1: not dense).  When the sample found too few candidates only
// dslot is written.  The last workgroup to finish writes the end of the tile ranges.
constexpr int kDenseChunk = 128;

template <bool kUserKeys>
__global__ void __launch_bounds__(kBlock) k_dense_build(const int64_t* rp, const int32_t* ci, const uint64_t* key,
                                                        const uint8_t* q8, uint64_t seed, int64_t n, int64_t nI,
                                                        int dense_min, const int32_t* samp, int samples, Meta* meta,
                                                        int32_t* drb, int32_t* dptr, int32_t* dcol, uint32_t* dbits,
                                                        int32_t* dslot) {
    __shared__ uint64_t skey[kWpb][kDenseCap];
    __shared__ uint32_t sbits[kWpb][kDenseTiles * 8];
    __shared__ int32_t srow[kWpb][17];
    __shared__ uint64_t skv[kWpb][16];
    __shared__ int32_t scount[kWpb];
    __shared__ int32_t snt[kDenseChunk];    // tiles of the chunk's dense blocks (0: not dense)
    __shared__ int32_t sslot[kDenseChunk];  // their list slots and first tiles within the chunk
    __shared__ int32_t stile[kDenseChunk];
    __shared__ int32_t sbase[2];
    __shared__ int32_t scand[kWpb];
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    const int64_t I0 = (int64_t)blockIdx.x * kDenseChunk;
    const int nb = (int)min<int64_t>(kDenseChunk, nI - I0);
    // the sample's verdict: at least 1% of the sampled blocks are candidates
    int cand = 0;
    for (int i = threadIdx.x; i < samples; i += kBlock) cand += samp[i];
    for (int off = kWave / 2; off > 0; off >>= 1) cand += __shfl_xor(cand, off, kWave);
    if (lane == 0) scand[wid] = cand;
    __syncthreads();
    cand = 0;
    for (int q = 0; q < kWpb; ++q) cand += scand[q];
    if (blockIdx.x == 0 && threadIdx.x == 0) meta->n_dcand = cand;
    if ((int64_t)cand * 100 < samples) {
        for (int i = threadIdx.x; i < nb; i += kBlock) dslot[I0 + i] = -1;
        if (blockIdx.x == 0 && threadIdx.x == 0) dptr[0] = 0;
        return;
    }
    uint64_t* sk = skey[wid];
    for (int i = wid; i < nb; i += kWpb) {
        const int64_t I = I0 + i;
        int nt = 0;
        if (block_candidate(ci, rp[16 * I], rp[min<int64_t>(16 * I + 16, n)], dense_min)) {
            const int total = dense_collect<kUserKeys>(rp, ci, key, q8, seed, n, I, sk, srow[wid], skv[wid],
                                                       &scount[wid]);
            if (total > 0) {
                const int t = dense_tiles(sk, total);
                if (t <= kDenseTiles && (int64_t)total >= (int64_t)dense_min * t) nt = t;
            }
        }
        if (lane == 0) snt[i] = nt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int c = 0, t = 0;
        for (int i = 0; i < nb; ++i) {
            sslot[i] = snt[i] ? c : -1;
            stile[i] = t;
            c += snt[i] ? 1 : 0;
            t += snt[i];
        }
        // slots and tiles in one 64-bit atomic (n_dense and n_dtiles are adjacent,
        // the count in the low word), so that consecutive slots own consecutive tile
        // ranges and dptr[p + 1] - dptr[p] is slot p's tile count
        const unsigned long long old =
            c ? atomicAdd(reinterpret_cast<unsigned long long*>(&meta->n_dense),
                          ((unsigned long long)(uint32_t)t << 32) | (uint32_t)c)
              : 0ull;
        sbase[0] = (int32_t)(uint32_t)old;
        sbase[1] = (int32_t)(old >> 32);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nb; i += kBlock) dslot[I0 + i] = sslot[i] >= 0 ? sbase[0] + sslot[i] : -1;
    for (int i = wid; i < nb; i += kWpb) {
        if (!snt[i]) continue;
        const int64_t I = I0 + i;
        const int total = dense_collect<kUserKeys>(rp, ci, key, q8, seed, n, I, sk, srow[wid], skv[wid], &scount[wid]);
        const int32_t t0 = sbase[1] + stile[i];   // the block's first tile
        for (int k = lane; k < kDenseTiles * 8; k += kWave) sbits[wid][k] = 0;
        wave_sync_lds();
        int seen = 0;
        for (int k0 = 0; k0 < total; k0 += kWave) {
            const int k = k0 + lane;
            const bool head = k < total && (k == 0 || (sk[k] >> 8) != (sk[k - 1] >> 8));
            const uint64_t hb = ballot(head);
            if (k < total) {
                // heads at or before this lane (lane 63: all of them)
                const int t = seen + __popcll(lane == kWave - 1 ? hb : hb & ((2ull << lane) - 1)) - 1;
                const uint64_t x = sk[k];
                const int r = (int)(x & 15u);
                const int col = (int)((x >> 4) & 15u);   // column within the tile
                atomicOr(&sbits[wid][t * 8 + (r >> 1)], 1u << (((r & 1) << 4) + col));
                if (head) dcol[t0 + t] = (int32_t)(x >> 8);
            }
            seen += __popcll(hb);
        }
        wave_sync_lds();
        for (int k = lane; k < seen * 8; k += kWave) dbits[(int64_t)t0 * 8 + k] = sbits[wid][k];
        if (lane == 0) {
            const int32_t p = sbase[0] + sslot[i];
            drb[p] = (int32_t)I;
            dptr[p] = t0;
        }
        wave_sync_lds();
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();   // this workgroup's reservations and writes before its arrival
        if (atomicAdd(&meta->n_done, 1) == (int32_t)gridDim.x - 1) {
            __threadfence();
            const int32_t nd = __hip_atomic_load(&meta->n_dense, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            dptr[nd] = __hip_atomic_load(&meta->n_dtiles, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// row capacities of a dynamic handle (each orientation: its degree plus the slack)
__global__ void k_dyn_caps(const int64_t* rp, int64_t n, int slack, int64_t* cap) {
    GRID_STRIDE(v, n) cap[v] = rp[v + 1] - rp[v] + slack;
}

// ---------------------------------------------------------------- rounds

struct HybArgs {
    int64_t n;
    const int64_t* rp;        // row starts of H (the input row pointer; a dynamic handle's own)
    int32_t* hcol;            // H rows (static handles: written for the vertices round 1 leaves undecided)
    int32_t* hcnt;
    const int64_t* crp;       // the caller's CSR (round 1 of a static handle reads it)
    const int32_t* ci;
    int64_t nnz;
    const uint64_t* key;      // priorities, with the one-byte degree classes of the default rule
    const uint8_t* q8;
    uint64_t seed;
    int user_keys;
    int oriented;             // H of every vertex was built (dynamic handles)
    uint32_t* A;
    uint32_t* S;
    int32_t* blk;             // round 1: a vertex's first higher-priority neighbour (nullptr: none kept)
    const int32_t* drb;       // round 1: the dense blocks (round 1 visits every vertex otherwise)
    int32_t* dact[2];         // dense blocks still undecided, listed by round parity for the next round
    int64_t nI;               // 16-row blocks
    const int32_t* dptr;      // per list slot: first tile (slot + 1: the end)
    const int32_t* dslot;     // dense block I -> its list slot (-1: entry lists); nullptr: no dense blocks
    const int32_t* dcol;
    const uint32_t* dbits;
    const Meta* meta;
    Ctrl* ctrl;
    int64_t* stripes;
    TraceRec* trace;
    int32_t* dround;          // batches: round in which each vertex was decided
};

// does u out-rank v (kv = v's key)?
__device__ inline bool hi(const HybArgs& a, int64_t u, int64_t v, uint64_t kv) {
    return a.user_keys ? higher<true>(u, v, kv, a.key, a.q8, a.seed) : higher<false>(u, v, kv, a.key, a.q8, a.seed);
}

// the dense blocks round r visits: all of them in round 1, else those round r-1's
// exclusion kernel listed
__device__ inline void dense_list(const HybArgs& a, int r, const int32_t** L, int64_t* nl) {
    if (!a.dslot) {
        *L = nullptr;
        *nl = 0;
    } else if (r == 1) {
        *L = a.drb;
        *nl = a.meta->n_dense;
    } else {
        *L = a.dact[(r - 1) & 1];
        *nl = a.ctrl->n_act[(r - 1) & 1][2];
    }
}

// does the handle hold dense blocks (wave-uniform; dslot is all -1 when the build
// found none, so the per-vertex checks are skipped)
__device__ inline bool dense_on(const HybArgs& a) { return a.dslot && a.meta->n_dense > 0; }

// the undecided list rows of bitmap word w (x = its alive bits): the rows of dense
// blocks are masked out (their blocks are visited through the dense lists)
__device__ inline uint32_t list_rows(const HybArgs& a, bool dn, int64_t w, uint32_t x) {
    if (dn) {
        const int64_t I0 = 2 * w;   // the word's two 16-row blocks
        if (I0 < a.nI && a.dslot[I0] >= 0) x &= 0xFFFF0000u;
        if (I0 + 1 < a.nI && a.dslot[I0 + 1] >= 0) x &= 0x0000FFFFu;
    }
    return x;
}

// Does H(v) (c entries from e0) name a vertex whose bit is set in m?  The whole wave,
// 64 entries per step, early exit; every lane calls it and gets the answer; *read
// (lane 0) counts the entries loaded.
__device__ inline bool wave_scan(const HybArgs& a, int64_t e0, int32_t c, const uint32_t* m, int64_t* read) {
    const int lane = lane_id();
    int32_t k = 0;
    bool hit = false;
    for (; k < c; k += kWave) {
        const int32_t u = k + lane < c ? a.hcol[e0 + k + lane] : -1;
        if (ballot(u >= 0 && bit_of(m, u))) { hit = true; k += kWave; break; }
    }
    if (lane == 0) *read += min(k, c);
    return hit;
}

// one dense block's product H x x over its tiles (x = alive or in-set bitmap, taken
// per column block), on v_mfma_i32_16x16x64_i8: four tiles along K per instruction,
// A = lane's row of tile g, B = tile g's column-block vector in every column; bits
// expanded to 0/1 bytes in registers.  Returns the rows with a nonzero sum.  Every
// lane of the wave calls it.
__device__ inline v4i expand16(uint32_t x) {
    v4i o;
    o[0] = (int)(((x & 0xFu) * 0x00204081u) & 0x01010101u);
    o[1] = (int)((((x >> 4) & 0xFu) * 0x00204081u) & 0x01010101u);
    o[2] = (int)((((x >> 8) & 0xFu) * 0x00204081u) & 0x01010101u);
    o[3] = (int)((((x >> 12) & 0xFu) * 0x00204081u) & 0x01010101u);
    return o;
}

__device__ inline uint32_t rows_of(const v4i& acc) {
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

__device__ inline uint32_t dense_product(const HybArgs& a, int64_t t0, int nt, const uint32_t* x, uint32_t* sb,
                                         uint32_t* sx, int64_t* mult) {
    const int lane = lane_id();
    // stage the tiles that meet a nonzero column vector (compacted), and their vectors
    uint32_t xJ = 0;
    uint32_t wd[8];
    if (lane < nt) {
        xJ = half_of(x, a.dcol[t0 + lane]);
        const uint4* p = reinterpret_cast<const uint4*>(a.dbits + (t0 + lane) * 8);
        const uint4 q0 = p[0], q1 = p[1];
        wd[0] = q0.x; wd[1] = q0.y; wd[2] = q0.z; wd[3] = q0.w;
        wd[4] = q1.x; wd[5] = q1.y; wd[6] = q1.z; wd[7] = q1.w;
    }
    const uint64_t live = ballot(xJ != 0);
    const int ntc = __popcll(live);
    if (ntc == 0) return 0;
    wave_sync_lds();
    if (xJ) {
        const int slot = __popcll(live & lanes_below());
        #pragma unroll
        for (int j = 0; j < 8; ++j) sb[slot * 8 + j] = wd[j];
        sx[slot] = xJ;
    }
    wave_sync_lds();
    const int g = lane >> 4, row = lane & 15;
    v4i acc = {0, 0, 0, 0};
    for (int b = 0; b < ntc; b += 4) {
        const int sl = b + g;
        const bool v = sl < ntc;
        const uint32_t m = v ? (sb[sl * 8 + (row >> 1)] >> ((row & 1) << 4)) & 0xFFFFu : 0u;
        const uint32_t cv = v ? sx[sl] : 0u;
        acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(expand16(m), expand16(cv), acc, 0, 0, 0);
    }
    *mult += lane == 0 ? ntc : 0;
    wave_sync_lds();
    return rows_of(acc);
}

// Does a row of c entries name a vertex whose bit is set in m?  One lane scans the
// row four entries at a time (four loads, then four bit gathers in flight) and stops
// after the group that holds the first hit; *read counts the entries loaded.
// Deleted entries of a dynamic handle (-1) are skipped.
__device__ inline bool scan4(const int32_t* row, int32_t c, const uint32_t* m, int64_t* read) {
    for (int32_t k = 0; k < c; k += 4) {
        int32_t u[4];
        #pragma unroll
        for (int j = 0; j < 4; ++j) u[j] = k + j < c ? row[k + j] : -1;
        bool hit = false;
        #pragma unroll
        for (int j = 0; j < 4; ++j) hit |= u[j] >= 0 && bit_of(m, u[j]);
        *read += min(c - k, 4);
        if (hit) return true;
    }
    return false;
}

// Round 1 reads a lane's row N entries per step (N = kGrp for the scans, kOGrp for
// writing an H row): the step's loads are issued together (a 16-byte load per four
// entries that start inside the row), then its key or class gathers (one per entry
// inside the row), then its comparisons.  u[j] = row[k + j] where k + j < c (c: the
// entries the lane takes), else v itself.  A load may read up to three entries past c
// (the next rows' entries, replaced by v), so the caller makes sure that row + k + N
// stays inside the array.
typedef int32_t i4u __attribute__((ext_vector_type(4), aligned(4)));

template <int N>
__device__ inline void load_grp(const int32_t* __restrict__ row, int k, int c, int32_t v, int32_t (&u)[N]) {
    static_assert(N % 4 == 0, "a step loads whole groups of four entries");
    #pragma unroll
    for (int i = 0; i < N / 4; ++i) {
        i4u x = {v, v, v, v};
        if (k + 4 * i < c) x = *reinterpret_cast<const i4u*>(row + k + 4 * i);
        u[4 * i] = x.x;
        u[4 * i + 1] = x.y;
        u[4 * i + 2] = x.z;
        u[4 * i + 3] = x.w;
    }
    #pragma unroll
    for (int j = 0; j < N; ++j) u[j] = k + j < c ? u[j] : v;
}

// Bit j (j < N, k + j < c) is set when u[j] out-ranks v (kv = v's key): the default
// rule gathers the step's class bytes before comparing (a class tie goes to the hash);
// caller keys are gathered four at a time.
template <int N>
__device__ inline uint32_t grp_mask(const HybArgs& a, const int32_t (&u)[N], int k, int c, int32_t v, uint64_t kv,
                                    bool uk) {
    uint32_t h = 0;
    if (uk) {
        #pragma unroll
        for (int j0 = 0; j0 < N; j0 += 4) {
            uint64_t ku[4];
            #pragma unroll
            for (int j = 0; j < 4; ++j) ku[j] = k + j0 + j < c ? a.key[(uint32_t)u[j0 + j]] : 0ull;
            #pragma unroll
            for (int j = 0; j < 4; ++j) h |= (ku[j] > kv ? 1u : 0u) << (j0 + j);
        }
        return h;
    }
    uint32_t q[N];
    #pragma unroll
    for (int j = 0; j < N; ++j) q[j] = k + j < c ? a.q8[(uint32_t)u[j]] : 0u;
    const uint32_t qv = (uint32_t)(kv >> 56);
    #pragma unroll
    for (int j = 0; j < N; ++j) {
        bool b = false;
        if (k + j < c) {
            b = q[j] > qv;
            if (q[j] == qv) b = tie_higher(u[j], v, kv, a.seed);
        }
        h |= (b ? 1u : 0u) << j;
    }
    return h;
}

// Does one of the entries u[j] (k + j < c) have its bit set in m?  The step's bitmap
// words are gathered together.
template <int N>
__device__ inline bool grp_hit(const uint32_t* m, const int32_t (&u)[N], int k, int c) {
    uint32_t w[N];
    #pragma unroll
    for (int j = 0; j < N; ++j) w[j] = k + j < c ? m[(uint32_t)u[j] >> 5] : 0u;
    uint32_t h = 0;
    #pragma unroll
    for (int j = 0; j < N; ++j) h |= w[j] >> (u[j] & 31);
    return (h & 1u) != 0;
}

// One step of a round-1 scan: entries [K, K + N) of a row of c (<= kHLight) entries.
// Round 1 takes a row in steps of 4, 12 and 16 entries: most rows of low-priority
// vertices meet a higher neighbour, and most rows outside S a neighbour in S, among
// their first few entries, so a short first step saves gathers, while the longer
// later steps keep the dependent steps of the other rows few.  *ent counts the
// entries compared.
// r1_higher returns the first entry of the step that out-ranks v, or -1.
template <int K, int N>
__device__ inline int32_t r1_higher(const HybArgs& a, const int32_t* row, int c, int32_t v, uint64_t kv, bool uk,
                                    int64_t* ent) {
    int32_t u[N];
    load_grp(row, K, c, v, u);
    *ent += min(c - K, N);
    const uint32_t h = grp_mask(a, u, K, c, v, kv, uk);
    int32_t b = -1;
    #pragma unroll
    for (int j = N - 1; j >= 0; --j)
        if ((h >> j) & 1u) b = u[j];
    return b;
}

template <int K, int N>
__device__ inline bool r1_in_s(const HybArgs& a, const int32_t* row, int c, int32_t v, int64_t* ent) {
    int32_t u[N];
    load_grp(row, K, c, v, u);
    *ent += min(c - K, N);
    return grp_hit(a.S, u, K, c);
}

// Does H(v) (c <= kHLight entries at hcol + e0, e0 = rp[v]) name, from its entry k0
// on, a vertex whose bit is set in m?  Static handles: kGrp entries per step, the step's loads and bitmap gathers in
// flight together (16-byte loads may read three entries past the row, so a row ending
// within three entries of the array's end takes four at a time, as do the rows of
// dynamic handles).  *read counts the entries compared.
__device__ inline bool scan_h_from(const HybArgs& a, int32_t v, int64_t e0, int32_t c, int32_t k0, const uint32_t* m,
                                   int64_t* read) {
    if (a.oriented || e0 + c + 3 > a.nnz) return scan4(a.hcol + e0 + k0, c - k0, m, read);
    bool hit = false;
    for (int k = k0; k < c && !hit; k += kGrp) {
        int32_t u[kGrp];
        load_grp(a.hcol + e0, k, c, v, u);
        hit = grp_hit(m, u, k, c);
        *read += min(c - k, kGrp);
    }
    return hit;
}

// The undecided rows `rows` of bitmap word w in the rounds after the first, four rows
// at a time on one lane: their entry counts and row starts are loaded together, then
// the first four entries of each, then those entries' words of m, so that the four
// rows' dependent steps overlap; a row with more entries and no hit among the first
// four continues alone (scan_h_from).  Returns the rows whose H row names a vertex set
// in m.  Rows of more than kHLight entries are left to the caller in *heavy.  Deleted
// entries of a dynamic handle (-1) are skipped.  *read counts the entries compared,
// *verts the rows examined.
__device__ inline uint32_t light_hits(const HybArgs& a, int64_t w, uint32_t rows, const uint32_t* m,
                                      uint32_t* heavy, int64_t* read, int64_t* verts) {
    uint32_t hit = 0;
    for (uint32_t mm = rows; mm;) {
        int32_t v[4], c[4];
        int64_t e0[4];
        #pragma unroll
        for (int j = 0; j < 4; ++j) {
            v[j] = mm ? (int32_t)(w * 32 + __builtin_ctz(mm)) : -1;
            mm &= mm - 1u;
        }
        #pragma unroll
        for (int j = 0; j < 4; ++j) {
            c[j] = v[j] >= 0 ? a.hcnt[v[j]] : 0;
            e0[j] = v[j] >= 0 ? a.rp[v[j]] : 0;
        }
        int32_t u[4][4];
        #pragma unroll
        for (int j = 0; j < 4; ++j)
            #pragma unroll
            for (int i = 0; i < 4; ++i) u[j][i] = i < c[j] && c[j] <= kHLight ? a.hcol[e0[j] + i] : -1;
        uint32_t wd[4][4];
        #pragma unroll
        for (int j = 0; j < 4; ++j)
            #pragma unroll
            for (int i = 0; i < 4; ++i) wd[j][i] = u[j][i] >= 0 ? m[(uint32_t)u[j][i] >> 5] : 0u;
        #pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (v[j] < 0) continue;
            const uint32_t bit = 1u << (v[j] & 31);
            if (c[j] > kHLight) {
                *heavy |= bit;
                continue;
            }
            ++*verts;
            uint32_t h = 0;
            #pragma unroll
            for (int i = 0; i < 4; ++i) h |= u[j][i] >= 0 ? wd[j][i] >> (u[j][i] & 31) : 0u;
            *read += min(c[j], 4);
            bool got = (h & 1u) != 0;
            if (!got && c[j] > 4) got = scan_h_from(a, v[j], e0[j], c[j], 4, m, read);
            if (got) hit |= bit;
        }
    }
    return hit;
}

// Which rounds a build of the phase code serves: any round (the persistent kernel and
// launches over several graphs), the rounds after the first, or round 1 alone (under
// the default key rule or under caller keys).  Round 1 of a static handle reads the
// caller's CSR with many loads in flight per lane; its own builds keep that code's
// registers out of the later rounds' kernels.
enum : int { kAnyRound = 0, kLaterRounds = 1, kRound1 = 2, kRound1Keys = 3 };

// Phase 1 of round r.  The workgroup is number vb of nvb working on this graph (the
// launch's grid, or the graph's share of a launch over several graphs).
template <int kMode>
__device__ void hyb_p1(const HybArgs& a, int r, int64_t vb, int64_t nvb) {
    __shared__ uint32_t sbits[kWpb][kDenseTiles * 8];
    __shared__ uint32_t svec[kWpb][kDenseTiles];
    open_round(a.ctrl, a.stripes, a.trace, r, vb);
    if (r == 1 && a.oriented) return;   // round 1's candidates were counted when the round state was set up
    const int32_t* L[3] = {nullptr, nullptr, nullptr};
    int64_t nl[3] = {0, 0, 0};
    dense_list(a, r, &L[2], &nl[2]);
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    const int64_t nthreads = nvb * kBlock;
    const int64_t tid = vb * kBlock + threadIdx.x;
    const int64_t nwaves = nthreads / kWave, wv = tid / kWave;
    int64_t n_cand = 0, ent = 0, verts = 0, mult = 0, blocks = 0;
    const bool first = kMode >= kRound1 || (kMode == kAnyRound && r == 1);
    const bool uk = kMode == kRound1Keys || (kMode == kAnyRound && a.user_keys);
    const bool dn = dense_on(a);
    if (first) {
        // Every vertex outside the dense blocks compares its neighbours in the
        // caller's CSR with itself until one out-ranks it (every vertex is undecided).
        // Each lane takes its vertex's first kHLight entries; the longer rows still
        // undecided after them continue with the whole wave, 64 entries per step, one
        // after another (most rows meet a higher neighbour early), and so do the rows
        // of the array's last kHLight entries, from their start.
        const int64_t nr = (a.n + kWave - 1) / kWave * kWave;   // whole waves iterate together
        for (int64_t i = tid; i < nr; i += nthreads) {
            const int32_t v = (int32_t)i;
            int64_t e0 = 0, d = 0, k0 = 0;
            uint64_t kv = 0;
            bool row = i < a.n, found = false;
            if (row) {   // the row bounds, the key and the block's slot in flight together
                e0 = a.crp[v];
                d = a.crp[v + 1] - e0;
                kv = a.key[v];
                row = !(dn && a.dslot[v >> 4] >= 0);
            }
            if (row) {
                ++verts;
                if (d > 0 && e0 + kHLight <= a.nnz) {
                    const int c = (int)min<int64_t>(d, kHLight);
                    const int32_t* row = a.ci + e0;
                    int32_t b = r1_higher<0, 4>(a, row, c, v, kv, uk, &ent);
                    if (b < 0 && c > 4) b = r1_higher<4, 12>(a, row, c, v, kv, uk, &ent);
                    if (b < 0 && c > 16) b = r1_higher<16, 16>(a, row, c, v, kv, uk, &ent);
                    found = b >= 0;
                    if (found && a.blk) a.blk[v] = b;   // phase 2 looks at it first
                    k0 = kHLight;
                }
            }
            const bool cont = row && !found && d > k0;
            int64_t w = -1;
            uint32_t m = 0;
            if (row && !found && !cont) { w = v >> 5; m = 1u << (v & 31); ++n_cand; }
            run_apply<false>(w, m, a.S);
            uint64_t hv = ballot(cont);
            while (hv) {
                const int l = __builtin_ctzll(hv);
                hv &= hv - 1;
                const int32_t vh = __shfl(v, l, kWave);
                const int64_t e0h = __shfl(e0, l, kWave), dh = __shfl(d, l, kWave), k0h = __shfl(k0, l, kWave);
                const uint64_t kvh = __shfl(kv, l, kWave);
                bool blocked = false;
                int64_t k = k0h;
                for (; k < dh; k += kWave) {
                    const int32_t u = k + lane < dh ? a.ci[e0h + k + lane] : -1;
                    const uint64_t bm = ballot(u >= 0 && hi(a, u, vh, kvh));
                    if (bm) {
                        blocked = true;
                        const int32_t ub = __shfl(u, __builtin_ctzll(bm), kWave);
                        if (lane == 0 && a.blk) a.blk[vh] = ub;
                        k += kWave;
                        break;
                    }
                }
                if (lane == 0) {
                    ent += min(k, dh) - k0h;
                    if (!blocked) { atomicOr(&a.S[vh >> 5], 1u << (vh & 31)); ++n_cand; }
                }
            }
        }
    } else if (kMode < kRound1) {
        // Undecided rows outside the dense blocks, a thread per bitmap word (32
        // vertices): rows of at most kHLight entries scan H(v) for an alive neighbour
        // (early exit); the longer rows of a wave's words then take the whole wave, one
        // after another.  Candidates set their S bits, one atomic per word.
        const int64_t nwords = (a.n + 31) >> 5;
        const int64_t nwr = (nwords + kWave - 1) / kWave * kWave;   // whole waves iterate together
        for (int64_t w = tid; w < nwr; w += nthreads) {
            const uint32_t rows = w < nwords ? list_rows(a, dn, w, a.A[w]) : 0u;
            uint32_t heavy = 0;
            const uint32_t met = light_hits(a, w, rows, a.A, &heavy, &ent, &verts);   // blocked rows
            uint32_t cand = rows & ~heavy & ~met;
            for (uint64_t hb = ballot(heavy != 0); hb; hb = ballot(heavy != 0)) {
                const int l = __builtin_ctzll(hb);
                const int b = __builtin_ctz(__shfl(heavy, l, kWave));
                const int32_t v = (int32_t)(__shfl(w, l, kWave) * 32 + b);
                const bool blocked = wave_scan(a, a.rp[v], a.hcnt[v], a.A, &ent);
                if (lane == 0) ++verts;
                if (lane == l) {
                    heavy &= ~(1u << b);
                    if (!blocked) cand |= 1u << b;
                }
            }
            if (cand) {
                atomicOr(&a.S[w], cand);
                n_cand += __popc(cand);
            }
        }
    }
    // dense blocks: blocked rows = H x alive
    for (int64_t i = wv; i < nl[2]; i += nwaves) {
        const int32_t I = L[2][i];
        const int32_t s = a.dslot[I];
        const int64_t t0 = a.dptr[s];
        const int nt = a.dptr[s + 1] - (int)t0;
        const uint32_t al = half_of(a.A, I);
        const uint32_t blk = dense_product(a, t0, nt, a.A, sbits[wid], svec[wid], &mult);
        const uint32_t c = al & ~blk;
        if (lane == 0) {
            ++blocks;
            if (c) { atomicOr(&a.S[I >> 1], c << ((I & 1) << 4)); n_cand += __popc(c); }
        }
    }
    int64_t x[5] = {n_cand, ent, verts, mult, blocks};
    block_count(a.stripes, r, {0, 2, 3, 6, 8}, x, vb);
}

// Phases 2 and 3 of round r: retire candidates, remove their neighbours, list the rest.
template <int kMode>
__device__ void hyb_p2(const HybArgs& a, int r, int64_t vb, int64_t nvb) {
    __shared__ int32_t lbuf[kWpb][kWave];
    __shared__ uint32_t sbits[kWpb][kDenseTiles * 8];
    __shared__ uint32_t svec[kWpb][kDenseTiles];
    const int32_t* DL = nullptr;
    int64_t ndl = 0;
    dense_list(a, r, &DL, &ndl);
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    int pend = 0;
    int32_t* dnext = a.dact[r & 1];
    int64_t* dcnt = &a.ctrl->n_act[r & 1][2];
    const int64_t nthreads = nvb * kBlock;
    const int64_t tid = vb * kBlock + threadIdx.x;
    const int64_t nwaves = nthreads / kWave, wv = tid / kWave;
    int64_t n_out = 0, ent = 0, verts = 0, mult = 0, blocks = 0;
    const bool first = kMode >= kRound1 || (kMode == kAnyRound && r == 1);
    const bool uk = kMode == kRound1Keys || (kMode == kAnyRound && a.user_keys);
    const bool dn = dense_on(a);
    if (first && !a.oriented) {
        // Every vertex outside the dense blocks: a candidate of round 1 joins the set;
        // any other scans its row of the caller's CSR for a candidate (a candidate
        // neighbour always out-ranks it) and leaves on the first.  A vertex with none
        // stays undecided: its H row is written now, for the later rounds (round 1 is
        // the only time its whole row is compared).  A wave takes kP2Words bitmap words
        // (their candidates need no work) and packs the other vertices onto its lanes,
        // one each: a lane scans its vertex's first kHLight entries; longer rows with
        // no candidate among them, and the rows of the array's last kHLight entries,
        // continue with the whole wave, one after another.  The decided vertices of the
        // words collect in LDS; one atomic per word clears their alive bits.
        __shared__ uint32_t sdec[kWpb][kP2Words];
        const int64_t nwords = (a.n + 31) >> 5;
        const int64_t ngroups = (nwords + kP2Words - 1) / kP2Words;
        for (int64_t gi = wv; gi < ngroups; gi += nwaves) {
            const int64_t w0 = gi * kP2Words;
            const bool own = lane < kP2Words && w0 + lane < nwords;   // lane k < kP2Words: word w0 + k
            const uint32_t rows = own ? list_rows(a, dn, w0 + lane, a.A[w0 + lane]) : 0u;
            const uint32_t sw = own ? a.S[w0 + lane] : 0u;
            if (lane < kP2Words) sdec[wid][lane] = 0;
            // lanes k < kP2Words: the word's vertices outside S, and how many come
            // before them in the group
            const uint32_t nc = rows & ~sw;
            int incl = __popc(nc);
            #pragma unroll
            for (int sh = 1; sh < kP2Words; sh <<= 1) {
                const int y = __shfl_up(incl, sh, kWave);
                if (lane >= sh) incl += y;
            }
            const int excl = incl - __popc(nc);
            const int total = __builtin_amdgcn_readlane(incl, kP2Words - 1);
            wave_sync_lds();
            for (int p0 = 0; p0 < total; p0 += kWave) {
                // the j-th vertex outside S among the group's rows: word k, then the bit
                const int j = p0 + lane;
                const bool act = j < total;
                int k = 0;
                #pragma unroll
                for (int kk = 1; kk < kP2Words; ++kk) k += j >= __builtin_amdgcn_readlane(excl, kk) ? 1 : 0;
                uint32_t x = (uint32_t)__shfl((int)nc, k, kWave);
                uint32_t rank = (uint32_t)(j - __shfl(excl, k, kWave));
                int pos = 0;   // bit of x with `rank` set bits below it
                #pragma unroll
                for (int sh = 16; sh > 0; sh >>= 1) {
                    const uint32_t c = __popc(x & ((1u << sh) - 1u));
                    if (rank >= c) { rank -= c; x >>= sh; pos += sh; }
                }
                const int32_t v = (int32_t)((w0 + k) * 32 + pos);
                int64_t e0 = 0, d = 0, k0 = 0;
                bool hit = false;
                if (act) {   // d >= 1: a vertex without neighbours is a candidate
                    // the higher-priority neighbour phase 1 met first is most often a
                    // candidate: its S bit alone decides, with no row read
                    const int32_t blk = a.blk ? a.blk[v] : -1;
                    e0 = a.crp[v];
                    d = a.crp[v + 1] - e0;
                    ++verts;
                    hit = blk >= 0 && bit_of(a.S, blk);
                    if (!hit && e0 + kHLight <= a.nnz) {
                        const int c = (int)min<int64_t>(d, kHLight);
                        const int32_t* row = a.ci + e0;
                        hit = r1_in_s<0, 4>(a, row, c, v, &ent);
                        if (!hit && c > 4) hit = r1_in_s<4, 12>(a, row, c, v, &ent);
                        if (!hit && c > 16) hit = r1_in_s<16, 16>(a, row, c, v, &ent);
                        if (!hit && d <= kHLight) {   // undecided: write H(v)
                            const uint64_t kv = a.key[v];
                            int32_t* __restrict__ out = a.hcol + a.rp[v];
                            int32_t m = 0;
                            #pragma nounroll
                            for (int k = 0; k < c; k += kOGrp) {
                                int32_t u[kOGrp];
                                load_grp(a.ci + e0, k, c, v, u);
                                const uint32_t keep = grp_mask(a, u, k, c, v, kv, uk);
                                #pragma unroll
                                for (int j = 0; j < kOGrp; ++j)
                                    if ((keep >> j) & 1u) out[m++] = u[j];
                            }
                            a.hcnt[v] = m;
                            ent += d;
                        }
                        k0 = kHLight;
                    }
                    if (hit) atomicOr(&sdec[wid][k], 1u << (v & 31));
                }
                const bool cont = act && !hit && d > k0;
                for (uint64_t hv = ballot(cont); hv; hv &= hv - 1) {
                    const int l = __builtin_ctzll(hv);
                    const int32_t vh = __shfl(v, l, kWave);
                    const int64_t e0h = __shfl(e0, l, kWave), dh = __shfl(d, l, kWave), k0h = __shfl(k0, l, kWave);
                    bool hit2 = false;
                    int64_t kk = k0h;
                    for (; kk < dh; kk += kWave) {
                        const int32_t u = kk + lane < dh ? a.ci[e0h + kk + lane] : -1;
                        if (ballot(u >= 0 && bit_of(a.S, u))) { hit2 = true; kk += kWave; break; }
                    }
                    if (lane == 0) ent += min(kk, dh) - k0h;
                    if (hit2) {
                        if (lane == 0) atomicOr(&sdec[wid][(vh >> 5) - w0], 1u << (vh & 31));
                    } else {
                        // H(vh), ballot-compacted 64 entries at a time
                        const uint64_t kvh = a.key[vh];
                        int32_t* out = a.hcol + a.rp[vh];
                        int32_t c = 0;
                        for (int64_t k2 = 0; k2 < dh; k2 += kWave) {
                            const int32_t u = k2 + lane < dh ? a.ci[e0h + k2 + lane] : -1;
                            const bool h = u >= 0 && hi(a, u, vh, kvh);
                            const uint64_t mk = ballot(h);
                            if (h) out[c + __popcll(mk & lanes_below())] = u;
                            c += __popcll(mk);
                        }
                        if (lane == 0) { a.hcnt[vh] = c; ent += dh; }
                    }
                }
            }
            wave_sync_lds();
            if (own) {
                const uint32_t hits = sdec[wid][lane];
                const uint32_t dec = (rows & sw) | hits;
                if (dec) atomicAnd(&a.A[w0 + lane], ~dec);
                n_out += __popc(hits);
                if (a.dround)
                    for (uint32_t mm = dec; mm; mm &= mm - 1) a.dround[(w0 + lane) * 32 + __builtin_ctz(mm)] = r;
            }
            wave_sync_lds();   // sdec is cleared for the next group only after every lane read it
        }
    } else if (first) {
        // Dynamic handles (H of every vertex built): a vertex without a higher-priority
        // neighbour is a candidate and already in the set (it was never undecided);
        // any other leaves if one of its higher-priority neighbours is a candidate.
        // Light rows take a lane each; the heavy rows of a wave's 64 vertices are then
        // scanned by the whole wave, one after another.
        const int64_t nr = (a.n + kWave - 1) / kWave * kWave;   // whole waves iterate together
        for (int64_t i = tid; i < nr; i += nthreads) {
            const int32_t v = (int32_t)i;
            const bool valid = i < a.n;
            const int32_t c = valid ? a.hcnt[v] : 0;
            const bool listed = valid && c > 0 && !(dn && a.dslot[v >> 4] >= 0);
            const bool light = listed && c <= kHLight;
            int64_t w = -1;
            uint32_t m = 0;
            if (light) {
                const bool hit = scan4(a.hcol + a.rp[v], c, a.S, &ent);
                ++verts;
                if (hit) {
                    w = v >> 5; m = 1u << (v & 31); ++n_out;
                    if (a.dround) a.dround[v] = r;
                }
            }
            run_apply<true>(w, m, a.A);
            for (uint64_t hv = ballot(listed && !light); hv; hv &= hv - 1) {
                const int l = __builtin_ctzll(hv);
                const int32_t vh = __shfl(v, l, kWave);
                const bool hit = wave_scan(a, a.rp[vh], a.hcnt[vh], a.S, &ent);
                if (lane == 0) {
                    ++verts;
                    if (hit) {
                        atomicAnd(&a.A[vh >> 5], ~(1u << (vh & 31)));
                        ++n_out;
                        if (a.dround) a.dround[vh] = r;
                    }
                }
            }
        }
    } else if (kMode < kRound1) {
        // Undecided rows outside the dense blocks, a thread per bitmap word:
        // candidates retire; every other row scans H(v) for a candidate (rows of at
        // most kHLight entries on their lane, longer ones with the whole wave) and
        // leaves on the first.  One atomic per word clears the decided rows.
        const int64_t nwords = (a.n + 31) >> 5;
        const int64_t nwr = (nwords + kWave - 1) / kWave * kWave;   // whole waves iterate together
        for (int64_t w = tid; w < nwr; w += nthreads) {
            const uint32_t rows = w < nwords ? list_rows(a, dn, w, a.A[w]) : 0u;
            const uint32_t sw = rows ? a.S[w] : 0u;
            uint32_t heavy = 0;
            const uint32_t out = light_hits(a, w, rows & ~sw, a.S, &heavy, &ent, &verts);
            uint32_t dec = (rows & sw) | out;
            n_out += __popc(out);
            for (uint64_t hb = ballot(heavy != 0); hb; hb = ballot(heavy != 0)) {
                const int l = __builtin_ctzll(hb);
                const int b = __builtin_ctz(__shfl(heavy, l, kWave));
                const int32_t v = (int32_t)(__shfl(w, l, kWave) * 32 + b);
                const bool hit = wave_scan(a, a.rp[v], a.hcnt[v], a.S, &ent);
                if (lane == 0) ++verts;
                if (lane == l) {
                    heavy &= ~(1u << b);
                    if (hit) { dec |= 1u << b; ++n_out; }
                }
            }
            if (dec) {
                atomicAnd(&a.A[w], ~dec);
                if (a.dround)
                    for (uint32_t mm = dec; mm; mm &= mm - 1) a.dround[w * 32 + __builtin_ctz(mm)] = r;
            }
        }
    }
    for (int64_t i = wv; i < ndl; i += nwaves) {
        const int32_t I = DL[i];
        const int32_t s = a.dslot[I];
        const int64_t t0 = a.dptr[s];
        const int nt = a.dptr[s + 1] - (int)t0;
        const uint32_t al = half_of(a.A, I), in = al & half_of(a.S, I);
        const uint32_t hit = dense_product(a, t0, nt, a.S, sbits[wid], svec[wid], &mult);
        const uint32_t out = al & ~in & hit, dec = in | out;
        if (lane == 0) {
            ++blocks;
            if (dec) atomicAnd(&a.A[I >> 1], ~(dec << ((I & 1) << 4)));
            n_out += __popc(out);
        }
        if (a.dround && lane < 16 && ((dec >> lane) & 1u)) a.dround[I * 16 + lane] = r;
        lbuf_push(lbuf[wid], pend, dnext, dcnt, lane == 0 && (al & ~dec) != 0, I);
    }
    lbuf_flush(lbuf[wid], pend, dnext, dcnt);
    int64_t x[5] = {n_out, ent, verts, mult, blocks};
    block_count(a.stripes, r, {1, 4, 5, 7, 9}, x, vb);
}

template <int kMode>
__global__ void __launch_bounds__(kBlock) k_hyb_p1(HybArgs a, int ri) {
    hyb_p1<kMode>(a, a.ctrl->rbase + ri, blockIdx.x, gridDim.x);
}
template <int kMode>
__global__ void __launch_bounds__(kBlock) k_hyb_p2(HybArgs a, int ri) {
    hyb_p2<kMode>(a, a.ctrl->rbase + ri, blockIdx.x, gridDim.x);
}

// Persistent variant: k rounds in one cooperative launch, a grid barrier after every
// phase; the last round is closed and the base advanced at the end.
__global__ void __launch_bounds__(kBlock) k_hyb_rounds(HybArgs a, int k) {
    const int rb = a.ctrl->rbase;
    for (int ri = 1; ri <= k; ++ri) {
        hyb_p1<kAnyRound>(a, rb + ri, blockIdx.x, gridDim.x);
        grid_barrier(a.ctrl);
        hyb_p2<kAnyRound>(a, rb + ri, blockIdx.x, gridDim.x);
        grid_barrier(a.ctrl);
    }
    finish_rounds(a.ctrl, a.stripes, a.trace, rb, k);
}

// Round state before round 1.  Static handles (hcnt == nullptr): every vertex is
// undecided and nothing is in the set.  Dynamic handles, from the higher-priority
// neighbour counts: a vertex without one is a candidate of round 1 (in the set,
// counted into round 1's |C|), every other vertex is undecided; batches record the
// round-1 candidates as decided in round 1.  vb / nvb: the workgroup's place in the
// graph's share (the grid, or its part of a launch over several graphs); whole waves
// iterate together, each writing the two bitmap words of its 64 vertices.
__device__ void hyb_init_body(const int32_t* hcnt, int64_t n, uint32_t* S, uint32_t* A, int32_t* dround,
                              int64_t* stripes, int64_t vb, int64_t nvb) {
    int64_t c1 = 0;
    const int64_t nthreads = nvb * kBlock;
    const int64_t nr = (n + kWave - 1) / kWave * kWave;
    const int lane = lane_id();
    for (int64_t v = vb * kBlock + threadIdx.x; v < nr; v += nthreads) {
        const bool valid = v < n;
        const int32_t c = !valid ? -1 : hcnt ? hcnt[v] : 1;
        const uint64_t bc = ballot(c == 0), ba = ballot(c > 0);
        c1 += lane == 0 ? __popcll(bc) : 0;
        if (dround && valid) dround[v] = c == 0 ? 1 : 0;
        if (lane < 2) {   // v - lane is the wave's first vertex (a multiple of 64)
            const int64_t w = (v - lane) / 32 + lane;
            if (w * 32 < n) {
                S[w] = (uint32_t)(bc >> (32 * lane));
                A[w] = (uint32_t)(ba >> (32 * lane));
            }
        }
    }
    // one atomic per workgroup into round 1's |C| counter
    __shared__ int64_t part[kWpb];
    for (int off = kWave / 2; off > 0; off >>= 1) c1 += __shfl_xor(c1, off, kWave);
    if (lane == 0) part[threadIdx.x / kWave] = c1;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int q = 0; q < kWpb; ++q) t += part[q];
        int64_t* st = stripes + ((int64_t)(1 & 1) * kStripes + vb % kStripes) * kStripeWords;
        if (t) atomicAdd((unsigned long long*)&st[0], (unsigned long long)t);
    }
}

__global__ void __launch_bounds__(kBlock) k_hyb_init(const int32_t* hcnt, int64_t n, uint32_t* S, uint32_t* A,
                                                     int32_t* dround, int64_t* stripes) {
    hyb_init_body(hcnt, n, S, A, dround, stripes, blockIdx.x, gridDim.x);
}

__global__ void k_hyb_ctrl(Ctrl* ctrl, Meta* smeta, const Meta* meta, int64_t* stripes, int64_t n) {
    ctrl_reset(ctrl, smeta, meta, stripes, n);
}

// Round state of a static handle solved alone before round 1, a thread per bitmap
// word: nothing in the set, every vertex undecided; workgroup 0 also resets the
// control block and the counter stripes.
__global__ void __launch_bounds__(kBlock) k_hyb_init_words(Ctrl* ctrl, Meta* smeta, const Meta* meta,
                                                           int64_t* stripes, int64_t n, uint32_t* S, uint32_t* A) {
    if (blockIdx.x == 0) ctrl_reset(ctrl, smeta, meta, stripes, n);
    const int64_t nw = (n + 31) >> 5;
    GRID_STRIDE(w, nw) {
        const int64_t left = n - w * 32;
        S[w] = 0;
        A[w] = left >= 32 ? ~0u : (1u << left) - 1u;
    }
}

// in_set[v] = S(v); with `gate`, only once every vertex is decided
__global__ void k_hyb_output(const Ctrl* gate, const uint32_t* S, int64_t n, uint8_t* in_set) {
    if (gate && gate->alive != 0) return;
    GRID_STRIDE(v, n) in_set[v] = (uint8_t)bit_of(S, v);
}

// four vertices per thread, one 4-byte store (in_set 4-byte aligned)
__global__ void k_hyb_output4(const Ctrl* gate, const uint32_t* S, int64_t n, uint8_t* in_set) {
    if (gate && gate->alive != 0) return;
    const int64_t nq = n >> 2;
    GRID_STRIDE(i, nq) {
        const uint32_t b = (S[i >> 3] >> ((i & 7) << 2)) & 0xFu;
        reinterpret_cast<uint32_t*>(in_set)[i] = (b & 1u) | ((b >> 1) & 1u) << 8 | ((b >> 2) & 1u) << 16 |
                                                 ((b >> 3) & 1u) << 24;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0)
        for (int64_t v = nq << 2; v < n; ++v) in_set[v] = (uint8_t)bit_of(S, v);
}

HybArgs make_args(GraphCore* g) {
    HybArgs a;
    a.n = g->n;
    a.rp = g->hrp;
    a.hcol = g->hcol;
    a.hcnt = g->hcnt;
    a.crp = g->row_ptr;
    a.ci = g->col_idx;
    a.nnz = g->nnz;
    a.key = g->key;
    a.q8 = g->q8;
    a.seed = g->seed;
    a.user_keys = g->user_keys ? 1 : 0;
    a.oriented = g->dyn_slack > 0 ? 1 : 0;
    a.A = g->hA;
    a.S = g->hS;
    a.blk = g->hblk;
    a.drb = g->drb;
    for (int b = 0; b < 2; ++b) a.dact[b] = g->hdact[b];
    a.nI = ceil_div(g->n, 16);
    a.dptr = g->dptr;
    a.dslot = g->dense_min > 0 && g->nnz > 0 ? g->dslot : nullptr;
    a.dcol = g->dcol;
    a.dbits = g->dbits;
    a.meta = g->meta;
    a.ctrl = g->ctrl;
    a.stripes = g->stripes;
    a.trace = g->trace;
    a.dround = g->count > 0 ? g->dround : nullptr;
    return a;
}

#define HLAUNCH(kernel, work, ...)                                                                            \
    do {                                                                                                      \
        if ((work) > 0) hipLaunchKernelGGL(kernel, dim3(stream_grid(work)), dim3(kBlock), 0, s, __VA_ARGS__); \
        TC_HIP(hipGetLastError());                                                                            \
    } while (0)

}  // namespace

int64_t hyb_blocks(int64_t nnz) { return ceil_div(nnz, kHE); }

int build_hybrid(mis_graph* g, hipStream_t s) {
    const int64_t n = g->n, nnz = g->nnz, nI = g->nI;
    // the key kernel cleared meta unless the keys came from the caller (or n = 0)
    if (g->user_keys || n == 0) TC_HIP(hipMemsetAsync(g->meta, 0, sizeof(Meta), s));
    if (n == 0) return MIS_OK;
    g->hrp = g->row_ptr;
    if (g->dyn_slack > 0) {
        // dynamic handle: both orientations of every edge, in rows of its own with
        // deg + slack slots each (stages: row search, orientation, none)
        TC_HIP(hipMemsetAsync(g->hcnt, 0, (size_t)n * 4, s));
        TC_HIP(hipMemsetAsync(g->lcnt, 0, (size_t)n * 4, s));
        HLAUNCH(k_dyn_caps, n, g->row_ptr, n, g->dyn_slack, g->hflag);
        TC_CHECK(scan_excl_i64(g->hflag, g->drp, n, g->drp + n, (int64_t*)g->scan_tmp, s));
        g->hrp = g->drp;
        const int64_t nb = hyb_blocks(nnz);
        if (nnz > 0) HLAUNCH(k_orient_rows, n, g->row_ptr, n, nnz, nb, g->hbrow);
        build_mark(g, s);
        if (nnz > 0) {
            OrientOut o{g->hrp, g->hcol, g->hcnt, g->lcol, g->lcnt, g->hbase, g->hoff, g->hloff};
            if (g->user_keys)
                hipLaunchKernelGGL(k_orient<true>, dim3((unsigned)nb), dim3(kBlock), 0, s, g->row_ptr, g->col_idx,
                                   g->key, g->q8, g->seed, nnz, g->hbrow, o);
            else
                hipLaunchKernelGGL(k_orient<false>, dim3((unsigned)nb), dim3(kBlock), 0, s, g->row_ptr, g->col_idx,
                                   g->key, g->q8, g->seed, nnz, g->hbrow, o);
            TC_HIP(hipGetLastError());
        }
        build_mark(g, s);
        build_mark(g, s);
        return MIS_OK;
    }
    // static handle: the dense blocks only (stages: dense blocks, then empty ones, as
    // many as a dynamic handle has; the key kernel took the dense-block sample);
    // everything else is read from the caller's CSR by round 1
    const bool dense = g->dense_min > 0 && nnz > 0;
    if (dense) {
        const int64_t stride = dense_stride(nI);
        const int samples = dense_samples(nI);
        if (g->user_keys)   // no key kernel ran
            hipLaunchKernelGGL(k_dense_sample, dim3((unsigned)ceil_div(samples, kWpb)), dim3(kBlock), 0, s,
                               g->row_ptr, g->col_idx, n, stride, samples, g->dense_min, g->dsamp);
        const dim3 grid((unsigned)ceil_div(nI, kDenseChunk));
        if (g->user_keys)
            hipLaunchKernelGGL(k_dense_build<true>, grid, dim3(kBlock), 0, s, g->row_ptr, g->col_idx, g->key, g->q8,
                               g->seed, n, nI, g->dense_min, g->dsamp, samples, g->meta, g->drb, g->dptr, g->dcol,
                               g->dbits, g->dslot);
        else
            hipLaunchKernelGGL(k_dense_build<false>, grid, dim3(kBlock), 0, s, g->row_ptr, g->col_idx, g->key, g->q8,
                               g->seed, n, nI, g->dense_min, g->dsamp, samples, g->meta, g->drb, g->dptr, g->dcol,
                               g->dbits, g->dslot);
        TC_HIP(hipGetLastError());
    }
    build_mark(g, s);
    build_mark(g, s);
    build_mark(g, s);
    return MIS_OK;
}

int hyb_init(GraphCore* g, hipStream_t s) {
    if (g->dyn_slack == 0 && g->count == 0) {   // one launch: a thread per bitmap word
        hipLaunchKernelGGL(k_hyb_init_words, dim3(stream_grid(ceil_div(g->n, 32))), dim3(kBlock), 0, s, g->ctrl,
                           g->smeta, g->meta, g->stripes, g->n, g->hS, g->hA);
        TC_HIP(hipGetLastError());
        return MIS_OK;
    }
    hipLaunchKernelGGL(k_hyb_ctrl, dim3(1), dim3(256), 0, s, g->ctrl, g->smeta, g->meta, g->stripes, g->n);
    TC_HIP(hipGetLastError());
    if (g->n > 0)
        hipLaunchKernelGGL(k_hyb_init, dim3(stream_grid(g->n)), dim3(kBlock), 0, s,
                           g->dyn_slack > 0 ? g->hcnt : nullptr, g->n, g->hS, g->hA,
                           g->count > 0 ? g->dround : nullptr, g->stripes);
    TC_HIP(hipGetLastError());
    return MIS_OK;
}

// phase 0 = candidate kernel, 1 = exclusion kernel
// (first: round 1 of the solve, which visits every vertex: a thread per vertex)
int hyb_enqueue_phase(GraphCore* g, int phase, int r, hipStream_t s, bool first) {
    HybArgs a = make_args(g);
    // the first batch's round 1: in the candidate phase a grid-stride loop with a
    // thread per vertex over 4 workgroups per compute unit (as fast as 8 or 16 per CU,
    // and 6% faster than a workgroup per 256 vertices on RMAT 2^22); in the exclusion
    // phase of a static handle a wave per kP2Words bitmap words
    const int64_t per = phase == 1 && g->dyn_slack == 0 ? (int64_t)kBlock * 32 * kP2Words / kWave : kBlock;
    int64_t grid = first ? std::max<int64_t>(g->grid_blocks, ceil_div(g->n, per)) : g->grid_blocks;
    if (first && phase == 0) grid = std::min<int64_t>(grid, 4 * (int64_t)g->cus);
    // later rounds: a thread per bitmap word at most
    if (!first) grid = std::min<int64_t>(grid, std::max<int64_t>(1, ceil_div(ceil_div(g->n, 32), kBlock)));
    const dim3 gd((unsigned)grid), bd(kBlock);
    if (!first) {
        if (phase == 0) hipLaunchKernelGGL(k_hyb_p1<kLaterRounds>, gd, bd, 0, s, a, r);
        else hipLaunchKernelGGL(k_hyb_p2<kLaterRounds>, gd, bd, 0, s, a, r);
    } else if (a.user_keys) {
        if (phase == 0) hipLaunchKernelGGL(k_hyb_p1<kRound1Keys>, gd, bd, 0, s, a, r);
        else hipLaunchKernelGGL(k_hyb_p2<kRound1Keys>, gd, bd, 0, s, a, r);
    } else {
        if (phase == 0) hipLaunchKernelGGL(k_hyb_p1<kRound1>, gd, bd, 0, s, a, r);
        else hipLaunchKernelGGL(k_hyb_p2<kRound1>, gd, bd, 0, s, a, r);
    }
    TC_HIP(hipGetLastError());
    return MIS_OK;
}

// k rounds as one cooperative launch (see k_hyb_rounds)
int hyb_enqueue_rounds(GraphCore* g, int k, hipStream_t s) {
    HybArgs a = make_args(g);
    return launch_cooperative((const void*)k_hyb_rounds, g, &a, k, s);
}

int hyb_output(GraphCore* g, uint8_t* in_set, bool if_done, hipStream_t s) {
    const Ctrl* gate = if_done ? g->ctrl : nullptr;
    if (g->n > 0 && ((uintptr_t)in_set & 3) == 0)
        hipLaunchKernelGGL(k_hyb_output4, dim3(stream_grid(ceil_div(g->n, 4))), dim3(kBlock), 0, s, gate, g->hS, g->n,
                           in_set);
    else if (g->n > 0)
        hipLaunchKernelGGL(k_hyb_output, dim3(stream_grid(g->n)), dim3(kBlock), 0, s, gate, g->hS, g->n, in_set);
    TC_HIP(hipGetLastError());
    return MIS_OK;
}

// ---------------------------------------------------------------- batches of handles
//
// Independently built hybrid handles solved together: every round kernel is one
// launch over all graphs.  Each graph keeps its own structure (only read) and gets
// its own round state in the caller's scratch; a launch's workgroups are split
// into per-graph shares (bstart: graph g owns workgroups bstart[g] .. bstart[g+1]-1,
// at least one), and a share runs the single-graph round code as if it were the
// whole grid.  Graphs share no edge, so each graph's rounds are those it runs
// alone (its rule reads only its own vertices).

namespace {

struct MultiDesc {
    HybArgs a;                // the graph's structure and its round state in the scratch
    const Meta* meta;
    Meta* smeta;
    int64_t n;
    uint8_t* out;             // the caller's in/out vector of this graph
};

constexpr int64_t kMultiVerts = 4096;   // vertices per workgroup of a graph's share

// the graph of workgroup b (largest g with bstart[g] <= b; b is uniform)
__device__ inline int graph_of(const int64_t* bstart, int count, int64_t b) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (bstart[mid] <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// round state before round 1, every graph: control block and counters (workgroup 0
// of the graph's share), then the bitmaps and round 1's candidate count (the
// counters are cleared in a launch before, so that no workgroup adds into a stripe
// another one is still clearing)
__global__ void __launch_bounds__(kBlock) k_multi_ctrl(const MultiDesc* d, int count) {
    const int64_t g = blockIdx.x;
    if (g >= count) return;
    const MultiDesc& D = d[g];
    if (threadIdx.x == 0) {
        Ctrl c;
        memset(&c, 0, sizeof(c));
        c.alive = D.n;
        *D.a.ctrl = c;
        *D.smeta = *D.meta;
    }
    for (int i = threadIdx.x; i < 2 * kStripes * kStripeWords; i += kBlock) D.a.stripes[i] = 0;
}

__global__ void __launch_bounds__(kBlock) k_multi_init(const MultiDesc* d, const int64_t* bstart, int count) {
    const int g = graph_of(bstart, count, blockIdx.x);
    const MultiDesc& D = d[g];
    hyb_init_body(D.a.oriented ? D.a.hcnt : nullptr, D.n, D.a.S, D.a.A, nullptr, D.a.stripes, blockIdx.x - bstart[g],
                  bstart[g + 1] - bstart[g]);
}

__global__ void __launch_bounds__(kBlock) k_multi_p1(const MultiDesc* d, const int64_t* bstart, int count, int ri) {
    const int g = graph_of(bstart, count, blockIdx.x);
    const HybArgs& a = d[g].a;
    if (a.ctrl->alive == 0) return;   // finished (and its last round closed) in an earlier launch
    hyb_p1<kAnyRound>(a, a.ctrl->rbase + ri, blockIdx.x - bstart[g], bstart[g + 1] - bstart[g]);
}

__global__ void __launch_bounds__(kBlock) k_multi_p2(const MultiDesc* d, const int64_t* bstart, int count, int ri) {
    const int g = graph_of(bstart, count, blockIdx.x);
    const HybArgs& a = d[g].a;
    if (a.ctrl->alive == 0) return;
    hyb_p2<kAnyRound>(a, a.ctrl->rbase + ri, blockIdx.x - bstart[g], bstart[g + 1] - bstart[g]);
}

// after k rounds: a wave per graph closes its last round and moves its base past
// it; the undecided vertices of all graphs are summed into sum->alive (cleared
// before), each graph's rounds and set size recorded
__global__ void __launch_bounds__(kBlock) k_multi_close(const MultiDesc* d, int count, int k, Ctrl* sum,
                                                        int32_t* g_rounds, int64_t* g_in) {
    const int64_t g = (int64_t)blockIdx.x * kWpb + threadIdx.x / kWave;
    if (g >= count) return;
    const HybArgs& a = d[g].a;
    const int rb = a.ctrl->rbase;
    close_round(a.ctrl, a.stripes, nullptr, rb + k);
    if (lane_id() == 0) {
        a.ctrl->rbase = rb + k;
        const int64_t alive = a.ctrl->alive;
        if (alive) atomicAdd((unsigned long long*)&sum->alive, (unsigned long long)alive);
        atomicOr(&sum->error, a.ctrl->error);
        g_rounds[g] = a.ctrl->round;
        g_in[g] = a.ctrl->n_in;
    }
}

__global__ void __launch_bounds__(kBlock) k_multi_output(const MultiDesc* d, const int64_t* bstart, int count) {
    const int g = graph_of(bstart, count, blockIdx.x);
    const int64_t vb = blockIdx.x - bstart[g], nvb = bstart[g + 1] - bstart[g];
    const MultiDesc& D = d[g];
    for (int64_t v = vb * kBlock + threadIdx.x; v < D.n; v += nvb * kBlock) D.out[v] = (uint8_t)bit_of(D.a.S, v);
}

}  // namespace

// Scratch of a batch of handles: a summary control block, the per-graph records
// (rounds, set sizes), the workgroup shares, the descriptors, then every graph's
// round state.
struct MultiLayout {
    size_t sum = 0, rounds = 0, in = 0, bstart = 0, bstart1 = 0, desc = 0;
    std::vector<size_t> state;
    size_t total = 0;
};

static MultiLayout multi_layout(mis_graph* const* gs, int32_t count) {
    MultiLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        off = (off + 255) & ~(size_t)255;
        const size_t o = off;
        off += bytes ? bytes : 8;
        return o;
    };
    L.sum = take(sizeof(Ctrl));
    L.rounds = take((size_t)count * 4);
    L.in = take((size_t)count * 8);
    L.bstart = take((size_t)(count + 1) * 8);
    L.bstart1 = take((size_t)(count + 1) * 8);
    L.desc = take((size_t)count * sizeof(MultiDesc));
    L.state.resize((size_t)count);
    for (int32_t i = 0; i < count; ++i) {
        GraphCore v = *gs[i];
        L.state[(size_t)i] = take(layout_state(&v, nullptr, false));
    }
    L.total = (off + 255) & ~(size_t)255;
    return L;
}

}  // namespace tcmis

using namespace tcmis;

extern "C" {

int mis_solve_batch_scratch_bytes(mis_graph* const* graphs, int32_t count, size_t* bytes) {
    set_error("");
    if (!bytes || count < 0 || (count > 0 && !graphs)) {
        set_error("bad argument");
        return MIS_EINVAL;
    }
    for (int32_t i = 0; i < count; ++i)
        if (!graphs[i]) { set_error("a handle is null"); return MIS_EINVAL; }
    *bytes = multi_layout(graphs, count).total;
    return MIS_OK;
}

int mis_solve_batch(mis_graph* const* graphs, int32_t count, uint8_t* const* in_sets, void* scratch,
                    size_t scratch_bytes, mis_stats* st, int32_t* graph_rounds, int64_t* graph_in, void* stream) {
    set_error("");
    if (count < 0 || (count > 0 && (!graphs || !in_sets))) {
        set_error("bad argument");
        return MIS_EINVAL;
    }
    int64_t nmax = 0, ntot = 0;
    int poll = 4;
    for (int32_t i = 0; i < count; ++i) {
        const mis_graph* g = graphs[i];
        if (!g) { set_error("a handle is null"); return MIS_EINVAL; }
        if (g->path != MIS_PATH_HYBRID || g->count > 0) {
            set_error("a batch of handles takes single-graph hybrid handles (mis_build_tiles, path hybrid)");
            return MIS_EINVAL;
        }
        if (g->n > 0 && !in_sets[i]) { set_error("an output vector is null"); return MIS_EINVAL; }
        nmax = std::max(nmax, g->n);
        ntot += g->n;
        poll = std::max(poll, g->poll_rounds);
    }
    const MultiLayout L = multi_layout(graphs, count);
    if (count > 0 && (!scratch || ((uintptr_t)scratch & 255) || scratch_bytes < L.total)) {
        set_error("scratch must be 256-byte aligned device memory of at least " + std::to_string(L.total) +
                  " bytes (mis_solve_batch_scratch_bytes)");
        return MIS_EINVAL;
    }
    if (st) {
        st->rounds = 0;
        st->n_in = 0;
        st->path = MIS_PATH_HYBRID;
        st->tile = 16;
        st->tiles = 0;
    }
    if (count == 0) return MIS_OK;
    hipStream_t s = (hipStream_t)stream;
    char* base = (char*)scratch;
    Ctrl* sum = (Ctrl*)(base + L.sum);
    int32_t* d_rounds = (int32_t*)(base + L.rounds);
    int64_t* d_in = (int64_t*)(base + L.in);
    int64_t* d_bstart = (int64_t*)(base + L.bstart);
    int64_t* d_bstart1 = (int64_t*)(base + L.bstart1);   // round 1: a thread per vertex
    MultiDesc* d_desc = (MultiDesc*)(base + L.desc);
    std::vector<MultiDesc> desc((size_t)count);
    std::vector<int64_t> bstart((size_t)count + 1, 0), bstart1((size_t)count + 1, 0);
    for (int32_t i = 0; i < count; ++i) {
        GraphCore v = *graphs[i];
        layout_state(&v, base + L.state[(size_t)i], false);
        MultiDesc& D = desc[(size_t)i];
        D.a = make_args(&v);
        D.a.trace = nullptr;
        D.a.dround = nullptr;
        D.meta = v.meta;
        D.smeta = v.smeta;
        D.n = v.n;
        D.out = in_sets[i];
        const int64_t share = std::min<int64_t>(std::max<int64_t>(1, ceil_div(v.n, kMultiVerts)),
                                                std::max(1, v.grid_blocks));
        bstart[(size_t)i + 1] = bstart[(size_t)i] + share;
        bstart1[(size_t)i + 1] = bstart1[(size_t)i] + std::max<int64_t>(share, ceil_div(v.n, kBlock));
    }
    const int64_t nblocks = bstart[(size_t)count], nblocks1 = bstart1[(size_t)count];
    if (nblocks1 >= (1ll << 31)) { set_error("too many workgroups for one launch"); return MIS_EINVAL; }
    TC_HIP(hipMemcpyAsync(d_desc, desc.data(), desc.size() * sizeof(MultiDesc), hipMemcpyHostToDevice, s));
    TC_HIP(hipMemcpyAsync(d_bstart, bstart.data(), bstart.size() * 8, hipMemcpyHostToDevice, s));
    TC_HIP(hipMemcpyAsync(d_bstart1, bstart1.data(), bstart1.size() * 8, hipMemcpyHostToDevice, s));
    const dim3 grid((unsigned)nblocks), grid1((unsigned)nblocks1), blk(kBlock), cgrid((unsigned)ceil_div(count, kWpb));
    hipLaunchKernelGGL(k_multi_ctrl, dim3((unsigned)count), blk, 0, s, d_desc, count);
    hipLaunchKernelGGL(k_multi_init, grid, blk, 0, s, d_desc, d_bstart, count);
    TC_HIP(hipGetLastError());
    Ctrl h;
    int32_t r = 0;
    for (;;) {
        for (int i = 1; i <= poll; ++i) {
            const bool first = r == 0 && i == 1;
            hipLaunchKernelGGL(k_multi_p1, first ? grid1 : grid, blk, 0, s, d_desc, first ? d_bstart1 : d_bstart, count, i);
            hipLaunchKernelGGL(k_multi_p2, first ? grid1 : grid, blk, 0, s, d_desc, first ? d_bstart1 : d_bstart, count, i);
        }
        TC_HIP(hipMemsetAsync(sum, 0, sizeof(Ctrl), s));
        hipLaunchKernelGGL(k_multi_close, cgrid, blk, 0, s, d_desc, count, poll, sum, d_rounds, d_in);
        TC_HIP(hipGetLastError());
        TC_HIP(hipMemcpyAsync(&h, sum, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
        TC_HIP(hipStreamSynchronize(s));
        r += poll;
        if (h.error) { set_error("a device-side check of the round kernels failed"); return MIS_EINTERNAL; }
        if (h.alive == 0) break;
        if (r > nmax + 1 + poll) { set_error("round limit exceeded (equal adjacent keys?)"); return MIS_EINTERNAL; }
    }
    hipLaunchKernelGGL(k_multi_output, grid, blk, 0, s, d_desc, d_bstart, count);
    TC_HIP(hipGetLastError());
    std::vector<int32_t> hr((size_t)count);
    std::vector<int64_t> hi((size_t)count);
    TC_HIP(hipMemcpyAsync(hr.data(), d_rounds, (size_t)count * 4, hipMemcpyDeviceToHost, s));
    TC_HIP(hipMemcpyAsync(hi.data(), d_in, (size_t)count * 8, hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    int32_t rmax = 0;
    int64_t in = 0;
    for (int32_t i = 0; i < count; ++i) {
        rmax = std::max(rmax, hr[(size_t)i]);
        in += hi[(size_t)i];
    }
    if (graph_rounds) std::copy(hr.begin(), hr.end(), graph_rounds);
    if (graph_in) std::copy(hi.begin(), hi.end(), graph_in);
    if (st) {
        st->rounds = rmax;
        st->n_in = in;
    }
    (void)ntot;
    return MIS_OK;
}

}  // extern "C"
