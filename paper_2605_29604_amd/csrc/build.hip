// Build stage: validation, priority keys, vertex reordering and the nonzero
// T x T bit tiles (Section 3.2: the adjacency matrix is kept as its nonzero tiles
// in a compressed block format), plus the degree-binned vertex lists of the CSR path.
//
// Everything is enqueued on the caller's stream inside the caller's workspace:
// no allocation and no host synchronisation (except optional validation and the
// host RCM order).  Tile construction:
//   1. new order p = new_id[v]; new row pointer by a scan of degrees in new order;
//      the new row of every new-order entry by a max-scan of row-start marks;
//   2. one entry per kept adjacency entry (v, u) in new-row order, packed as
//      (block(q) | p | q mod T) with q = new_id[u]; with `orient`, only entries
//      whose column u has a lower priority than v are kept;
//   3. a stable radix sort on block(q) alone: entries come out ordered by
//      (block(q), p), which, read transposed as row q / column p (the matrix is
//      symmetric, and the kept orientation is transposed on purpose), is exactly
//      the tile order (row block, column block) with each tile's entries contiguous;
//   4. tile heads by a scan of head flags; one lane per tile (four for T=32) ORs its
//      entries into registers, stores the bitmap and ORs the tile's nonempty rows
//      into its row-block's mask; row-block pointers by binary search.
#include <algorithm>
#include <vector>

#include "dense.hpp"
#include "graph.hpp"

namespace tcmis {

namespace {

enum : uint32_t { kErrRange = 1, kErrLoop = 2, kErrDup = 4, kErrAsym = 8, kErrTie = 16, kErrCross = 32 };


__device__ inline int64_t row_of(const int64_t* rp, int64_t n, int64_t e) {
    int64_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (rp[mid] <= e) lo = mid; else hi = mid;
    }
    return lo;
}

// graph of input vertex v in a batch: largest g with goff[g] <= v
__device__ inline int64_t graph_of(const int64_t* goff, int64_t count, int64_t v) {
    int64_t lo = 0, hi = count - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (goff[mid] <= v) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ void k_validate_rows(const int64_t* rp, int64_t n, int64_t nnz, uint32_t* err) {
    GRID_STRIDE(v, n) {
        const int64_t a = rp[v], b = rp[v + 1];
        if (a < 0 || b < a || b > nnz) atomicOr(err, kErrRange);
    }
}

__global__ void k_validate_edges(const int64_t* rp, const int32_t* ci, int64_t n, int64_t nnz, const uint64_t* key,
                                 const int64_t* goff, int64_t count, uint32_t* err) {
    GRID_STRIDE(e, nnz) {
        const int64_t v = row_of(rp, n, e);
        const int64_t u = ci[e];
        if (u < 0 || u >= n) { atomicOr(err, kErrRange); continue; }
        if (u == v) { atomicOr(err, kErrLoop); continue; }
        if (e > rp[v] && (int64_t)ci[e - 1] >= u) atomicOr(err, kErrDup);
        int64_t lo = rp[u], hi = rp[u + 1];
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if ((int64_t)ci[mid] < v) lo = mid + 1; else hi = mid;
        }
        if (lo >= rp[u + 1] || (int64_t)ci[lo] != v) atomicOr(err, kErrAsym);
        if (key && key[u] == key[v]) atomicOr(err, kErrTie);
        if (goff && graph_of(goff, count, u) != graph_of(goff, count, v)) atomicOr(err, kErrCross);
    }
}

// Default priority keys (Section 3.3): q << 56 | hash << 24 | v with hash = top 32
// bits of output v+1 of the SplitMix64 stream seeded with `seed` (the random
// perturbation) and q by the rule:
//   MIS_KEY_DEGREE  floor(255 / (1 + deg)) (lower degree wins)
//   MIS_KEY_HASH    0 (purely random priority, H1)
//   MIS_KEY_EQ1     Eq. 1, d / (d + deg - eps), scaled to 255 and discretised in
//                   integers: D = floor(256 nnz / n) is the average degree with 8
//                   fractional bits, e = the low 8 bits of the same SplitMix64
//                   output is eps in 1/256, q = min(255, floor(255 D / (D + 256 deg -
//                   e))), 255 where that denominator is not positive
// In a batch the id in the key is graph-local (v - goff[g]) and n, nnz are graph g's.
// With `sk` the kernel also writes the priority order's sort keys (k_order_keys'
// layout: ~key at position n-1-v), saving that pass a read of the keys.  With `q8`
// it also writes q alone, one byte per vertex (the hybrid path's orientation
// compares classes from this table and rebuilds the hash in registers on a tie).
__device__ inline uint64_t key_class(int rule, int64_t deg, int64_t gn, int64_t gnnz, uint64_t z) {
    if (rule == MIS_KEY_HASH) return 0;
    if (rule == MIS_KEY_DEGREE) return (uint64_t)(255 / (1 + deg));
    const int64_t D = gn > 0 ? (256 * gnnz) / gn : 0;
    const int64_t den = D + 256 * deg - (int64_t)(z & 0xFFu);
    if (den <= 0) return 255;
    const int64_t q = (255 * D) / den;
    return (uint64_t)(q < 255 ? q : 255);
}

__device__ inline void key_one(int64_t v, int64_t lv, int64_t gn, int64_t gnnz, const int64_t* rp, int64_t n,
                               uint64_t seed, int rule, uint64_t* key, uint64_t* sk, uint8_t* q8) {
    const int64_t deg = rp[v + 1] - rp[v];
    const uint64_t z = splitmix_at(seed, (uint64_t)lv + 1);
    const uint64_t q = key_class(rule, deg, gn, gnnz, z);
    const uint64_t k = (q << 56) | ((z >> 32) << 24) | (uint64_t)lv;
    key[v] = k;
    if (sk) sk[n - 1 - v] = ~k;
    if (q8) q8[v] = (uint8_t)q;
}

// Batches: a workgroup takes kKeysSpan consecutive vertices (kKeysPer per thread, a
// workgroup's width apart), finds the graph of the first once and keeps the graph's
// bounds in registers, stepping to the next graph where a vertex passes its end.
constexpr int kKeysPer = 16;
constexpr int64_t kKeysSpan = (int64_t)kBlock * kKeysPer;

// With `samp` (hybrid path with dense blocks) the kernel's waves also take the
// dense-block sample (dense.hpp), sparing the build a launch.
__global__ void k_keys(const int64_t* rp, int64_t n, uint64_t seed, const int64_t* goff, int64_t count, int rule,
                       uint64_t* key, uint64_t* sk, uint8_t* q8, Meta* meta, const int32_t* ci, int64_t stride,
                       int samples, int dense_min, int32_t* samp) {
    if (meta && blockIdx.x == 0 && threadIdx.x == 0) *meta = Meta{};   // the hybrid build's sizes start at 0
    if (!goff) {
        const int64_t nnz = rp[n] - rp[0];
        GRID_STRIDE(v, n) key_one(v, v, n, nnz, rp, n, seed, rule, key, sk, q8);
    } else {
        for (int64_t s0 = (int64_t)blockIdx.x * kKeysSpan; s0 < n; s0 += (int64_t)gridDim.x * kKeysSpan) {
            int64_t g = graph_of(goff, count, s0);   // the same for the whole workgroup
            int64_t gs = goff[g], ge = goff[g + 1], gnnz = rp[ge] - rp[gs];
            for (int i = 0; i < kKeysPer; ++i) {
                const int64_t v = s0 + (int64_t)i * kBlock + threadIdx.x;
                if (v >= n) break;
                if (v >= ge) {
                    while (g + 1 < count && goff[g + 1] <= v) ++g;
                    gs = goff[g];
                    ge = goff[g + 1];
                    gnnz = rp[ge] - rp[gs];
                }
                key_one(v, v - gs, ge - gs, gnnz, rp, n, seed, rule, key, sk, q8);
            }
        }
    }
    if (samp)
        dense_sample(rp, ci, n, stride, samples, dense_min, samp, ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave,
                     (int64_t)gridDim.x * blockDim.x / kWave);
}

// Every kernel that fixes the vertex order also writes ndeg[p], the degree of the
// vertex at new position p (the new row pointer is its exclusive scan).
__global__ void k_identity_order(const int64_t* rp, int32_t* order, int32_t* new_id, int32_t* ndeg, int64_t n) {
    GRID_STRIDE(v, n) {
        order[v] = (int32_t)v;
        new_id[v] = (int32_t)v;
        ndeg[v] = (int32_t)(rp[v + 1] - rp[v]);
    }
}

__global__ void k_invert(const int64_t* rp, const int32_t* new_id, int32_t* order, int32_t* ndeg, int64_t n) {
    GRID_STRIDE(v, n) {
        const int32_t p = new_id[v];
        order[p] = (int32_t)v;
        ndeg[p] = (int32_t)(rp[v + 1] - rp[v]);
    }
}

// Sort keys of the degree-class and priority orders (ascending, stable sort).
//   degree class: 255 - floor(255 / (1 + deg)) (the discretised priority of the key
//                 rule, highest first), one 8-bit pass; ties keep increasing id.
//   priority:     ~key, input laid out by decreasing id.  With the default key rule
//                 the low 24 key bits are the id, so sorting bits 24..63 stably
//                 already yields decreasing key order; user keys sort all 64 bits.
__global__ void k_order_keys(const int64_t* rp, const uint64_t* key, int64_t n, int mode, uint64_t* sk,
                             uint32_t* payload) {
    GRID_STRIDE(i, n) {
        if (mode == MIS_REORDER_DEGREE) {
            const int64_t deg = rp[i + 1] - rp[i];
            sk[i] = (uint64_t)(255 - 255 / (1 + deg));
            payload[i] = (uint32_t)i;
        } else {
            const int64_t v = n - 1 - i;
            sk[i] = ~key[v];
            if (payload) payload[i] = (uint32_t)v;
        }
    }
}

// Order and new ids from sorted ~keys that carry the vertex id in their low 24 bits.
// The keys were sorted on bits [lo, 64) only: a key inside a run of keys equal in
// those bits goes to the run's start plus its rank in the run by the whole key (the
// ids make the keys distinct).  The sorted keys are only read, so the runs need no
// coordination between threads; they are short (the bits below lo hold hash bits
// and the id).
__global__ void k_scatter_order_keys(const int64_t* rp, const uint64_t* sorted_sk, int64_t n, int lo,
                                     int32_t* order, int32_t* new_id, int32_t* ndeg) {
    GRID_STRIDE(p, n) {
        // the key and both neighbours (clamped indices) in one round trip
        const uint64_t x = sorted_sk[p], xp = sorted_sk[p > 0 ? p - 1 : p], xn = sorted_sk[p + 1 < n ? p + 1 : p];
        const uint64_t t = x >> lo;
        int64_t q = p;
        if ((p > 0 && (xp >> lo) == t) || (p + 1 < n && (xn >> lo) == t)) {
            int64_t s0 = p, e = p + 1;
            while (s0 > 0 && (sorted_sk[s0 - 1] >> lo) == t) --s0;
            while (e < n && (sorted_sk[e] >> lo) == t) ++e;
            int64_t rank = 0;
            for (int64_t j = s0; j < e; ++j) rank += sorted_sk[j] < x;
            q = s0 + rank;
        }
        const int32_t v = (int32_t)(~x & 0xFFFFFFull);
        order[q] = v;
        new_id[v] = (int32_t)q;
        ndeg[q] = (int32_t)(rp[v + 1] - rp[v]);
    }
}

__global__ void k_scatter_order(const int64_t* rp, const uint32_t* sorted_payload, int64_t n, int32_t* order,
                                int32_t* new_id, int32_t* ndeg) {
    GRID_STRIDE(p, n) {
        const int32_t v = (int32_t)sorted_payload[p];
        order[p] = v;
        new_id[v] = (int32_t)p;
        ndeg[p] = (int32_t)(rp[v + 1] - rp[v]);
    }
}

// kMode: 0 all entries, 1 entries whose column has a lower priority, by new id (the
// priority order), 2 the same by key.  Entry = block(q) << 36 | p << 5 | q mod T for
// new row p and new column q: read transposed (row q, column p) after a stable sort
// on block(q), the kept entries are each lower-priority vertex's higher-priority
// neighbours, in tile order.
template <int kTshift, int kMode>
__device__ inline bool make_entry(int32_t p, int32_t q, uint64_t kv, uint64_t ku, uint64_t* out) {
    bool keep = true;
    if (kMode == 1) keep = q > p;
    if (kMode == 2) keep = ku < kv;
    *out = ((uint64_t)(q >> kTshift) << 36) | ((uint64_t)p << 5) | (uint64_t)(q & ((1 << kTshift) - 1));
    return keep;
}

constexpr int kEntIters = 16;
constexpr int kEntBlock = kBlock * kEntIters;   // new-order entries per workgroup (= one sort block)
constexpr int kEntWindow = 2048;                // new rows a workgroup keeps in LDS
constexpr int kEntSteps = 11;                   // 2^kEntSteps = kEntWindow

// largest row p in [lo, hi] with nrp[p] <= e (the row that holds new-order entry e)
__device__ inline int32_t find_row(const int32_t* nrp, int64_t lo, int64_t hi, int64_t e) {
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (nrp[mid] <= e) lo = mid; else hi = mid - 1;
    }
    return (int32_t)lo;
}

// first row of every workgroup's entry range
__global__ void k_block_rows(const int32_t* nrp, int64_t n, int64_t nnz, int64_t nblocks, int32_t* brow) {
    GRID_STRIDE(b, nblocks + 1) {
        const int64_t e = b < nblocks ? b * kEntBlock : nnz - 1;
        brow[b] = find_row(nrp, 0, n - 1, e);
    }
}

// One candidate entry per adjacency entry in new-row order, coalesced over entries.
// When the workgroup's rows fit in LDS (the common case), their new and old row
// starts (and, for key orientation, vertices) are staged there first; each thread
// then finds the rows of its kEntIters entries with a fixed-step search in LDS and
// issues all their column reads, then all their new-id (and key) gathers, so that
// every stage has kEntIters loads in flight instead of a chain of dependent loads
// per entry.  The column reads and the entry stores are non-temporal: the caches
// are left to the randomly gathered new ids.  The kept entries are compacted to the
// front of the workgroup's range (order preserved) and their number goes to
// cnt[block].
template <int kTshift, int kMode>
__global__ void __launch_bounds__(kBlock) k_entries(const int64_t* rp, const int32_t* ci, const int32_t* order,
                                                    const int32_t* nrp, const int32_t* brow, const int32_t* new_id,
                                                    const uint64_t* key, int64_t nnz, uint64_t* ent, int32_t* cnt) {
    constexpr bool kVert = kMode == 2;   // the row's vertex is needed beyond its old row start
    __shared__ int32_t win[kEntWindow];                 // new row starts
    __shared__ int32_t wold[kEntWindow];                // old row starts (nnz < 2^31)
    __shared__ int32_t wver[kVert ? kEntWindow : 1];    // row vertices
    __shared__ int32_t wcnt[kEntIters][kBlock / kWave];
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    const int64_t base = (int64_t)blockIdx.x * kEntBlock;
    const int64_t p0 = brow[blockIdx.x], p1 = brow[blockIdx.x + 1];
    const int64_t w = p1 - p0 + 1;
    const bool in_lds = w <= kEntWindow;   // uniform over the workgroup
    if (in_lds)
        for (int64_t i = threadIdx.x; i < w; i += kBlock) {
            const int32_t v = order[p0 + i];
            win[i] = nrp[p0 + i];
            wold[i] = (int32_t)rp[v];
            if (kVert) wver[i] = v;
        }
    __syncthreads();
    int32_t pr[kEntIters], uu[kEntIters], vv[kEntIters];   // row (-1: none), column, row vertex
    if (in_lds) {
        const int wl = (int)w - 1;
        int li[kEntIters];
        #pragma unroll
        for (int it = 0; it < kEntIters; ++it) {
            const int32_t e = (int32_t)std::min<int64_t>(base + (int64_t)it * kBlock + threadIdx.x, nnz - 1);
            int lo = 0;   // win[0] <= e: row p0 holds the workgroup's first entry
            #pragma unroll
            for (int k = kEntSteps - 1; k >= 0; --k) {
                const int c = lo + (1 << k);
                const int32_t wc = win[std::min(c, wl)];
                lo = ((c <= wl) & (wc <= e)) ? c : lo;
            }
            li[it] = lo;
        }
        #pragma unroll
        for (int it = 0; it < kEntIters; ++it) {
            const int64_t e = base + (int64_t)it * kBlock + threadIdx.x;
            const int32_t ec = (int32_t)std::min<int64_t>(e, nnz - 1);
            uu[it] = __builtin_nontemporal_load(&ci[wold[li[it]] + (ec - win[li[it]])]);
            vv[it] = kVert ? wver[li[it]] : 0;
            pr[it] = e < nnz ? (int32_t)(p0 + li[it]) : -1;
        }
    } else {
        #pragma unroll
        for (int it = 0; it < kEntIters; ++it) {
            const int64_t e = base + (int64_t)it * kBlock + threadIdx.x;
            pr[it] = -1;
            uu[it] = vv[it] = 0;
            if (e < nnz) {
                const int32_t p = find_row(nrp, p0, p1, e);
                const int32_t v = order[p];
                uu[it] = ci[rp[v] + (e - nrp[p])];
                vv[it] = v;
                pr[it] = p;
            }
        }
    }
    // every uu / vv is a valid vertex here (entries past the end repeat the last one)
    int32_t qv[kEntIters];
    uint64_t kv[kEntIters], ku[kEntIters];
    #pragma unroll
    for (int it = 0; it < kEntIters; ++it) {
        qv[it] = new_id[uu[it]];
        kv[it] = kMode == 2 ? key[vv[it]] : 0;
        ku[it] = kMode == 2 ? key[uu[it]] : 0;
    }
    uint64_t kept = 0;   // bit it: entry it is kept
    uint64_t x[kEntIters];
    #pragma unroll
    for (int it = 0; it < kEntIters; ++it) {
        x[it] = 0;
        if (pr[it] >= 0 && make_entry<kTshift, kMode>(pr[it], qv[it], kv[it], ku[it], &x[it])) kept |= 1ull << it;
    }
    #pragma unroll
    for (int it = 0; it < kEntIters; ++it) {
        const uint64_t b = ballot((kept >> it) & 1);
        if (lane == 0) wcnt[it][wid] = __popcll(b);
    }
    __syncthreads();
    int written = 0;
    #pragma unroll
    for (int it = 0; it < kEntIters; ++it) {
        int before = written, total = written;
        for (int q = 0; q < kBlock / kWave; ++q) {
            if (q < wid) before += wcnt[it][q];
            total += wcnt[it][q];
        }
        const uint64_t b = ballot((kept >> it) & 1);
        if ((kept >> it) & 1) __builtin_nontemporal_store(x[it], &ent[base + before + __popcll(b & lanes_below())]);
        written = total;
    }
    if (threadIdx.x == 0) cnt[blockIdx.x] = written;
}

constexpr int kHeadIters = 8;
constexpr int kHeadChunk = kBlock * kHeadIters;   // sorted entries per workgroup

template <int kTshift>
__device__ inline uint64_t tile_key(uint64_t x) {
    return ((x >> 36) << 32) | ((uint32_t)((x >> 5) & 0x7FFFFFFFull) >> kTshift);
}

// does sorted entry e start a tile (its (row block, column block) differs from e-1's)?
// (both loads issued together; loading e-1 costs less than taking it from the lane
// below, whose shuffle would wait for this lane's load)
template <int kTshift>
__device__ inline bool is_head(const uint64_t* ent, int64_t e, int64_t nvalid, uint64_t* x) {
    if (e >= nvalid) return false;
    *x = ent[e];
    return e == 0 || tile_key<kTshift>(*x) != tile_key<kTshift>(ent[e - 1]);
}

// heads per chunk of sorted entries; also clears hrows (n_rows words) and the
// row-block tile counts (n_rows + 1 words) that the bitmap pass adds up
template <int kTshift>
__global__ void __launch_bounds__(kBlock) k_head_count(const uint64_t* ent, const Meta* meta, int32_t* sums,
                                                       uint32_t* hrows, int64_t* rb_cnt, int64_t n_rows) {
    __shared__ int32_t wsum[kBlock / kWave];
    GRID_STRIDE(I, n_rows + 1) {
        if (I < n_rows) hrows[I] = 0;
        rb_cnt[I] = 0;
    }
    const int64_t nvalid = meta->nvalid;
    const int64_t base = (int64_t)blockIdx.x * kHeadChunk;
    int c = 0;
    for (int it = 0; it < kHeadIters; ++it) {
        uint64_t x;
        c += __popcll(ballot(is_head<kTshift>(ent, base + (int64_t)it * kBlock + threadIdx.x, nvalid, &x)));
    }
    if (lane_id() == 0) wsum[threadIdx.x / kWave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int q = 0; q < kBlock / kWave; ++q) t += wsum[q];
        sums[blockIdx.x] = t;
    }
}

template <int kTshift>
__global__ void __launch_bounds__(kBlock) k_head_write(const uint64_t* ent, const Meta* meta, const int32_t* chunk_off,
                                                       int32_t* tile_start, int32_t* tile_col) {
    __shared__ int32_t wcnt[kBlock / kWave];
    const int64_t nvalid = meta->nvalid;
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    const int64_t base = (int64_t)blockIdx.x * kHeadChunk;
    int run = chunk_off[blockIdx.x];
    for (int it = 0; it < kHeadIters; ++it) {
        const int64_t e = base + (int64_t)it * kBlock + threadIdx.x;
        uint64_t x = 0;
        const bool h = is_head<kTshift>(ent, e, nvalid, &x);
        const uint64_t b = ballot(h);
        if (lane == 0) wcnt[wid] = __popcll(b);
        __syncthreads();
        int before = run, total = run;
        for (int q = 0; q < kBlock / kWave; ++q) {
            if (q < wid) before += wcnt[q];
            total += wcnt[q];
        }
        if (h) {
            const int t = before + __popcll(b & lanes_below());
            tile_start[t] = (int32_t)e;
            tile_col[t] = (int32_t)(((x >> 5) & 0x7FFFFFFFull) >> kTshift);
        }
        run = total;
        __syncthreads();
    }
}

// Tile bitmaps, the rows with entries and the tiles of each row-block.  A wavefront
// takes 64 consecutive tiles, reads their sorted entries together (coalesced), finds
// each entry's tile by a binary search over the 64 tile starts in LDS, ORs the
// entry's bit into that tile's bitmap in LDS (a tile's first entry also gives its
// row-block), and writes the 64 bitmaps out as one contiguous run.  Bit (row r,
// column c) of a tile is bit r * T + c of its words.  Lanes of one row-block
// combine their rows into hrows and their tile count into rb_cnt, one atomic each.
template <int T>
__global__ void __launch_bounds__(kBlock) k_tile_bits(const uint64_t* ent, const int32_t* tile_start,
                                                      const Meta* meta, uint32_t* bits, uint32_t* hrows,
                                                      int64_t* rb_cnt) {
    constexpr int W = T * T / 32;   // bitmap words per tile
    constexpr int kWpb = kBlock / kWave;
    __shared__ uint32_t sbits[kWpb][kWave * W];
    __shared__ int32_t sstart[kWpb][kWave];
    __shared__ int32_t srow[kWpb][kWave];
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    uint32_t* sb = sbits[wid];
    int32_t* ss = sstart[wid];
    int32_t* sr = srow[wid];
    const int64_t nt = meta->ntiles, nvalid = meta->nvalid;
    const int64_t ntask = (nt + kWave - 1) / kWave;
    const int64_t tstride = (int64_t)gridDim.x * kWpb;
    // a task's tile starts and entry bound, loaded one task ahead
    int32_t n_start = 0;
    int64_t n_hi = 0;
    auto fetch = [&](int64_t task) {
        if (task >= ntask) return;
        const int64_t t0 = task * kWave;
        const int ntl = (int)min<int64_t>(kWave, nt - t0);
        n_start = lane < ntl ? tile_start[t0 + lane] : 0x7FFFFFFF;
        n_hi = t0 + ntl < nt ? (int64_t)tile_start[t0 + ntl] : nvalid;
    };
    int64_t task = (int64_t)blockIdx.x * kWpb + wid;
    fetch(task);
    for (; task < ntask; task += tstride) {
        const int64_t t0 = task * kWave;
        const int ntl = (int)min<int64_t>(kWave, nt - t0);   // tiles of this task
        const int32_t start = n_start;
        const int64_t e_hi = n_hi;
        fetch(task + tstride);
        const int64_t e_lo = __shfl(start, 0, kWave);
        ss[lane] = start;
        #pragma unroll
        for (int q = 0; q < W; ++q) sb[q * kWave + lane] = 0;
        wave_sync_lds();
        for (int64_t eb = e_lo; eb < e_hi; eb += 4 * kWave) {
            uint64_t xs[4];
            #pragma unroll
            for (int u = 0; u < 4; ++u) {   // four entry loads in flight per lane
                const int64_t e = eb + u * kWave + lane;
                xs[u] = e < e_hi ? ent[e] : 0;
            }
            #pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t e = eb + u * kWave + lane;
                if (e < e_hi) {
                    int lo = 0, hi = ntl - 1;   // the last tile whose start is <= e
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (ss[mid] <= e) lo = mid; else hi = mid - 1;
                    }
                    const uint64_t x = xs[u];
                    const int b = (int)((x & (T - 1)) * T + ((x >> 5) & (T - 1)));
                    atomicOr(&sb[lo * W + (b >> 5)], 1u << (b & 31));
                    if (e == ss[lo]) sr[lo] = (int32_t)(x >> 36);   // the tile's first entry
                }
            }
        }
        wave_sync_lds();
        // the task's bitmaps: one contiguous run of ntl * W words, 16 bytes per store
        uint4* dst = reinterpret_cast<uint4*>(bits + t0 * W);
        const uint4* src = reinterpret_cast<const uint4*>(sb);
        for (int k = lane; k < ntl * W / 4; k += kWave) dst[k] = src[k];
        uint32_t rm = 0;
        if (lane < ntl) {
            #pragma unroll
            for (int j = 0; j < W; ++j) {
                const uint32_t wj = sb[lane * W + j];
                if (T == 16) {
                    rm |= (uint32_t)((wj & 0xFFFFu) != 0) << (2 * j);
                    rm |= (uint32_t)((wj >> 16) != 0) << (2 * j + 1);
                } else {
                    rm |= (uint32_t)(wj != 0) << j;
                }
            }
        }
        const int32_t row = lane < ntl ? sr[lane] : -1;
        run_or(row, rm, hrows);
        // tiles of each row-block in the task: from a run's first lane to the next run's
        const bool first = lane < ntl && (lane == 0 || sr[lane - 1] != row);
        const uint64_t firsts = ballot(first);
        if (first) {
            const uint64_t above = lane == kWave - 1 ? 0ull : firsts & (~0ull << (lane + 1));
            const int next = above ? __ffsll((long long)above) - 1 : ntl;
            atomicAdd((unsigned long long*)&rb_cnt[row], (unsigned long long)(next - lane));
        }
        wave_sync_lds();   // the next task clears sb
    }
}

// chunks of each row-block (at most tpi tiles each)
// chunks per row-block; also marks every slot of the round-1 list a hole (r1 has
// r1_len slots), before the chunk fill writes the chunks
__global__ void k_chunk_count(const int64_t* rb_ptr, int64_t nI, int tpi, int64_t* cnt, uint64_t* r1, int64_t r1_len) {
    GRID_STRIDE(I, nI) cnt[I] = (rb_ptr[I + 1] - rb_ptr[I] + tpi - 1) / tpi;
    GRID_STRIDE(q, r1_len) r1[q] = kChunkHole;
}

// chunk q belongs to the last row-block whose first chunk is <= q
// every chunk of the round-1 list twice over: in row-block order (out), and with each
// row-block's first chunk ahead of all later ones (r1: first chunks at [I], later
// chunks at nI + their index, holes elsewhere), so that round 1 settles most
// row-blocks before their later chunks are reached and those are skipped
// (first[nI], the end of the last row-block's range, is written here too; the
// searches read first[0 .. nI - 1] only)
__global__ void k_chunk_fill(int64_t* first, const int64_t* rb_ptr, const Meta* meta, int64_t nI, int tpi,
                             int64_t cap, uint64_t* out, uint64_t* r1) {
    const int64_t total = meta->nchunks;
    if (blockIdx.x == 0 && threadIdx.x == 0) first[nI] = total;
    GRID_STRIDE(q, cap) {
        if (q >= total) break;
        int64_t lo = 0, hi = nI - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (first[mid] <= q) lo = mid; else hi = mid - 1;
        }
        const int64_t t0 = rb_ptr[lo] + (q - first[lo]) * tpi;
        const uint64_t w = chunk_word(t0, min((int64_t)tpi, rb_ptr[lo + 1] - t0), lo);
        out[q] = w;
        r1[q == first[lo] ? lo : nI + q] = w;
    }
}

__global__ void k_permute_keys(const uint64_t* key, const int32_t* new_id, int64_t n, uint64_t* key_p) {
    GRID_STRIDE(v, n) key_p[new_id[v]] = key[v];
}

__global__ void k_light_flags(const int64_t* rp, int64_t n, int32_t* flag) {
    GRID_STRIDE(v, n) flag[v] = (rp[v + 1] - rp[v] <= kLightDeg) ? 1 : 0;
}

__global__ void k_csr_lists(const int64_t* rp, const int32_t* pos, int64_t n, int32_t* light, int32_t* heavy) {
    GRID_STRIDE(v, n) {
        if (rp[v + 1] - rp[v] <= kLightDeg) light[pos[v]] = (int32_t)v;
        else heavy[v - pos[v]] = (int32_t)v;
    }
}

int bits_for(int64_t x) {   // bits to hold 0..x, so x itself is never all ones
    int b = 1;
    while ((1ll << b) <= x) ++b;
    return b;
}

#define LAUNCH(kernel, work, ...)                                                                          \
    do {                                                                                                   \
        if ((work) > 0) hipLaunchKernelGGL(kernel, dim3(stream_grid(work)), dim3(kBlock), 0, s, __VA_ARGS__); \
        TC_HIP(hipGetLastError());                                                                         \
    } while (0)

}  // namespace

int host_rcm(const int64_t* rp, const int32_t* ci, int64_t n, std::vector<int32_t>& new_id);
int64_t hyb_blocks(int64_t nnz);
int64_t dyn_counter_words();

namespace {
// hands out 256-byte aligned arrays from base (base == nullptr: sizes only)
struct Carver {
    char* base;
    size_t off = 0;
    template <typename P>
    void take(P** p, size_t bytes) {
        off = (off + 255) & ~(size_t)255;
        if (base) *p = reinterpret_cast<P*>(base + off);
        off += bytes ? bytes : 8;
    }
};
}  // namespace

size_t layout_state(GraphCore* g, char* base, bool with_trace) {
    Carver c{base};
    const int64_t n = g->n;
    // ctrl, the sizes and the trace ring first and together: a solve reads them back
    // with one copy
    c.take(&g->ctrl, sizeof(Ctrl));
    c.take(&g->smeta, sizeof(Meta));
    if (with_trace) c.take(&g->trace, sizeof(TraceRec) * kTraceCap);
    else g->trace = nullptr;
    c.take(&g->stripes, sizeof(int64_t) * 2 * kStripes * kStripeWords);
    if (g->count > 0) {
        c.take(&g->g_rounds, (size_t)g->count * 4);
        c.take(&g->g_in, (size_t)g->count * 8);
    }
    if (g->path == MIS_PATH_HYBRID) {
        const int64_t nI = ceil_div(n, 16), nw = ceil_div(n, 64) * 2 + 2;   // bitmap words (whole waves)
        c.take(&g->hA, (size_t)nw * 4);
        c.take(&g->hS, (size_t)nw * 4);
        if (g->dyn_slack == 0) c.take(&g->hblk, (size_t)n * 4);
        else g->hblk = nullptr;
        for (int b = 0; b < 2; ++b) c.take(&g->hdact[b], (size_t)(g->dense_min > 0 ? nI : 0) * 4);
        if (g->count > 0) c.take(&g->dround, (size_t)n * 4);
    } else if (g->path == MIS_PATH_CSR) {
        for (int b = 0; b < 2; ++b)
            for (int k = 0; k < 2; ++k) c.take(&g->act[b][k], (size_t)n * 4);
        c.take(&g->st, (size_t)n * 4);
        c.take(&g->ak, (size_t)n * 8);
    } else {
        const int T = g->tile;
        const int64_t nI = ceil_div(n, T);
        const int64_t chunk_cap = (g->orient ? g->nnz / 2 + 1 : g->nnz + 1) / (T == 16 ? 64 : 16) + nI + 1;
        for (int b = 0; b < 2; ++b) {
            c.take(&g->chunks[b], (size_t)chunk_cap * 8);
            c.take(&g->rbl[b], (size_t)nI * 4);
        }
        c.take(&g->rs, (size_t)nI * 8);
        c.take(&g->hit, (size_t)nI * 4);
        c.take(&g->inmask, (size_t)nI * 4);
        c.take(&g->dround, (size_t)nI * T * 4);
    }
    return (c.off + 255) & ~(size_t)255;
}

size_t layout(GraphCore* g, char* base) {
    Carver c{base};
    const int64_t n = g->n, nnz = g->nnz;
    c.take(&g->meta, sizeof(Meta));
    c.take(&g->key, (size_t)n * 8);
    if (g->count > 0) c.take(&g->goff, (size_t)(g->count + 1) * 8);
    c.take(&g->scan_tmp, (size_t)scan_scratch_elems(std::max(n, nnz) + 1) * 8);
    if (g->path == MIS_PATH_HYBRID) {
        g->nI = ceil_div(n, 16);
        const int64_t nI = g->nI, nw = ceil_div(n, 64) * 2 + 2;   // bitmap words (whole waves)
        c.take(&g->q8, (size_t)n);
        // H rows (static handles: those of the vertices round 1 leaves undecided, at
        // their input row starts; dynamic handles: every row, with slack)
        const int64_t rows = g->dyn_slack > 0 ? nnz + n * (int64_t)g->dyn_slack : nnz;   // slots per orientation
        c.take(&g->hcol, (size_t)rows * 4);
        c.take(&g->hcnt, (size_t)n * 4);
        if (g->dyn_slack > 0) {
            c.take(&g->hbrow, (size_t)(hyb_blocks(nnz) + 2) * 4);
            c.take(&g->hbase, (size_t)n * 4);
            c.take(&g->hoff, (size_t)n * 4);
            c.take(&g->drp, (size_t)(n + 1) * 8);
            c.take(&g->lcol, (size_t)rows * 4);
            c.take(&g->lcnt, (size_t)n * 4);
            c.take(&g->hloff, (size_t)n * 4);
            c.take(&g->rS, (size_t)nw * 4);
            c.take(&g->rP, (size_t)nw * 4);
            c.take(&g->rC, (size_t)nw * 4);
            c.take(&g->rlist[0], (size_t)n * 4);
            c.take(&g->rlist[1], (size_t)n * 4);
            c.take(&g->rflip, (size_t)n * 4);
            c.take(&g->rdec, (size_t)n * 4);
            c.take(&g->rcnt, (size_t)dyn_counter_words() * 8);
            c.take(&g->hflag, (size_t)n * 8);
        }
        if (g->dense_min > 0) {
            const int64_t tcap = nnz / 2 + 1;   // a dense tile holds at least one oriented entry
            c.take(&g->dsamp, (size_t)kGateSamples * 4);
            c.take(&g->dslot, (size_t)nI * 4);
            c.take(&g->drb, (size_t)nI * 4);
            c.take(&g->dptr, (size_t)(nI + 1) * 4);
            c.take(&g->dcol, (size_t)tcap * 4);
            c.take(&g->dbits, (size_t)tcap * 32);
        }
    } else if (g->path == MIS_PATH_CSR) {
        c.take(&g->light, (size_t)n * 4);
        c.take(&g->heavy, (size_t)n * 4);
        c.take(&g->flag32, (size_t)n * 4);
    } else {
        const int T = g->tile;
        g->nI = ceil_div(n, T);
        const int64_t nI = g->nI;
        g->tile_cap = g->orient ? nnz / 2 + 1 : nnz + 1;
        g->chunk_cap = g->tile_cap / (T == 16 ? 64 : 16) + nI + 1;
        const int64_t cap = g->tile_cap;
        c.take(&g->new_id, (size_t)n * 4);
        c.take(&g->order, (size_t)n * 4);
        c.take(&g->sk, (size_t)n * 8);
        c.take(&g->sk2, (size_t)n * 8);
        c.take(&g->pl, (size_t)n * 4);
        c.take(&g->pl2, (size_t)n * 4);
        c.take(&g->sort_tmp, sort_scratch_bytes(std::max(n, nnz)));
        c.take(&g->ndeg, (size_t)(n + 1) * 4);
        c.take(&g->brow, (size_t)(ceil_div(nnz, kEntBlock) + 2) * 4);
        c.take(&g->ent, (size_t)nnz * 8);
        c.take(&g->ent2, (size_t)nnz * 8);
        c.take(&g->hsums, (size_t)(ceil_div(nnz, 2048) + 2) * 4);
        c.take(&g->ecnt, (size_t)(ceil_div(nnz, kEntBlock) + 1) * 4);
        c.take(&g->rb_ptr, (size_t)(nI + 1) * 8);
        c.take(&g->rb_chunk, (size_t)(nI + 1) * 8);
        c.take(&g->tile_col, (size_t)cap * 4);
        c.take(&g->tile_start, (size_t)cap * 4);
        c.take(&g->tile_bits, (size_t)cap * (T * T / 32) * 4);
        if (!g->orient) c.take(&g->key_p, (size_t)nI * T * 8);
        c.take(&g->hrows, (size_t)nI * 4);
        c.take(&g->chunks_all, (size_t)g->chunk_cap * 8);
        c.take(&g->chunks_r1, (size_t)(nI + g->chunk_cap) * 8);
    }
    // the handle's own round state follows the structure
    const size_t so = (c.off + 255) & ~(size_t)255;
    g->state_off = so;
    return so + layout_state(g, base ? base + so : nullptr);
}

int validate_graph(const mis_csr* csr, const uint64_t* user_keys, const int64_t* goff, int64_t count, uint32_t* d_err,
                   hipStream_t s) {
    TC_HIP(hipMemsetAsync(d_err, 0, 4, s));
    int64_t ends[2] = {0, 0};
    TC_HIP(hipMemcpyAsync(&ends[0], csr->row_ptr, 8, hipMemcpyDeviceToHost, s));
    TC_HIP(hipMemcpyAsync(&ends[1], csr->row_ptr + csr->n, 8, hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    if (ends[0] != 0 || ends[1] != csr->nnz) {
        set_error("row_ptr[0] must be 0 and row_ptr[n] must equal nnz");
        return MIS_ERANGE;
    }
    LAUNCH(k_validate_rows, csr->n, csr->row_ptr, csr->n, csr->nnz, d_err);
    uint32_t h = 0;
    TC_HIP(hipMemcpyAsync(&h, d_err, 4, hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    if (h) { set_error("row_ptr is not monotone within [0, nnz]"); return MIS_ERANGE; }
    LAUNCH(k_validate_edges, csr->nnz, csr->row_ptr, csr->col_idx, csr->n, csr->nnz, user_keys, goff, count, d_err);
    TC_HIP(hipMemcpyAsync(&h, d_err, 4, hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    if (h & kErrRange) { set_error("column index out of range"); return MIS_ERANGE; }
    if (h & kErrLoop) { set_error("self-loop"); return MIS_ESELFLOOP; }
    if (h & kErrDup) { set_error("duplicate or unsorted adjacency entries"); return MIS_EDUP; }
    if (h & kErrAsym) { set_error("adjacency is not symmetric"); return MIS_ENOTSYM; }
    if (h & kErrTie) { set_error("two adjacent vertices have equal keys"); return MIS_EINVAL; }
    if (h & kErrCross) { set_error("an edge joins two graphs of the batch"); return MIS_EINVAL; }
    return MIS_OK;
}

// default keys of a single graph hold the vertex id in their low 24 bits: the order
// sort then moves the keys alone and the order is read back from them
bool default_keys_in_order(const mis_graph* g) {
    return g->reorder == MIS_REORDER_KEY && !g->user_keys && g->count == 0 && g->n <= (1 << 24);
}

int build_keys(mis_graph* g, const mis_build_opts* o, hipStream_t s) {
    if (g->n == 0) return MIS_OK;
    if (o->keys) {
        TC_HIP(hipMemcpyAsync(g->key, o->keys, (size_t)g->n * 8, hipMemcpyDeviceToDevice, s));
    } else {
        // the key order of one graph with default keys: the sort keys come with the keys
        uint64_t* sk = g->path == MIS_PATH_TILE && default_keys_in_order(g) ? g->sk : nullptr;
        const bool hyb = g->path == MIS_PATH_HYBRID;
        const bool sample = hyb && g->dense_min > 0 && g->nnz > 0;   // the dense-block sample
        // a batch takes kKeysSpan vertices per workgroup (see k_keys)
        const unsigned grid = g->count > 0 ? (unsigned)std::min<int64_t>(ceil_div(g->n, kKeysSpan), 65536)
                                           : stream_grid(g->n);
        hipLaunchKernelGGL(k_keys, dim3(grid), dim3(kBlock), 0, s, g->row_ptr, g->n, o->seed,
                           g->count > 0 ? g->goff : nullptr, (int64_t)g->count, o->key_rule, g->key, sk,
                           hyb ? g->q8 : nullptr, hyb ? g->meta : nullptr, g->col_idx, dense_stride(g->nI),
                           dense_samples(g->nI), g->dense_min, sample ? g->dsamp : nullptr);
        TC_HIP(hipGetLastError());
    }
    return MIS_OK;
}

int build_csr_lists(mis_graph* g, hipStream_t s) {
    const int64_t n = g->n;
    TC_HIP(hipMemsetAsync(g->meta, 0, sizeof(Meta), s));
    LAUNCH(k_light_flags, n, g->row_ptr, n, g->flag32);
    TC_CHECK(scan_excl_i32(g->flag32, g->flag32, n, &g->meta->n_light, (int32_t*)g->scan_tmp, s));
    LAUNCH(k_csr_lists, n, g->row_ptr, g->flag32, n, g->light, g->heavy);
    return MIS_OK;
}


int build_order(mis_graph* g, hipStream_t s) {
    const int64_t n = g->n;
    if (n == 0) return MIS_OK;
    if (g->reorder == MIS_REORDER_NONE) {
        LAUNCH(k_identity_order, n, g->row_ptr, g->order, g->new_id, g->ndeg, n);
        return MIS_OK;
    }
    if (g->reorder == MIS_REORDER_RCM) {
        std::vector<int64_t> rp(n + 1);
        std::vector<int32_t> ci(g->nnz);
        TC_HIP(hipMemcpyAsync(rp.data(), g->row_ptr, (n + 1) * 8, hipMemcpyDeviceToHost, s));
        if (g->nnz) TC_HIP(hipMemcpyAsync(ci.data(), g->col_idx, g->nnz * 4, hipMemcpyDeviceToHost, s));
        TC_HIP(hipStreamSynchronize(s));
        std::vector<int32_t> nid;
        TC_CHECK(host_rcm(rp.data(), ci.data(), n, nid));
        TC_HIP(hipMemcpyAsync(g->new_id, nid.data(), n * 4, hipMemcpyHostToDevice, s));
        LAUNCH(k_invert, n, g->row_ptr, g->new_id, g->order, g->ndeg, n);
        TC_HIP(hipStreamSynchronize(s));   // nid is freed on return
        return MIS_OK;
    }
    const bool ids_in_key = default_keys_in_order(g);
    if (!ids_in_key)   // (with default keys of one graph k_keys wrote the sort keys)
        LAUNCH(k_order_keys, n, g->row_ptr, g->key, n, g->reorder, g->sk, g->pl);
    bool alt = false;
    const int lo = g->reorder == MIS_REORDER_DEGREE ? 0 : (g->user_keys ? 0 : 24);
    const int hi = g->reorder == MIS_REORDER_DEGREE ? 8 : 64;
    if (ids_in_key) {
        // bits 34..63 (degree class and 22 hash bits) in three 10-bit passes, then the
        // runs that tie on them are ordered on the rest (10 hash bits and the id)
        constexpr int kTieBits = 34;
        TC_CHECK(radix_sort_u64(g->sk, g->sk2, nullptr, nullptr, n, nullptr, kTieBits, hi, g->sort_tmp, &alt, s));
        LAUNCH(k_scatter_order_keys, n, g->row_ptr, alt ? g->sk2 : g->sk, n, kTieBits, g->order, g->new_id, g->ndeg);
        return MIS_OK;
    }
    TC_CHECK(radix_sort_u64(g->sk, g->sk2, g->pl, g->pl2, n, nullptr, lo, hi, g->sort_tmp, &alt, s));
    LAUNCH(k_scatter_order, n, g->row_ptr, alt ? g->pl2 : g->pl, n, g->order, g->new_id, g->ndeg);
    return MIS_OK;
}

template <int T>
int build_tiles_t(mis_graph* g, hipStream_t s) {
    constexpr int kTshift = T == 16 ? 4 : 5;
    const int64_t n = g->n, nnz = g->nnz, nI = g->nI;
    // with entries, every Meta field is the total of a scan below before anything reads it
    if (nnz == 0) TC_HIP(hipMemsetAsync(g->meta, 0, sizeof(Meta), s));
    // 1. new row pointer (the degrees in new order were written with the order)
    TC_CHECK(scan_excl_i32(g->ndeg, g->ndeg, n, g->ndeg + n, (int32_t*)g->scan_tmp, s));
    // 2. entries in new-row order, one lane per entry
    const int mode = !g->orient ? 0 : (g->reorder == MIS_REORDER_KEY ? 1 : 2);
    const int64_t eblocks = ceil_div(nnz, kEntBlock);
    if (nnz > 0) {
        LAUNCH(k_block_rows, eblocks + 1, g->ndeg, n, nnz, eblocks, g->brow);
        const dim3 grid((unsigned)eblocks), blk(kBlock);
#define TC_ENTRIES(M)                                                                                     \
    hipLaunchKernelGGL((k_entries<kTshift, M>), grid, blk, 0, s, g->row_ptr, g->col_idx, g->order, g->ndeg, \
                       g->brow, g->new_id, g->key, nnz, g->ent, g->ecnt)
        if (mode == 0) TC_ENTRIES(0);
        if (mode == 1) TC_ENTRIES(1);
        if (mode == 2) TC_ENTRIES(2);
#undef TC_ENTRIES
        TC_HIP(hipGetLastError());
        // number of kept entries
        TC_CHECK(scan_excl_i32(g->ecnt, g->hsums, eblocks, &g->meta->nvalid, (int32_t*)g->scan_tmp, s));
    }
    // 3. stable sort of the kept entries on the row-block of the transposed entry
    bool alt = false;
    if (nnz > 0)
        TC_CHECK(radix_sort_u64(g->ent, g->ent2, nullptr, nullptr, nnz, g->ecnt, 36,
                                36 + bits_for(std::max<int64_t>(nI - 1, 1)), g->sort_tmp, &alt, s));
    const uint64_t* sorted = alt ? g->ent2 : g->ent;
    // 4. tiles: count heads per chunk, scan, write tile heads; then the bitmaps and
    //    the rows with entries; row-block tile ranges
    const int64_t nheads = ceil_div(nnz, kHeadChunk);
    if (nheads > 0) {
        hipLaunchKernelGGL((k_head_count<kTshift>), dim3((unsigned)nheads), dim3(kBlock), 0, s, sorted, g->meta,
                           g->hsums, g->hrows, g->rb_ptr, nI);
        TC_HIP(hipGetLastError());
        TC_CHECK(scan_excl_i32(g->hsums, g->hsums, nheads, &g->meta->ntiles, (int32_t*)g->scan_tmp, s));
        hipLaunchKernelGGL((k_head_write<kTshift>), dim3((unsigned)nheads), dim3(kBlock), 0, s, sorted, g->meta,
                           g->hsums, g->tile_start, g->tile_col);
        TC_HIP(hipGetLastError());
    }
    if (nheads == 0) {   // else cleared by the head count
        TC_HIP(hipMemsetAsync(g->hrows, 0, (size_t)nI * 4, s));
        TC_HIP(hipMemsetAsync(g->rb_ptr, 0, (size_t)(nI + 1) * 8, s));
    }
    if (nheads > 0) {   // one wavefront per 64 tiles (the tile count is on the device: sized by capacity)
        const int64_t blocks = std::min<int64_t>(ceil_div(ceil_div(g->tile_cap, kWave), kBlock / kWave), 8192);
        hipLaunchKernelGGL((k_tile_bits<T>), dim3((unsigned)blocks), dim3(kBlock), 0, s, sorted, g->tile_start,
                           g->meta, g->tile_bits, g->hrows, g->rb_ptr);
        TC_HIP(hipGetLastError());
    }
    // row-block tile counts -> each row-block's first tile (rb_ptr[nI] = all tiles)
    TC_CHECK(scan_excl_i64(g->rb_ptr, g->rb_ptr, nI + 1, (int64_t*)nullptr, (int64_t*)g->scan_tmp, s));
    // 5. the round-1 chunk list: every row-block's tiles in chunks of kTpi; rb_chunk
    //    holds each row-block's first chunk
    constexpr int kTpi = T == 16 ? 64 : 16;
    LAUNCH(k_chunk_count, nI, g->rb_ptr, nI, kTpi, g->rb_chunk, g->chunks_r1, nI + g->chunk_cap);
    TC_CHECK(scan_excl_i64(g->rb_chunk, g->rb_chunk, nI, &g->meta->nchunks, (int64_t*)g->scan_tmp, s));
    LAUNCH(k_chunk_fill, g->chunk_cap, g->rb_chunk, g->rb_ptr, g->meta, nI, kTpi, g->chunk_cap, g->chunks_all,
           g->chunks_r1);
    if (!g->orient) {
        TC_HIP(hipMemsetAsync(g->key_p, 0, (size_t)nI * T * 8, s));
        LAUNCH(k_permute_keys, n, g->key, g->new_id, n, g->key_p);
    }
    return MIS_OK;
}

int build_tiles(mis_graph* g, hipStream_t s) {
    return g->tile == 16 ? build_tiles_t<16>(g, s) : build_tiles_t<32>(g, s);
}

}  // namespace tcmis
