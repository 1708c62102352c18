// Hybrid path: the rounds of Algorithm 2 over the edges to higher-priority
// neighbours, stored per 16-row block of the input order either as nonzero 16 x 16
// bit tiles (Section 3.2) or as sorted entry lists (Section 3.2, "Memory Footprint
// and Representation Trade-offs": a tile only pays where it holds enough edges).
//
// Why only higher-priority neighbours.  A candidate neighbour of an undecided
// vertex always out-ranks it (a candidate beats every undecided neighbour), and
// Phase 1 only asks whether an undecided neighbour out-ranks the vertex.  So both
// phases read only H(v) = { u in N(v) : key(u) > key(v) }, half the adjacency, and
// neither reads a key:
//   Phase 1  C(v) = alive(v) and no u in H(v) is alive
//   Phase 2  v leaves the undecided set if some u in H(v) joined the set this round
// With the in-set bitmap S, "joined this round" is simply S(u): a neighbour that
// joined in an earlier round would already have removed v.
//
// Build (no reordering, no global sort):
//   1. keys and the one-byte degree class q(v) of every vertex (k_keys);
//   2. orientation (k_orient): every adjacency entry (v, u) is compared by priority;
//      the higher-priority ones are compacted into row v's own range of the input
//      column array's layout, hcol[rp[v] .. rp[v] + hcnt[v]).  Workgroups take
//      2048 entries each; a row split between workgroups gets its pieces with one
//      atomic add per piece (the order inside such a row is unspecified, the set is
//      not).  Comparing the degree class decides most pairs from a 1-byte table;
//      only on a tie is the neighbour's hash rebuilt in registers;
//   3. dense blocks (optional): a wave per 16-row block gathers its oriented
//      entries, sorts their column blocks in LDS and counts the nonzero tiles; blocks
//      that average at least dense_min entries per tile (at most 64 tiles) are
//      written as bitmaps;
//   4. lists: round 1's candidates are the vertices with no higher-priority
//      neighbour (known from the orientation, so round 1 has no Phase-1 pass);
//      the other rows of entry-list blocks go to a light list (at most kHLight
//      entries: a lane each) or a heavy list (a wavefront each).
//
// Round r (two kernels):
//   P1  (r >= 2)  for every listed row: scan H(v) for an alive neighbour (early
//       exit); dense blocks: blocked rows = H x alive on the matrix cores (int8 x
//       int8 -> int32, exact); candidates set their S bit.
//   P2  listed rows: S(v) -> IN; else scan H(v) for an S neighbour -> OUT; dense
//       blocks: N_c = H x S on the matrix cores.  Decided vertices clear their
//       alive bit; the rest go to the next round's lists.
// P1 only reads alive and writes S; P2 only reads S and writes alive; every hand-over
// crosses a kernel boundary (or a grid barrier in the persistent kernel).
#include "round.hpp"

namespace tcmis {

namespace {

constexpr int kHE = 2048;                 // adjacency entries per orientation workgroup
constexpr int kHIters = kHE / kBlock;     // entries per thread
constexpr int kHWin = 512;                // rows a workgroup stages in LDS
constexpr int kHSteps = 9;                // 2^kHSteps = kHWin
constexpr int kHLight = 32;               // rows with at most this many entries take one lane
constexpr int kDenseCap = 1024;           // most oriented entries a block may hold to be dense
constexpr int kDenseTiles = 64;           // most tiles of a dense block (one per lane)
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

// first row of every orientation workgroup's entry range (the last slot: the row of
// the last entry)
__global__ void k_orient_rows(const int64_t* rp, int64_t n, int64_t nnz, int64_t nblocks, int32_t* brow) {
    GRID_STRIDE(b, nblocks + 1) {
        const int64_t e = b < nblocks ? b * kHE : nnz - 1;
        int64_t lo = 0, hi = n - 1;   // largest row whose start is <= e
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (rp[mid] <= e) lo = mid; else hi = mid - 1;
        }
        brow[b] = (int32_t)lo;
    }
}

// does column u out-rank row v?  kUserKeys: compare the keys; else the default key
// rule: the degree class decides unless it ties, then the hash of the graph-local
// id, then the id (kv is row v's whole key, so its class, hash and local id are known)
template <bool kUserKeys>
__device__ inline bool higher(int64_t u, int64_t v, uint64_t kv, const uint64_t* key, const uint8_t* q8, uint64_t seed) {
    if (kUserKeys) return key[u] > kv;
    const uint32_t qu = q8[u], qv = (uint32_t)(kv >> 56);
    if (qu != qv) return qu > qv;
    const int64_t lv = (int64_t)(kv & 0xFFFFFFull);
    const int64_t lu = u - (v - lv);   // same graph: same offset
    const uint32_t hu = (uint32_t)(splitmix_at(seed, (uint64_t)lu + 1) >> 32);
    const uint32_t hv = (uint32_t)(kv >> 24);
    return hu != hv ? hu > hv : lu > lv;
}

// Orientation.  Workgroup b takes entries [b*kHE, (b+1)*kHE), thread t entries
// b*kHE + it*kBlock + t.  With the workgroup's rows staged in LDS (row starts
// relative to the range, row keys), each thread finds its entries' rows with a
// fixed-step search, issues its column reads, then its degree-class gathers.  The
// kept entries of a row piece are ranked by a workgroup prefix count in entry
// order; a row wholly inside the range is written from its row start, a piece of a
// longer row from the offset its atomic add returned.
// Where the orientation writes: the higher-priority entries of row v go to
// hcol[hrp[v] + ...] (hrp = the input row pointer, or the dynamic layout's own);
// with lcol (dynamic handles) the lower-priority ones go to lcol[hrp[v] + ...].
struct OrientOut {
    const int64_t* hrp;
    int32_t* hcol;
    int32_t* hcnt;
    int32_t* lcol;      // nullptr: higher-priority entries only
    int32_t* lcnt;
    int32_t* g_base;    // [n] scratch of workgroups whose rows exceed LDS
    int32_t* g_off;
    int32_t* g_loff;
};

template <bool kUserKeys, bool kLds>
__device__ void orient_body(const int64_t* rp, const int32_t* ci, const uint64_t* key, const uint8_t* q8,
                            uint64_t seed, int64_t nnz, int64_t u0, int64_t u1, const OrientOut& o, int32_t* wst,
                            uint64_t* wkey, int32_t* wbase, int32_t* woff, int32_t* wloff) {
    int32_t* g_base = o.g_base;
    int32_t* g_off = o.g_off;
    int32_t* hcnt = o.hcnt;
    __shared__ int32_t wcnt[kHIters][kWpb];
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    const int64_t base = (int64_t)blockIdx.x * kHE;
    const int64_t end = min(nnz, base + kHE);
    const int w = (int)(u1 - u0 + 1);
    int li[kHIters];   // row of each entry, relative to u0
    int32_t cu[kHIters];
    #pragma unroll
    for (int it = 0; it < kHIters; ++it) {
        const int64_t e = min(base + it * kBlock + (int64_t)threadIdx.x, end - 1);
        if (kLds) {
            const int32_t er = (int32_t)(e - base);
            int lo = 0;   // wst[0] <= 0 <= er
            #pragma unroll
            for (int k = kHSteps - 1; k >= 0; --k) {
                const int c = lo + (1 << k);
                const int32_t wc = wst[min(c, w - 1)];
                lo = ((c <= w - 1) & (wc <= er)) ? c : lo;
            }
            li[it] = lo;
        } else {
            int64_t lo = u0, hi = u1;
            while (lo < hi) {
                const int64_t mid = (lo + hi + 1) >> 1;
                if (rp[mid] <= e) lo = mid; else hi = mid - 1;
            }
            li[it] = (int)(lo - u0);
        }
    }
    #pragma unroll
    for (int it = 0; it < kHIters; ++it) {
        const int64_t e = min(base + it * kBlock + (int64_t)threadIdx.x, end - 1);
        cu[it] = __builtin_nontemporal_load(&ci[e]);
    }
    uint32_t keep = 0;   // bit it: entry it is kept
    #pragma unroll
    for (int it = 0; it < kHIters; ++it) {
        const int64_t e = base + it * kBlock + (int64_t)threadIdx.x;
        const int64_t v = u0 + li[it];
        const uint64_t kv = kLds ? wkey[li[it]] : key[v];
        if (e < end && higher<kUserKeys>(cu[it], v, kv, key, q8, seed)) keep |= 1u << it;
    }
    #pragma unroll
    for (int it = 0; it < kHIters; ++it) {
        const uint64_t b = ballot((keep >> it) & 1u);
        if (lane == 0) wcnt[it][wid] = __popcll(b);
    }
    __syncthreads();
    // exclusive prefix count of kept entries at each of the thread's entries
    int32_t pre[kHIters];
    {
        int run = 0;
        #pragma unroll
        for (int it = 0; it < kHIters; ++it) {
            int before = run, total = run;
            for (int q = 0; q < kWpb; ++q) {
                if (q < wid) before += wcnt[it][q];
                total += wcnt[it][q];
            }
            const uint64_t b = ballot((keep >> it) & 1u);
            pre[it] = before + __popcll(b & lanes_below());
            run = total;
        }
    }
    // a row piece's first entry records the prefix there
    #pragma unroll
    for (int it = 0; it < kHIters; ++it) {
        const int64_t e = base + it * kBlock + (int64_t)threadIdx.x;
        const int64_t v = u0 + li[it];
        if (e < end && e == max(rp[v], base)) {
            if (kLds) wbase[li[it]] = pre[it]; else g_base[v] = pre[it];
        }
    }
    __syncthreads();
    // a row piece's last entry: its kept count; a whole row stores it, a piece adds it
    // (and the same for the lower-priority entries of a dynamic handle)
    #pragma unroll
    for (int it = 0; it < kHIters; ++it) {
        const int64_t e = base + it * kBlock + (int64_t)threadIdx.x;
        const int64_t v = u0 + li[it];
        if (e < end) {
            const int64_t r0 = rp[v], r1 = rp[v + 1];
            if (e == min(r1, end) - 1) {
                const int32_t b0 = kLds ? wbase[li[it]] : g_base[v];
                const int32_t cnt = pre[it] + (int32_t)((keep >> it) & 1u) - b0;
                const int32_t lc = (int32_t)(e + 1 - max(r0, base)) - cnt;
                const bool whole = r0 >= base && r1 <= end;
                int32_t off = 0, loff = 0;
                if (whole) hcnt[v] = cnt;
                else if (cnt > 0) off = atomicAdd(&hcnt[v], cnt);
                if (o.lcol) {
                    if (whole) o.lcnt[v] = lc;
                    else if (lc > 0) loff = atomicAdd(&o.lcnt[v], lc);
                }
                if (kLds) { woff[li[it]] = off; wloff[li[it]] = loff; }
                else { g_off[v] = off; if (o.lcol) o.g_loff[v] = loff; }
            }
        }
    }
    __syncthreads();
    #pragma unroll
    for (int it = 0; it < kHIters; ++it) {
        const int64_t e = base + it * kBlock + (int64_t)threadIdx.x;
        const bool kept = (keep >> it) & 1u;
        if (!kept && (!o.lcol || e >= end)) continue;
        const int64_t v = u0 + li[it];
        const int32_t b0 = kLds ? wbase[li[it]] : g_base[v];
        if (kept) {
            const int32_t off = kLds ? woff[li[it]] : g_off[v];
            o.hcol[o.hrp[v] + off + (pre[it] - b0)] = cu[it];
        } else {
            const int32_t loff = kLds ? wloff[li[it]] : o.g_loff[v];
            const int32_t rank = (int32_t)(e - max(rp[v], base)) - (pre[it] - b0);
            o.lcol[o.hrp[v] + loff + rank] = cu[it];
        }
    }
}

template <bool kUserKeys>
__global__ void __launch_bounds__(kBlock) k_orient(const int64_t* rp, const int32_t* ci, const uint64_t* key,
                                                   const uint8_t* q8, uint64_t seed, int64_t nnz,
                                                   const int32_t* brow, OrientOut o) {
    __shared__ int32_t wst[kHWin];      // row starts relative to the range (the first row: <= 0)
    __shared__ uint64_t wkey[kHWin];    // row keys
    __shared__ int32_t wbase[kHWin];    // prefix at each row piece's first entry
    __shared__ int32_t woff[kHWin];     // offset of each row piece inside its row
    __shared__ int32_t wloff[kHWin];    // the same for the lower-priority entries (dynamic handles)
    const int64_t base = (int64_t)blockIdx.x * kHE;
    const int64_t u0 = brow[blockIdx.x], u1 = brow[blockIdx.x + 1];
    const int64_t w = u1 - u0 + 1;
    if (w <= kHWin) {   // uniform over the workgroup
        for (int64_t i = threadIdx.x; i < w; i += kBlock) {
            wst[i] = (int32_t)max<int64_t>(rp[u0 + i] - base, i == 0 ? INT32_MIN : 0);
            wkey[i] = key[u0 + i];
        }
        __syncthreads();
        orient_body<kUserKeys, true>(rp, ci, key, q8, seed, nnz, u0, u1, o, wst, wkey, wbase, woff, wloff);
    } else {
        orient_body<kUserKeys, false>(rp, ci, key, q8, seed, nnz, u0, u1, o, wst, wkey, wbase, woff, wloff);
    }
}

// Dense-block test, one wave per 16-row block: the block's oriented entries as
// (column block << 4 | row) keys in LDS, sorted (bitonic), nonzero tiles = distinct
// column blocks.  dflag[I] = 1 and dtcnt[I] = tiles if the block is dense.
// kFill: for dense blocks (dflag already scanned into dpos, dtcnt into dfirst), writes
// the tiles' column blocks and bitmaps and the block's list slot.
template <bool kFill>
__global__ void __launch_bounds__(kBlock) k_dense(const int64_t* rp, const int32_t* hcol, const int32_t* hcnt,
                                                  int64_t n, int64_t nI, int dense_min, int32_t* dflag,
                                                  int32_t* dtcnt, const int32_t* dpos, int32_t* drb, int32_t* dptr,
                                                  int32_t* dcol, uint32_t* dbits) {
    __shared__ uint64_t skey[kWpb][kDenseCap];
    __shared__ uint32_t sbits[kWpb][kDenseTiles * 8];
    __shared__ int32_t srow[kWpb][17];
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    uint64_t* sk = skey[wid];
    int32_t* sr = srow[wid];
    const int64_t nwaves = (int64_t)gridDim.x * kWpb;
    for (int64_t I = (int64_t)blockIdx.x * kWpb + wid; I < nI; I += nwaves) {
        if (kFill && !dflag[I]) continue;
        // entries per row of the block and their prefix (lanes 0..15)
        const int64_t v = I * 16 + lane;
        const int32_t c = lane < 16 && v < n ? hcnt[v] : 0;
        int32_t incl = c;
        #pragma unroll
        for (int off = 1; off < 16; off <<= 1) {
            const int32_t o = __shfl_up(incl, off, kWave);
            if (lane >= off) incl += o;
        }
        const int32_t total = __shfl(incl, 15, kWave);
        if (!kFill) {
            if (total == 0 || total > kDenseCap) {
                if (lane == 0) { dflag[I] = 0; dtcnt[I] = 0; }
                continue;
            }
        }
        wave_sync_lds();
        if (lane < 16) sr[lane + 1] = incl;
        if (lane == 0) sr[0] = 0;
        wave_sync_lds();
        // gather: key = column << 4 | row (so column block = key >> 8), padded to a
        // power of two with ~0
        int P = 64;
        while (P < total) P <<= 1;
        for (int k = lane; k < P; k += kWave) {
            uint64_t x = ~0ull;
            if (k < total) {
                int r = 0;
                while (sr[r + 1] <= k) ++r;
                const int32_t u = hcol[rp[I * 16 + r] + (k - sr[r])];
                x = ((uint64_t)(uint32_t)u << 4) | (uint64_t)r;
            }
            sk[k] = x;
        }
        wave_sync_lds();
        for (int size = 2; size <= P; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int k = lane; k < P; k += kWave) {
                    const int j = k ^ stride;
                    if (j > k) {
                        const uint64_t a = sk[k], b = sk[j];
                        const bool up = (k & size) == 0;
                        if ((a > b) == up) { sk[k] = b; sk[j] = a; }
                    }
                }
                wave_sync_lds();
            }
        }
        // tiles = distinct column blocks among the first `total` keys
        int tiles = 0;
        for (int k0 = 0; k0 < total; k0 += kWave) {
            const int k = k0 + lane;
            const bool head = k < total && (k == 0 || (sk[k] >> 8) != (sk[k - 1] >> 8));
            tiles += __popcll(ballot(head));
        }
        if (!kFill) {
            const bool dense = tiles <= kDenseTiles && (int64_t)total >= (int64_t)dense_min * tiles;
            if (lane == 0) { dflag[I] = dense ? 1 : 0; dtcnt[I] = dense ? tiles : 0; }
            continue;
        }
        // fill: tile of each key = number of heads at or before it, minus one
        for (int k = lane; k < kDenseTiles * 8; k += kWave) sbits[wid][k] = 0;
        wave_sync_lds();
        const int32_t t0 = dtcnt[I];   // first tile (scanned)
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
        for (int k = lane; k < tiles * 8; k += kWave) dbits[(int64_t)t0 * 8 + k] = sbits[wid][k];
        if (lane == 0) {
            const int32_t p = dpos[I];
            drb[p] = (int32_t)I;
            dptr[p] = t0;
        }
        wave_sync_lds();
    }
}

// a dynamic handle classifies its rows again after edits: the counters start at zero
__global__ void k_hyb_meta_clear(Meta* meta) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        meta->n_c1 = 0;
        meta->n_hl[0] = meta->n_hl[1] = 0;
    }
}

// row capacities of a dynamic handle (each orientation: its degree plus the slack)
__global__ void k_dyn_caps(const int64_t* rp, int64_t n, int slack, int64_t* cap) {
    GRID_STRIDE(v, n) cap[v] = rp[v + 1] - rp[v] + slack;
}

__global__ void k_dense_end(const Meta* meta, int32_t* dptr) {
    if (threadIdx.x == 0 && blockIdx.x == 0) dptr[meta->n_dense] = meta->n_dtiles;
}

// Round-1 classification of every vertex: no higher-priority neighbour -> candidate
// of round 1 (bit in s1); else undecided (bit in a1) and, outside dense blocks, a
// light or heavy list row.  flag packs (light, heavy) as (1, 1 << 32) for the scan.
__global__ void k_hyb_class(const int32_t* hcnt, const int32_t* dflag, int64_t n, int64_t* flag, uint32_t* s1,
                            uint32_t* a1, int64_t* n_c1) {
    int64_t c1 = 0;
    const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
    const int64_t nr = (n + kWave - 1) / kWave * kWave;   // whole waves iterate together
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nr; v += nthreads) {
        const bool valid = v < n;
        const int32_t c = valid ? hcnt[v] : -1;
        const bool dense = valid && dflag && dflag[v >> 4];
        if (valid) flag[v] = (c == 0 || dense) ? 0 : (c <= kHLight ? 1ll : (1ll << 32));
        const uint64_t bc = ballot(c == 0), ba = ballot(c > 0);
        c1 += lane_id() == 0 ? __popcll(bc) : 0;
        const int lane = lane_id();
        if (lane < 2 && v - lane < n) {   // v - lane is the wave's first vertex (a multiple of 64)
            const int64_t w = (v - lane) / 32 + lane;
            if (w * 32 < n) {
                s1[w] = (uint32_t)(bc >> (32 * lane));
                a1[w] = (uint32_t)(ba >> (32 * lane));
            }
        }
    }
    for (int off = kWave / 2; off > 0; off >>= 1) c1 += __shfl_xor(c1, off, kWave);
    if (lane_id() == 0 && c1) atomicAdd((unsigned long long*)n_c1, (unsigned long long)c1);
}

__global__ void k_hyb_lists(const int64_t* flag, const int64_t* pos, int64_t n, int32_t* light, int32_t* heavy,
                            Meta* meta) {
    GRID_STRIDE(v, n) {
        const int64_t f = flag[v], p = pos[v];
        if (f == 1) light[(uint32_t)p] = (int32_t)v;
        else if (f) heavy[p >> 32] = (int32_t)v;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const int64_t t = pos[n];
        meta->n_hl[0] = (uint32_t)t;
        meta->n_hl[1] = t >> 32;
    }
}

// ---------------------------------------------------------------- rounds

struct HybArgs {
    const int64_t* rp;
    const int32_t* hcol;
    const int32_t* hcnt;
    uint32_t* A;
    uint32_t* S;
    const int32_t* l1[3];     // round 1: light rows, heavy rows, dense blocks
    int32_t* act[2][3];       // later rounds, by round parity
    const int32_t* dptr;      // dense block (by round-1 list slot order of drb) -> first tile
    const int32_t* dslot;     // dense block I -> its slot in drb (for dptr)
    const int32_t* dcol;
    const uint32_t* dbits;
    const Meta* meta;
    Ctrl* ctrl;
    int64_t* stripes;
    TraceRec* trace;
    int32_t* dround;          // batches: round in which each vertex was decided
};

__device__ inline void hyb_lists(const HybArgs& a, int r, const int32_t* (&L)[3], int64_t (&nl)[3]) {
    if (r == 1) {
        for (int k = 0; k < 3; ++k) L[k] = a.l1[k];
        nl[0] = a.meta->n_hl[0];
        nl[1] = a.meta->n_hl[1];
        nl[2] = a.meta->n_dense;
    } else {
        const int b = (r - 1) & 1;
        for (int k = 0; k < 3; ++k) {
            L[k] = a.act[b][k];
            nl[k] = a.ctrl->n_act[b][k];
        }
    }
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

// Phase 1 of round r >= 2 (round 1's candidates come from the build).
__device__ void hyb_p1(const HybArgs& a, int r) {
    __shared__ uint32_t sbits[kWpb][kDenseTiles * 8];
    __shared__ uint32_t svec[kWpb][kDenseTiles];
    open_round(a.ctrl, a.stripes, a.trace, r);
    if (r == 1) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            int64_t* st = a.stripes + (int64_t)(r & 1) * kStripes * kStripeWords;
            if (a.meta->n_c1) atomicAdd((unsigned long long*)&st[0], (unsigned long long)a.meta->n_c1);
        }
        return;
    }
    const int32_t* L[3];
    int64_t nl[3];
    hyb_lists(a, r, L, nl);
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    const int64_t nthreads = (int64_t)gridDim.x * kBlock;
    const int64_t tid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t nwaves = nthreads / kWave, wv = tid / kWave;
    int64_t n_cand = 0, ent = 0, verts = 0, mult = 0, blocks = 0;
    // light rows: a lane each (whole waves iterate together for the combined atomics)
    const int64_t nlr = (nl[0] + kWave - 1) / kWave * kWave;
    for (int64_t i = tid; i < nlr; i += nthreads) {
        int64_t w = -1;
        uint32_t m = 0;
        if (i < nl[0]) {
            const int32_t v = L[0][i];
            const int64_t e0 = a.rp[v];
            const int32_t c = a.hcnt[v];
            int32_t k = 0;
            bool blocked = false;
            for (; k < c; ++k) {
                const int32_t u = a.hcol[e0 + k];
                if (u >= 0 && bit_of(a.A, u)) { blocked = true; ++k; break; }
            }
            ent += k;
            ++verts;
            if (!blocked) { w = v >> 5; m = 1u << (v & 31); ++n_cand; }
        }
        run_apply<false>(w, m, a.S);
    }
    // heavy rows: a wave each, 64 entries per step, early exit on the first alive one
    for (int64_t i = wv; i < nl[1]; i += nwaves) {
        const int32_t v = L[1][i];
        const int64_t e0 = a.rp[v];
        const int32_t c = a.hcnt[v];
        bool blocked = false;
        int32_t k = 0;
        for (; k < c; k += kWave) {
            const int32_t u = k + lane < c ? a.hcol[e0 + k + lane] : -1;
            const bool b = u >= 0 && bit_of(a.A, u);
            if (ballot(b)) { blocked = true; k += kWave; break; }
        }
        if (lane == 0) {
            ent += min(k, c);
            ++verts;
            if (!blocked) { atomicOr(&a.S[v >> 5], 1u << (v & 31)); ++n_cand; }
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
    block_count(a.stripes, r, {0, 2, 3, 6, 8}, x);
}

// Phases 2 and 3 of round r: retire candidates, remove their neighbours, list the rest.
__device__ void hyb_p2(const HybArgs& a, int r) {
    __shared__ int32_t lbuf[kWpb][3][kWave];
    __shared__ uint32_t sbits[kWpb][kDenseTiles * 8];
    __shared__ uint32_t svec[kWpb][kDenseTiles];
    const int32_t* L[3];
    int64_t nl[3];
    hyb_lists(a, r, L, nl);
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    int pend[3] = {0, 0, 0};
    int32_t* next[3];
    int64_t* cnt[3];
    for (int k = 0; k < 3; ++k) {
        next[k] = a.act[r & 1][k];
        cnt[k] = &a.ctrl->n_act[r & 1][k];
    }
    const int64_t nthreads = (int64_t)gridDim.x * kBlock;
    const int64_t tid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t nwaves = nthreads / kWave, wv = tid / kWave;
    int64_t n_out = 0, ent = 0, verts = 0, mult = 0, blocks = 0;
    const int64_t nlr = (nl[0] + kWave - 1) / kWave * kWave;
    for (int64_t i = tid; i < nlr; i += nthreads) {
        int64_t w = -1;
        uint32_t m = 0;
        bool keep = false;
        int32_t v = 0;
        if (i < nl[0]) {
            v = L[0][i];
            if (bit_of(a.S, v)) {
                w = v >> 5; m = 1u << (v & 31);
                if (a.dround) a.dround[v] = r;
            } else {
                const int64_t e0 = a.rp[v];
                const int32_t c = a.hcnt[v];
                int32_t k = 0;
                bool hit = false;
                for (; k < c; ++k) {
                    const int32_t u = a.hcol[e0 + k];
                    if (u >= 0 && bit_of(a.S, u)) { hit = true; ++k; break; }
                }
                ent += k;
                ++verts;
                if (hit) {
                    w = v >> 5; m = 1u << (v & 31); ++n_out;
                    if (a.dround) a.dround[v] = r;
                } else {
                    keep = true;
                }
            }
        }
        run_apply<true>(w, m, a.A);
        lbuf_push(lbuf[wid][0], pend[0], next[0], cnt[0], keep, v);
    }
    lbuf_flush(lbuf[wid][0], pend[0], next[0], cnt[0]);
    for (int64_t i = wv; i < nl[1]; i += nwaves) {
        const int32_t v = L[1][i];
        bool hit = false, in = false;
        if (bit_of(a.S, v)) {
            in = true;
        } else {
            const int64_t e0 = a.rp[v];
            const int32_t c = a.hcnt[v];
            int32_t k = 0;
            for (; k < c; k += kWave) {
                const int32_t u = k + lane < c ? a.hcol[e0 + k + lane] : -1;
                const bool b = u >= 0 && bit_of(a.S, u);
                if (ballot(b)) { hit = true; k += kWave; break; }
            }
            if (lane == 0) { ent += min(k, c); ++verts; }
        }
        if (lane == 0 && (in || hit)) {
            atomicAnd(&a.A[v >> 5], ~(1u << (v & 31)));
            if (a.dround) a.dround[v] = r;
            n_out += hit ? 1 : 0;
        }
        lbuf_push(lbuf[wid][1], pend[1], next[1], cnt[1], lane == 0 && !in && !hit, v);
    }
    lbuf_flush(lbuf[wid][1], pend[1], next[1], cnt[1]);
    for (int64_t i = wv; i < nl[2]; i += nwaves) {
        const int32_t I = L[2][i];
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
        lbuf_push(lbuf[wid][2], pend[2], next[2], cnt[2], lane == 0 && (al & ~dec) != 0, I);
    }
    lbuf_flush(lbuf[wid][2], pend[2], next[2], cnt[2]);
    int64_t x[5] = {n_out, ent, verts, mult, blocks};
    block_count(a.stripes, r, {1, 4, 5, 7, 9}, x);
}

__global__ void __launch_bounds__(kBlock) k_hyb_p1(HybArgs a, int ri) { hyb_p1(a, a.ctrl->rbase + ri); }
__global__ void __launch_bounds__(kBlock) k_hyb_p2(HybArgs a, int ri) { hyb_p2(a, a.ctrl->rbase + ri); }

// Persistent variant: k rounds in one cooperative launch, a grid barrier after every
// phase; the last round is closed and the base advanced at the end.
__global__ void __launch_bounds__(kBlock) k_hyb_rounds(HybArgs a, int k) {
    const int rb = a.ctrl->rbase;
    for (int ri = 1; ri <= k; ++ri) {
        hyb_p1(a, rb + ri);
        grid_barrier(a.ctrl);
        hyb_p2(a, rb + ri);
        grid_barrier(a.ctrl);
    }
    finish_rounds(a.ctrl, a.stripes, a.trace, rb, k);
}

// round state before round 1: the bitmaps of the build; batches: round-1 candidates
// are decided in round 1, everything else undecided
__global__ void k_hyb_init(const uint32_t* s1, const uint32_t* a1, uint32_t* S, uint32_t* A, int32_t* dround,
                           int64_t n, int64_t nw) {
    GRID_STRIDE(w, nw) {
        S[w] = s1[w];
        A[w] = a1[w];
    }
    if (dround)
        GRID_STRIDE(v, n) dround[v] = bit_of(s1, v) ? 1 : 0;
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

HybArgs make_args(mis_graph* g) {
    HybArgs a;
    a.rp = g->hrp;
    a.hcol = g->hcol;
    a.hcnt = g->hcnt;
    a.A = g->hA;
    a.S = g->hS;
    a.l1[0] = g->hl1[0];
    a.l1[1] = g->hl1[1];
    a.l1[2] = g->drb;
    for (int b = 0; b < 2; ++b)
        for (int k = 0; k < 3; ++k) a.act[b][k] = g->hact[b][k];
    a.dptr = g->dptr;
    a.dslot = g->dslot;
    a.dcol = g->dcol;
    a.dbits = g->dbits;
    a.meta = g->meta;
    a.ctrl = g->ctrl;
    a.stripes = g->stripes;
    a.trace = g->trace;
    a.dround = g->count > 0 ? g->dround : nullptr;
    return a;
}

__global__ void k_dense_slots(const int32_t* dflag, const int32_t* dpos, int64_t nI, int32_t* dslot) {
    GRID_STRIDE(I, nI) dslot[I] = dflag[I] ? dpos[I] : -1;
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
    TC_HIP(hipMemsetAsync(g->meta, 0, sizeof(Meta), s));
    if (n == 0) return MIS_OK;
    // 1. orientation (stages: row search, orientation, dense blocks, lists)
    TC_HIP(hipMemsetAsync(g->hcnt, 0, (size_t)n * 4, s));
    g->hrp = g->row_ptr;
    if (g->dyn_slack > 0) {
        // dynamic handle: rows of its own, deg + slack slots for each orientation
        TC_HIP(hipMemsetAsync(g->lcnt, 0, (size_t)n * 4, s));
        HLAUNCH(k_dyn_caps, n, g->row_ptr, n, g->dyn_slack, g->hflag);
        TC_CHECK(scan_excl_i64(g->hflag, g->drp, n, g->drp + n, (int64_t*)g->scan_tmp, s));
        g->hrp = g->drp;
    }
    const int64_t nb = hyb_blocks(nnz);
    if (nnz > 0) HLAUNCH(k_orient_rows, nb + 1, g->row_ptr, n, nnz, nb, g->hbrow);
    build_mark(g, s);
    if (nnz > 0) {
        OrientOut o{g->hrp, g->hcol, g->hcnt, g->dyn_slack > 0 ? g->lcol : nullptr, g->lcnt, g->hbase, g->hoff,
                    g->hloff};
        if (g->user_keys)
            hipLaunchKernelGGL(k_orient<true>, dim3((unsigned)nb), dim3(kBlock), 0, s, g->row_ptr, g->col_idx, g->key,
                               g->q8, g->seed, nnz, g->hbrow, o);
        else
            hipLaunchKernelGGL(k_orient<false>, dim3((unsigned)nb), dim3(kBlock), 0, s, g->row_ptr, g->col_idx,
                               g->key, g->q8, g->seed, nnz, g->hbrow, o);
        TC_HIP(hipGetLastError());
    }
    build_mark(g, s);
    // 2. dense blocks
    const bool dense = g->dense_min > 0 && nnz > 0;
    if (dense) {
        const unsigned blocks = (unsigned)std::min<int64_t>(ceil_div(nI, kWpb), 16384);
        hipLaunchKernelGGL(k_dense<false>, dim3(blocks), dim3(kBlock), 0, s, g->row_ptr, g->hcol, g->hcnt, n, nI,
                           g->dense_min, g->dflag, g->dtcnt, (const int32_t*)nullptr, (int32_t*)nullptr,
                           (int32_t*)nullptr, (int32_t*)nullptr, (uint32_t*)nullptr);
        TC_HIP(hipGetLastError());
        // list slots of dense blocks and their first tiles (dflag keeps the flags)
        TC_CHECK(scan_excl_i32(g->dflag, g->dpos, nI, &g->meta->n_dense, (int32_t*)g->scan_tmp, s));
        TC_CHECK(scan_excl_i32(g->dtcnt, g->dtcnt, nI, &g->meta->n_dtiles, (int32_t*)g->scan_tmp, s));
        hipLaunchKernelGGL(k_dense<true>, dim3(blocks), dim3(kBlock), 0, s, g->row_ptr, g->hcol, g->hcnt, n, nI,
                           g->dense_min, g->dflag, g->dtcnt, g->dpos, g->drb, g->dptr, g->dcol, g->dbits);
        TC_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_dense_end, dim3(1), dim3(1), 0, s, g->meta, g->dptr);
        TC_HIP(hipGetLastError());
        HLAUNCH(k_dense_slots, nI, g->dflag, g->dpos, nI, g->dslot);
    }
    build_mark(g, s);
    // 3. round-1 classes and lists
    HLAUNCH(k_hyb_class, n, g->hcnt, dense ? g->dflag : nullptr, n, g->hflag, g->s1, g->a1, &g->meta->n_c1);
    TC_CHECK(scan_excl_i64(g->hflag, g->hpos, n, g->hpos + n, (int64_t*)g->scan_tmp, s));
    HLAUNCH(k_hyb_lists, n, g->hflag, g->hpos, n, g->hl1[0], g->hl1[1], g->meta);
    return MIS_OK;
}

int hyb_classify(mis_graph* g, hipStream_t s);

// round-1 classes and lists from the rows' current counts
int hyb_classify(mis_graph* g, hipStream_t s) {
    const int64_t n = g->n;
    HLAUNCH(k_hyb_meta_clear, 1, g->meta);
    HLAUNCH(k_hyb_class, n, g->hcnt, g->dense_min > 0 ? g->dflag : nullptr, n, g->hflag, g->s1, g->a1, &g->meta->n_c1);
    TC_CHECK(scan_excl_i64(g->hflag, g->hpos, n, g->hpos + n, (int64_t*)g->scan_tmp, s));
    HLAUNCH(k_hyb_lists, n, g->hflag, g->hpos, n, g->hl1[0], g->hl1[1], g->meta);
    return MIS_OK;
}

int hyb_init(mis_graph* g, hipStream_t s) {
    if (g->dyn_edited && g->n > 0) {   // a dynamic handle's rows changed since they were classified
        TC_CHECK(hyb_classify(g, s));
        g->dyn_edited = false;
    }
    const int64_t nw = ceil_div(g->n, 32);
    if (g->n > 0)
        hipLaunchKernelGGL(k_hyb_init, dim3(stream_grid(std::max(nw, g->count > 0 ? g->n : 0))), dim3(kBlock), 0, s,
                           g->s1, g->a1, g->hS, g->hA, g->count > 0 ? g->dround : nullptr, g->n, nw);
    TC_HIP(hipGetLastError());
    return MIS_OK;
}

// phase 0 = candidate kernel, 1 = exclusion kernel
int hyb_enqueue_phase(mis_graph* g, int phase, int r, hipStream_t s) {
    HybArgs a = make_args(g);
    if (phase == 0) hipLaunchKernelGGL(k_hyb_p1, dim3(g->grid_blocks), dim3(kBlock), 0, s, a, r);
    else hipLaunchKernelGGL(k_hyb_p2, dim3(g->grid_blocks), dim3(kBlock), 0, s, a, r);
    TC_HIP(hipGetLastError());
    return MIS_OK;
}

// k rounds as one cooperative launch (see k_hyb_rounds)
int hyb_enqueue_rounds(mis_graph* g, int k, hipStream_t s) {
    HybArgs a = make_args(g);
    return launch_cooperative((const void*)k_hyb_rounds, g, &a, k, s);
}

int hyb_output(mis_graph* g, uint8_t* in_set, bool if_done, hipStream_t s) {
    const Ctrl* gate = if_done ? g->ctrl : nullptr;
    if (g->n > 0 && ((uintptr_t)in_set & 3) == 0)
        hipLaunchKernelGGL(k_hyb_output4, dim3(stream_grid(ceil_div(g->n, 4))), dim3(kBlock), 0, s, gate, g->hS, g->n,
                           in_set);
    else if (g->n > 0)
        hipLaunchKernelGGL(k_hyb_output, dim3(stream_grid(g->n)), dim3(kBlock), 0, s, gate, g->hS, g->n, in_set);
    TC_HIP(hipGetLastError());
    return MIS_OK;
}

}  // namespace tcmis
