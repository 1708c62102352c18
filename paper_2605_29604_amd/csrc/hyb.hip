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

// Dense-block test, one wave per 16-row block: the number of nonzero tiles is the
// number of distinct column blocks among the block's oriented entries, counted with
// an open-addressing set in LDS.  dflag[I] = 1 and dtcnt[I] = tiles if the block is
// dense (at most 64 tiles, at least dense_min entries per tile on average).
__global__ void __launch_bounds__(kBlock) k_dense_test(const int64_t* rp, const int32_t* hcol, const int32_t* hcnt,
                                                       int64_t n, int64_t nI, int dense_min, int32_t* dflag,
                                                       int32_t* dtcnt) {
    constexpr uint32_t kEmpty = 0xFFFFFFFFu;
    __shared__ uint32_t tab[kWpb][2 * kDenseCap];
    __shared__ int32_t srow[kWpb][17];
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    uint32_t* T = tab[wid];
    int32_t* sr = srow[wid];
    const int64_t nwaves = (int64_t)gridDim.x * kWpb;
    for (int64_t I = (int64_t)blockIdx.x * kWpb + wid; I < nI; I += nwaves) {
        const int64_t v = I * 16 + lane;
        const int32_t c = lane < 16 && v < n ? hcnt[v] : 0;
        int32_t incl = c;
        #pragma unroll
        for (int off = 1; off < 16; off <<= 1) {
            const int32_t o = __shfl_up(incl, off, kWave);
            if (lane >= off) incl += o;
        }
        const int32_t total = __shfl(incl, 15, kWave);
        // a dense block holds at least dense_min entries (one tile) and at most the cap
        if (total == 0 || total > kDenseCap || total < dense_min) {
            if (lane == 0) { dflag[I] = 0; dtcnt[I] = 0; }
            continue;
        }
        int bits = 6;
        while ((1 << bits) < 2 * total) ++bits;   // table of 2^bits >= 2 * total slots
        const uint32_t mask = (1u << bits) - 1u;
        wave_sync_lds();
        if (lane < 16) sr[lane + 1] = incl;
        if (lane == 0) sr[0] = 0;
        for (int k = lane; k <= (int)mask; k += kWave) T[k] = kEmpty;
        wave_sync_lds();
        int fresh = 0;
        for (int k = lane; k < total; k += kWave) {
            int r = 0;
            while (sr[r + 1] <= k) ++r;
            const uint32_t J = (uint32_t)hcol[rp[I * 16 + r] + (k - sr[r])] >> 4;
            uint32_t h = (J * 2654435761u) >> (32 - bits);
            for (;;) {
                const uint32_t old = atomicCAS(&T[h], kEmpty, J);
                if (old == kEmpty) { ++fresh; break; }
                if (old == J) break;
                h = (h + 1) & mask;
            }
        }
        for (int off = kWave / 2; off > 0; off >>= 1) fresh += __shfl_xor(fresh, off, kWave);
        const bool dense = fresh <= kDenseTiles && (int64_t)total >= (int64_t)dense_min * fresh;
        if (lane == 0) { dflag[I] = dense ? 1 : 0; dtcnt[I] = dense ? fresh : 0; }
    }
}

// Tiles of the dense blocks (dflag set; dpos = their list slots, dtcnt = their first
// tiles), one wave per block: the block's entries as (column << 4 | row) keys in
// LDS, sorted (bitonic), tile = run of one column block; bitmaps built in LDS and
// written out, with the tiles' column blocks and the block's list slot.
__global__ void __launch_bounds__(kBlock) k_dense_fill(const int64_t* rp, const int32_t* hcol, const int32_t* hcnt,
                                                       int64_t n, int64_t nI, const int32_t* dflag, const int32_t* dtcnt,
                                                       const int32_t* dpos, int32_t* drb, int32_t* dptr, int32_t* dcol,
                                                       uint32_t* dbits) {
    __shared__ uint64_t skey[kWpb][kDenseCap];
    __shared__ uint32_t sbits[kWpb][kDenseTiles * 8];
    __shared__ int32_t srow[kWpb][17];
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    uint64_t* sk = skey[wid];
    int32_t* sr = srow[wid];
    const int64_t nwaves = (int64_t)gridDim.x * kWpb;
    for (int64_t I = (int64_t)blockIdx.x * kWpb + wid; I < nI; I += nwaves) {
        if (!dflag[I]) continue;
        const int64_t v = I * 16 + lane;
        const int32_t c = lane < 16 && v < n ? hcnt[v] : 0;
        int32_t incl = c;
        #pragma unroll
        for (int off = 1; off < 16; off <<= 1) {
            const int32_t o = __shfl_up(incl, off, kWave);
            if (lane >= off) incl += o;
        }
        const int32_t total = __shfl(incl, 15, kWave);
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
        // tile of each key = number of heads at or before it, minus one
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
        for (int k = lane; k < seen * 8; k += kWave) dbits[(int64_t)t0 * 8 + k] = sbits[wid][k];
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
    // one atomic per workgroup (a same-address atomic per wave serialises the kernel)
    __shared__ int64_t part[kWpb];
    for (int off = kWave / 2; off > 0; off >>= 1) c1 += __shfl_xor(c1, off, kWave);
    if (lane_id() == 0) part[threadIdx.x / kWave] = c1;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int q = 0; q < kWpb; ++q) t += part[q];
        if (t) atomicAdd((unsigned long long*)n_c1, (unsigned long long)t);
    }
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
            const bool blocked = scan4(a.hcol + a.rp[v], a.hcnt[v], a.A, &ent);
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
                const bool hit = scan4(a.hcol + a.rp[v], a.hcnt[v], a.S, &ent);
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

// round-1 classes (bitmaps, candidate count) and the light / heavy row lists
int hyb_lists_build(mis_graph* g, const int32_t* dflag, hipStream_t s) {
    const int64_t n = g->n;
    if (n > 0) {
        const unsigned blocks = (unsigned)std::min<int64_t>(ceil_div(n, kBlock), 1024);
        hipLaunchKernelGGL(k_hyb_class, dim3(blocks), dim3(kBlock), 0, s, g->hcnt, dflag, n, g->hflag, g->s1, g->a1,
                           &g->meta->n_c1);
        TC_HIP(hipGetLastError());
    }
    TC_CHECK(scan_excl_i64(g->hflag, g->hpos, n, g->hpos + n, (int64_t*)g->scan_tmp, s));
    HLAUNCH(k_hyb_lists, n, g->hflag, g->hpos, n, g->hl1[0], g->hl1[1], g->meta);
    return MIS_OK;
}

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
        hipLaunchKernelGGL(k_dense_test, dim3(blocks), dim3(kBlock), 0, s, g->row_ptr, g->hcol, g->hcnt, n, nI,
                           g->dense_min, g->dflag, g->dtcnt);
        TC_HIP(hipGetLastError());
        // list slots of dense blocks and their first tiles (dflag keeps the flags)
        TC_CHECK(scan_excl_i32(g->dflag, g->dpos, nI, &g->meta->n_dense, (int32_t*)g->scan_tmp, s));
        TC_CHECK(scan_excl_i32(g->dtcnt, g->dtcnt, nI, &g->meta->n_dtiles, (int32_t*)g->scan_tmp, s));
        hipLaunchKernelGGL(k_dense_fill, dim3(blocks), dim3(kBlock), 0, s, g->row_ptr, g->hcol, g->hcnt, n, nI,
                           g->dflag, g->dtcnt, g->dpos, g->drb, g->dptr, g->dcol, g->dbits);
        TC_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_dense_end, dim3(1), dim3(1), 0, s, g->meta, g->dptr);
        TC_HIP(hipGetLastError());
        HLAUNCH(k_dense_slots, nI, g->dflag, g->dpos, nI, g->dslot);
    }
    build_mark(g, s);
    // 3. round-1 classes and lists
    TC_CHECK(hyb_lists_build(g, dense ? g->dflag : nullptr, s));
    return MIS_OK;
}

int hyb_classify(mis_graph* g, hipStream_t s);

// round-1 classes and lists from the rows' current counts (after edits)
int hyb_classify(mis_graph* g, hipStream_t s) {
    HLAUNCH(k_hyb_meta_clear, 1, g->meta);
    return hyb_lists_build(g, g->dense_min > 0 ? g->dflag : nullptr, s);
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
