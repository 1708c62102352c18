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

// a column block's bit in a row-block's 64-bit signature
__device__ inline uint64_t sig_bit(int64_t J) { return 1ull << (((uint64_t)J * 0x9E3779B97F4A7C15ull) >> 58); }

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
// With sig, every 16-row block's higher-priority entries also OR the signature bits of
// their column blocks into sig[I] (popcount(sig[I]) is a lower bound on the block's
// nonzero tiles).
struct OrientOut {
    const int64_t* hrp;
    int32_t* hcol;
    int32_t* hcnt;
    int32_t* lcol;      // nullptr: higher-priority entries only
    int32_t* lcnt;
    int32_t* g_base;    // [n] scratch of workgroups whose rows exceed LDS
    int32_t* g_off;
    int32_t* g_loff;
    uint64_t* sig;      // [nI] or nullptr
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
    if (o.sig) {
        // the thread's entries lie in at most a few row-blocks (rows are consecutive):
        // all but the last run are ORed in directly, the last one is combined across
        // the wave first (adjacent lanes mostly share it)
        int64_t I = (u0 + li[0]) >> 4;
        uint64_t m = 0;
        #pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int64_t Ij = (u0 + li[j]) >> 4;
            if (Ij != I) {
                if (m) atomicOr((unsigned long long*)&o.sig[I], (unsigned long long)m);
                I = Ij;
                m = 0;
            }
            if ((keep >> j) & 1u) m |= sig_bit(cu[j] >> 4);
        }
        #pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const uint64_t mo = __shfl_down(m, off, kWave);
            const int64_t Io = __shfl_down(I, off, kWave);
            if (lane + off < kWave && Io == I) m |= mo;
        }
        const int64_t Ip = __shfl_up(I, 1, kWave);
        if ((lane == 0 || Ip != I) && m) atomicOr((unsigned long long*)&o.sig[I], (unsigned long long)m);
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
// dense (at most 64 tiles, at least dense_min entries per tile on average).  The
// block's signature bounds its tiles from below (distinct column blocks set at least
// popcount(sig) bits), so a block with fewer than dense_min * popcount(sig) entries is
// rejected without reading its entries.
__global__ void __launch_bounds__(kBlock) k_dense_test(const int64_t* rp, const int32_t* hcol, const int32_t* hcnt,
                                                       const uint64_t* sig, int64_t n, int64_t nI, int dense_min,
                                                       int32_t* dflag, int32_t* dtcnt) {
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
        // a dense block holds at least dense_min entries per tile and at most the cap
        const int64_t lower = __popcll(sig[I]);
        if (total == 0 || total > kDenseCap || (int64_t)total < (int64_t)dense_min * lower) {
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

// row capacities of a dynamic handle (each orientation: its degree plus the slack)
__global__ void k_dyn_caps(const int64_t* rp, int64_t n, int slack, int64_t* cap) {
    GRID_STRIDE(v, n) cap[v] = rp[v + 1] - rp[v] + slack;
}

__global__ void k_dense_end(const Meta* meta, int32_t* dptr) {
    if (threadIdx.x == 0 && blockIdx.x == 0) dptr[meta->n_dense] = meta->n_dtiles;
}

// ---------------------------------------------------------------- rounds

struct HybArgs {
    int64_t n;
    const int64_t* rp;
    const int32_t* hcol;
    const int32_t* hcnt;
    uint32_t* A;
    uint32_t* S;
    const int32_t* drb;       // round 1: the dense blocks (round 1 visits every vertex otherwise)
    int32_t* act[2][3];       // later rounds, by round parity: light rows, heavy rows, dense blocks
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

// the lists of round r >= 2 (written by round r-1's exclusion kernel)
__device__ inline void hyb_lists(const HybArgs& a, int r, const int32_t* (&L)[3], int64_t (&nl)[3]) {
    const int b = (r - 1) & 1;
    for (int k = 0; k < 3; ++k) {
        L[k] = a.act[b][k];
        nl[k] = a.ctrl->n_act[b][k];
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

// Phase 1 of round r >= 2 (round 1's candidates come from the build).  The
// workgroup is number vb of nvb working on this graph (the launch's grid, or the
// graph's share of a launch over several graphs).
__device__ void hyb_p1(const HybArgs& a, int r, int64_t vb, int64_t nvb) {
    __shared__ uint32_t sbits[kWpb][kDenseTiles * 8];
    __shared__ uint32_t svec[kWpb][kDenseTiles];
    open_round(a.ctrl, a.stripes, a.trace, r, vb);
    if (r == 1) return;   // round 1's candidates were counted when the round state was set up
    const int32_t* L[3];
    int64_t nl[3];
    hyb_lists(a, r, L, nl);
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    const int64_t nthreads = nvb * kBlock;
    const int64_t tid = vb * kBlock + threadIdx.x;
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
    block_count(a.stripes, r, {0, 2, 3, 6, 8}, x, vb);
}

// Phases 2 and 3 of round r: retire candidates, remove their neighbours, list the rest.
__device__ void hyb_p2(const HybArgs& a, int r, int64_t vb, int64_t nvb) {
    __shared__ int32_t lbuf[kWpb][3][kWave];
    __shared__ uint32_t sbits[kWpb][kDenseTiles * 8];
    __shared__ uint32_t svec[kWpb][kDenseTiles];
    const int32_t* L[3] = {nullptr, nullptr, a.drb};
    int64_t nl[3] = {0, 0, a.dslot ? (int64_t)a.meta->n_dense : 0};
    if (r > 1) hyb_lists(a, r, L, nl);
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    int pend[3] = {0, 0, 0};
    int32_t* next[3];
    int64_t* cnt[3];
    for (int k = 0; k < 3; ++k) {
        next[k] = a.act[r & 1][k];
        cnt[k] = &a.ctrl->n_act[r & 1][k];
    }
    const int64_t nthreads = nvb * kBlock;
    const int64_t tid = vb * kBlock + threadIdx.x;
    const int64_t nwaves = nthreads / kWave, wv = tid / kWave;
    int64_t n_out = 0, ent = 0, verts = 0, mult = 0, blocks = 0;
    if (r == 1) {
        // Every vertex outside the dense blocks: a vertex without a higher-priority
        // neighbour is a candidate and already in the set (it was never undecided);
        // any other leaves if one of its higher-priority neighbours is a candidate,
        // else it goes to round 2's lists.  Light rows take a lane each; the heavy rows
        // of a wave's 64 vertices are then scanned by the whole wave, one after another.
        const int64_t nr = (a.n + kWave - 1) / kWave * kWave;   // whole waves iterate together
        for (int64_t i = tid; i < nr; i += nthreads) {
            const int32_t v = (int32_t)i;
            const bool valid = i < a.n;
            const int32_t c = valid ? a.hcnt[v] : 0;
            const bool listed = valid && c > 0 && !(a.dslot && a.dslot[v >> 4] >= 0);
            const bool light = listed && c <= kHLight;
            int64_t w = -1;
            uint32_t m = 0;
            bool keep = false;
            if (light) {
                const bool hit = scan4(a.hcol + a.rp[v], c, a.S, &ent);
                ++verts;
                if (hit) {
                    w = v >> 5; m = 1u << (v & 31); ++n_out;
                    if (a.dround) a.dround[v] = r;
                } else {
                    keep = true;
                }
            }
            run_apply<true>(w, m, a.A);
            lbuf_push(lbuf[wid][0], pend[0], next[0], cnt[0], keep, v);
            uint64_t hv = ballot(listed && !light);
            while (hv) {
                const int l = __builtin_ctzll(hv);
                hv &= hv - 1;
                const int32_t vh = __shfl(v, l, kWave);
                const int64_t e0 = a.rp[vh];
                const int32_t ch = a.hcnt[vh];
                bool hit = false;
                int32_t k = 0;
                for (; k < ch; k += kWave) {
                    const int32_t u = k + lane < ch ? a.hcol[e0 + k + lane] : -1;
                    const bool b = u >= 0 && bit_of(a.S, u);
                    if (ballot(b)) { hit = true; k += kWave; break; }
                }
                if (lane == 0) {
                    ent += min(k, ch);
                    ++verts;
                    if (hit) {
                        atomicAnd(&a.A[vh >> 5], ~(1u << (vh & 31)));
                        ++n_out;
                        if (a.dround) a.dround[vh] = r;
                    }
                }
                lbuf_push(lbuf[wid][1], pend[1], next[1], cnt[1], lane == 0 && !hit, vh);
            }
        }
        lbuf_flush(lbuf[wid][0], pend[0], next[0], cnt[0]);
        lbuf_flush(lbuf[wid][1], pend[1], next[1], cnt[1]);
    } else {
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
    }
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
    block_count(a.stripes, r, {1, 4, 5, 7, 9}, x, vb);
}

__global__ void __launch_bounds__(kBlock) k_hyb_p1(HybArgs a, int ri) {
    hyb_p1(a, a.ctrl->rbase + ri, blockIdx.x, gridDim.x);
}
__global__ void __launch_bounds__(kBlock) k_hyb_p2(HybArgs a, int ri) {
    hyb_p2(a, a.ctrl->rbase + ri, blockIdx.x, gridDim.x);
}

// Persistent variant: k rounds in one cooperative launch, a grid barrier after every
// phase; the last round is closed and the base advanced at the end.
__global__ void __launch_bounds__(kBlock) k_hyb_rounds(HybArgs a, int k) {
    const int rb = a.ctrl->rbase;
    for (int ri = 1; ri <= k; ++ri) {
        hyb_p1(a, rb + ri, blockIdx.x, gridDim.x);
        grid_barrier(a.ctrl);
        hyb_p2(a, rb + ri, blockIdx.x, gridDim.x);
        grid_barrier(a.ctrl);
    }
    finish_rounds(a.ctrl, a.stripes, a.trace, rb, k);
}

// Round state before round 1, from the higher-priority neighbour counts: a vertex
// without one is a candidate of round 1 (in the set, counted into round 1's |C|),
// every other vertex is undecided.  Batches: round-1 candidates are decided in round
// 1, everything else later.  vb / nvb: the workgroup's place in the graph's share
// (the grid, or its part of a launch over several graphs); whole waves iterate
// together, each writing the two bitmap words of its 64 vertices.
__device__ void hyb_init_body(const int32_t* hcnt, int64_t n, uint32_t* S, uint32_t* A, int32_t* dround,
                              int64_t* stripes, int64_t vb, int64_t nvb) {
    int64_t c1 = 0;
    const int64_t nthreads = nvb * kBlock;
    const int64_t nr = (n + kWave - 1) / kWave * kWave;
    const int lane = lane_id();
    for (int64_t v = vb * kBlock + threadIdx.x; v < nr; v += nthreads) {
        const bool valid = v < n;
        const int32_t c = valid ? hcnt[v] : -1;
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
    a.A = g->hA;
    a.S = g->hS;
    a.drb = g->drb;
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
    // 1. orientation (stages: row search, orientation, dense blocks)
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
    const bool dense = g->dense_min > 0 && nnz > 0;
    if (nnz > 0) HLAUNCH(k_orient_rows, n, g->row_ptr, n, nnz, nb, g->hbrow);
    if (dense) TC_HIP(hipMemsetAsync(g->hsig, 0, (size_t)nI * 8, s));
    build_mark(g, s);
    if (nnz > 0) {
        OrientOut o{g->hrp, g->hcol, g->hcnt, g->dyn_slack > 0 ? g->lcol : nullptr, g->lcnt, g->hbase, g->hoff,
                    g->hloff, dense ? g->hsig : nullptr};
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
    if (dense) {
        const unsigned blocks = (unsigned)std::min<int64_t>(ceil_div(nI, kWpb), 16384);
        hipLaunchKernelGGL(k_dense_test, dim3(blocks), dim3(kBlock), 0, s, g->row_ptr, g->hcol, g->hcnt, g->hsig, n,
                           nI, g->dense_min, g->dflag, g->dtcnt);
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
    return MIS_OK;
}

int hyb_init(GraphCore* g, hipStream_t s) {
    if (g->n > 0)
        hipLaunchKernelGGL(k_hyb_init, dim3(stream_grid(g->n)), dim3(kBlock), 0, s, g->hcnt, g->n, g->hS, g->hA,
                           g->count > 0 ? g->dround : nullptr, g->stripes);
    TC_HIP(hipGetLastError());
    return MIS_OK;
}

// phase 0 = candidate kernel, 1 = exclusion kernel
int hyb_enqueue_phase(GraphCore* g, int phase, int r, hipStream_t s) {
    HybArgs a = make_args(g);
    if (phase == 0) hipLaunchKernelGGL(k_hyb_p1, dim3(g->grid_blocks), dim3(kBlock), 0, s, a, r);
    else hipLaunchKernelGGL(k_hyb_p2, dim3(g->grid_blocks), dim3(kBlock), 0, s, a, r);
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
    hyb_init_body(D.a.hcnt, D.n, D.a.S, D.a.A, nullptr, D.a.stripes, blockIdx.x - bstart[g], bstart[g + 1] - bstart[g]);
}

__global__ void __launch_bounds__(kBlock) k_multi_p1(const MultiDesc* d, const int64_t* bstart, int count, int ri) {
    const int g = graph_of(bstart, count, blockIdx.x);
    const HybArgs& a = d[g].a;
    if (a.ctrl->alive == 0) return;   // finished (and its last round closed) in an earlier launch
    hyb_p1(a, a.ctrl->rbase + ri, blockIdx.x - bstart[g], bstart[g + 1] - bstart[g]);
}

__global__ void __launch_bounds__(kBlock) k_multi_p2(const MultiDesc* d, const int64_t* bstart, int count, int ri) {
    const int g = graph_of(bstart, count, blockIdx.x);
    const HybArgs& a = d[g].a;
    if (a.ctrl->alive == 0) return;
    hyb_p2(a, a.ctrl->rbase + ri, blockIdx.x - bstart[g], bstart[g + 1] - bstart[g]);
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
    size_t sum = 0, rounds = 0, in = 0, bstart = 0, desc = 0;
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
    MultiDesc* d_desc = (MultiDesc*)(base + L.desc);
    std::vector<MultiDesc> desc((size_t)count);
    std::vector<int64_t> bstart((size_t)count + 1, 0);
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
    }
    const int64_t nblocks = bstart[(size_t)count];
    if (nblocks >= (1ll << 31)) { set_error("too many workgroups for one launch"); return MIS_EINVAL; }
    TC_HIP(hipMemcpyAsync(d_desc, desc.data(), desc.size() * sizeof(MultiDesc), hipMemcpyHostToDevice, s));
    TC_HIP(hipMemcpyAsync(d_bstart, bstart.data(), bstart.size() * 8, hipMemcpyHostToDevice, s));
    const dim3 grid((unsigned)nblocks), blk(kBlock), cgrid((unsigned)ceil_div(count, kWpb));
    hipLaunchKernelGGL(k_multi_ctrl, dim3((unsigned)count), blk, 0, s, d_desc, count);
    hipLaunchKernelGGL(k_multi_init, grid, blk, 0, s, d_desc, d_bstart, count);
    TC_HIP(hipGetLastError());
    Ctrl h;
    int32_t r = 0;
    for (;;) {
        for (int i = 1; i <= poll; ++i) {
            hipLaunchKernelGGL(k_multi_p1, grid, blk, 0, s, d_desc, d_bstart, count, i);
            hipLaunchKernelGGL(k_multi_p2, grid, blk, 0, s, d_desc, d_bstart, count, i);
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
