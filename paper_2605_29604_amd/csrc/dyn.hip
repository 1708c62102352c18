// Dynamic graphs: edge insertions and deletions applied in place to a hybrid
// handle's oriented rows, then a local repair of the set (the paper's future-work
// setting of a graph whose structure changes, Section 5).
//
// Priorities stay those of the build (a vertex's key is fixed once it is computed,
// Section 3.1), so after the edits the set to reach is the one the round-synchronous
// rule gives on the new graph with the same keys: the lexicographically-first MIS in
// key order, which satisfies in(v) <=> no u in H(v) is in (H(v) = higher-priority
// neighbours).  An edit {u, v} can only change that recursion at its lower-priority
// end, and a vertex's status can only change if an H-neighbour's did, so only the
// lower ends of the edits and what lies below a vertex that changed need new
// decisions; everything else keeps its status.
//
// Storage: a dynamic handle keeps both orientations in rows of its own (capacity
// deg + slack each): H(v) in hcol, L(v) (lower-priority neighbours) in lcol.  A
// delete writes -1 over the entry in both rows, then every row that lost an entry is
// compacted (once, by the first delete that claims it); an insert appends to both
// rows, after the deletes.
//
// Repair: P = vertices whose status is being recomputed (the edits' lower ends to
// start), S = the set (the previous result to start; stale where P is set).  Round r:
//   cand    v in P is a candidate iff every u in H(v) is neither in P nor in S;
//   decide  candidates join; v in P with a candidate or a settled member in H(v)
//           leaves; the rest stay in P for the next round;
//   apply   decisions are written to S and P; a vertex whose status differs from the
//           one it had before is recorded as flipped;
//   wake    every lower neighbour of a flipped vertex that is not in P joins P.
// The four steps are separate kernels, so no step reads what its own kernel writes.
// A vertex decides only when no H-neighbour is pending, so decisions move down the
// priority order; the repair ends when P is empty, and then the recursion holds
// everywhere (a vertex outside P has kept the status its H-neighbours imply, or it
// would have been woken).
#include "round.hpp"

namespace tcmis {

namespace {

// rcnt layout
enum : int { kRcList0 = 0, kRcList1 = 1, kRcDecided = 2, kRcFlipped = 3, kRcErr = 4, kRcWork = 5, kRcIn = 6,
             kRcMaxRow = 7, kRcWords = 8 };

// The repair re-decides the pending vertices round by round, one wave per long row;
// a pending vertex with a very long H row (a hub of a power-law graph) makes every
// round wait for its scan, and a large pending set costs as much as a solve.  Past
// either bound the set is recomputed by a full solve of the edited handle instead
// (the same result: the recursion has one solution).
constexpr int64_t kRepairRowMax = 4096;   // longest H row among the edits' lower ends
constexpr int64_t kRepairShare = 256;     // pending vertices above n / kRepairShare
enum : int64_t { kErrFull = 1, kErrMissing = 2, kErrEdge = 4 };

__device__ inline uint32_t bitv(const uint32_t* m, int64_t v) { return (m[v >> 5] >> (v & 31)) & 1u; }

struct DynArgs {
    const int64_t* drp;
    int32_t* hcol;
    int32_t* hcnt;
    int32_t* lcol;
    int32_t* lcnt;
    const uint64_t* key;
    int64_t n;
    uint32_t* S;
    uint32_t* P;
    uint32_t* C;
    int32_t* list[2];    // pending vertices by round parity
    int32_t* dec;        // this round's decisions: v (in) or ~v (out)
    uint32_t* claim_h;   // rows claimed for compaction (scratch bitmaps)
    uint32_t* claim_l;
    int32_t* flip;       // this round's flipped vertices
    int64_t* rcnt;
};

// marks v pending; the first marker appends it to list (count at *cnt)
__device__ inline void make_pending(const DynArgs& a, int32_t v, int32_t* list, int64_t* cnt) {
    const uint32_t b = 1u << (v & 31);
    if (!(atomicOr(&a.P[v >> 5], b) & b)) {
        const unsigned long long i = atomicAdd((unsigned long long*)cnt, 1ull);
        list[i] = v;
    }
}

// an edit's lower end: pending, and its H row length into the edits' maximum
__device__ inline void lower_end(const DynArgs& a, int32_t lo) {
    make_pending(a, lo, a.list[1], &a.rcnt[kRcList1]);
    atomicMax((unsigned long long*)&a.rcnt[kRcMaxRow], (unsigned long long)max(a.hcnt[lo], 0));
}

// Rows longer than kDynLight entries (a hub's row holds up to the graph's largest
// degree) are handled by the whole wave, one after another, 64 entries per step; the
// shorter ones on their item's lane.  The kernels below take one item (an edit, a
// pending or a flipped vertex) per thread, and whole waves iterate together
// (DYN_ITEMS) so that those wave steps can ballot.
constexpr int32_t kDynLight = 32;

#define DYN_ITEMS(i, count)                                                                                  \
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x,                                          \
                 i##_end = ((count) + kWave - 1) / kWave * kWave;                                             \
         i < i##_end; i += (int64_t)gridDim.x * blockDim.x)

// With at most as many items as the launch has waves, each item takes a wave of its
// own (every row then on 64 lanes), instead of 64 items sharing one wave.
__device__ inline int64_t wave_index() { return ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; }
__device__ inline int64_t wave_count() { return (int64_t)gridDim.x * (blockDim.x / kWave); }

// sets the entry x of row[0, c) to -1 (the edge is in the row at most once); true if found
__device__ inline bool lane_clear(int32_t* row, int32_t c, int32_t x) {
    for (int32_t j = 0; j < c; ++j)
        if (row[j] == x) {
            row[j] = -1;
            return true;
        }
    return false;
}

// The wave forms take several steps of 64 entries at a time, all their loads in flight
// together (a hub's row takes hundreds of such steps): kDynUnroll where each entry also
// costs bitmap gathers, kClearUnroll where it is only compared or moved.
constexpr int kDynUnroll = 8;
constexpr int kClearUnroll = 16;

__device__ inline bool wave_clear(int32_t* row, int32_t c, int32_t x) {
    for (int32_t k0 = 0; k0 < c; k0 += kClearUnroll * kWave) {
        int32_t u[kClearUnroll];
        #pragma unroll
        for (int q = 0; q < kClearUnroll; ++q) {
            const int32_t j = k0 + q * kWave + lane_id();
            u[q] = j < c ? row[j] : -1;
        }
        #pragma unroll
        for (int q = 0; q < kClearUnroll; ++q) {
            const uint64_t m = ballot(u[q] == x);
            if (m) {
                if (lane_id() == __builtin_ctzll(m)) row[k0 + q * kWave + lane_id()] = -1;
                return true;
            }
        }
    }
    return false;
}

// moves a row's live entries (>= 0) to its front; returns the new count (the wave
// form: each step's entries are all read before any of them is written, and an entry
// moves only towards the front)
__device__ inline int32_t compact_row(int32_t* row, int32_t c) {
    int32_t w = 0;
    for (int32_t j = 0; j < c; ++j) {
        const int32_t x = row[j];
        if (x >= 0) row[w++] = x;
    }
    return w;
}

__device__ inline int32_t wave_compact(int32_t* row, int32_t c) {
    constexpr int kU = kClearUnroll / 2;
    int32_t w = 0;
    for (int32_t k0 = 0; k0 < c; k0 += kU * kWave) {
        int32_t x[kU];
        #pragma unroll
        for (int q = 0; q < kU; ++q) {
            const int32_t j = k0 + q * kWave + lane_id();
            x[q] = j < c ? row[j] : -1;
        }
        #pragma unroll
        for (int q = 0; q < kU; ++q) {
            const uint64_t m = ballot(x[q] >= 0);
            if (x[q] >= 0) row[w + __popcll(m & lanes_below())] = x[q];
            w += __popcll(m);
        }
    }
    return w;
}

// does row[0, c) name a vertex u (>= 0) with hit(u)?  The whole wave, early exit;
// *read (lane 0) counts the entries loaded
template <typename F>
__device__ inline bool wave_any(const int32_t* row, int32_t c, F hit, int64_t* read) {
    int32_t k0 = 0;
    bool any = false;
    {   // the first 64 entries alone (most rows that hit, hit early)
        const int32_t u = lane_id() < c ? row[lane_id()] : -1;
        if (ballot(u >= 0 && hit(u))) any = true;
        k0 = kWave;
    }
    for (; !any && k0 < c; k0 += kDynUnroll * kWave) {
        int32_t u[kDynUnroll];
        #pragma unroll
        for (int q = 0; q < kDynUnroll; ++q) {
            const int32_t j = k0 + q * kWave + lane_id();
            u[q] = j < c ? row[j] : -1;
        }
        bool h = false;
        #pragma unroll
        for (int q = 0; q < kDynUnroll; ++q) h = h | (u[q] >= 0 ? hit(u[q]) : false);
        if (ballot(h)) {
            any = true;
            k0 += kDynUnroll * kWave;
            break;
        }
    }
    if (lane_id() == 0) *read += min(k0, c);
    return any;
}

__global__ void k_dyn_clear(uint32_t* P, uint32_t* C, uint32_t* S, int64_t nw, int64_t* rcnt) {
    GRID_STRIDE(w, nw) {
        P[w] = 0;
        C[w] = 0;
        S[w] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x < kRcWords) rcnt[threadIdx.x] = 0;
}

// after the deletes: every row that lost an entry is compacted once (the first
// delete to claim it does it), so rows hold no deleted entries afterwards
__global__ void k_dyn_compact(DynArgs a, const int32_t* edges, const int8_t* ops, int64_t k) {
    if (k <= wave_count()) {
        const int64_t i = wave_index();
        if (i >= k || ops[i]) return;
        const int32_t u = edges[2 * i], v = edges[2 * i + 1];
        if (u < 0 || v < 0 || u >= a.n || v >= a.n || u == v) return;
        const int32_t hi = a.key[u] > a.key[v] ? u : v, lo = hi == u ? v : u;
        int own = 0;
        if (lane_id() == 0) {
            const uint32_t bl = 1u << (lo & 31), bh = 1u << (hi & 31);
            own = (!(atomicOr(&a.claim_h[lo >> 5], bl) & bl) ? 1 : 0) | (!(atomicOr(&a.claim_l[hi >> 5], bh) & bh) ? 2 : 0);
        }
        own = __shfl(own, 0, kWave);
        if (own & 1) {
            const int32_t c = wave_compact(a.hcol + a.drp[lo], a.hcnt[lo]);
            if (lane_id() == 0) a.hcnt[lo] = c;
        }
        if (own & 2) {
            const int32_t c = wave_compact(a.lcol + a.drp[hi], a.lcnt[hi]);
            if (lane_id() == 0) a.lcnt[hi] = c;
        }
        return;
    }
    DYN_ITEMS(i, k) {
        bool own_h = false, own_l = false;
        int32_t hi = 0, lo = 0;
        if (i < k && !ops[i]) {
            const int32_t u = edges[2 * i], v = edges[2 * i + 1];
            if (u >= 0 && v >= 0 && u < a.n && v < a.n && u != v) {
                hi = a.key[u] > a.key[v] ? u : v;
                lo = hi == u ? v : u;
                const uint32_t bl = 1u << (lo & 31), bh = 1u << (hi & 31);
                own_h = !(atomicOr(&a.claim_h[lo >> 5], bl) & bl);
                own_l = !(atomicOr(&a.claim_l[hi >> 5], bh) & bh);
            }
        }
        const int32_t ch = own_h ? a.hcnt[lo] : 0, cl = own_l ? a.lcnt[hi] : 0;
        if (own_h && ch <= kDynLight) a.hcnt[lo] = compact_row(a.hcol + a.drp[lo], ch);
        if (own_l && cl <= kDynLight) a.lcnt[hi] = compact_row(a.lcol + a.drp[hi], cl);
        for (uint64_t hv = ballot(own_h && ch > kDynLight); hv; hv &= hv - 1) {
            const int l = __builtin_ctzll(hv);
            const int32_t x = __shfl(lo, l, kWave);
            const int32_t c = wave_compact(a.hcol + a.drp[x], __shfl(ch, l, kWave));
            if (lane_id() == 0) a.hcnt[x] = c;
        }
        for (uint64_t hv = ballot(own_l && cl > kDynLight); hv; hv &= hv - 1) {
            const int l = __builtin_ctzll(hv);
            const int32_t x = __shfl(hi, l, kWave);
            const int32_t c = wave_compact(a.lcol + a.drp[x], __shfl(cl, l, kWave));
            if (lane_id() == 0) a.lcnt[x] = c;
        }
    }
}

__global__ void k_dyn_unclaim(uint32_t* claim, int64_t nw) { GRID_STRIDE(w, nw) claim[w] = 0; }

// deletes: -1 over the entry in H(lo) and in L(hi)
__global__ void k_dyn_delete(DynArgs a, const int32_t* edges, const int8_t* ops, int64_t k) {
    if (k <= wave_count()) {
        const int64_t i = wave_index();
        if (i >= k || ops[i]) return;
        const int32_t u = edges[2 * i], v = edges[2 * i + 1];
        if (u < 0 || v < 0 || u >= a.n || v >= a.n || u == v) {
            if (lane_id() == 0) atomicOr((unsigned long long*)&a.rcnt[kRcErr], (unsigned long long)kErrEdge);
            return;
        }
        const int32_t hi = a.key[u] > a.key[v] ? u : v, lo = hi == u ? v : u;
        const bool fh = wave_clear(a.hcol + a.drp[lo], a.hcnt[lo], hi);
        const bool fl = wave_clear(a.lcol + a.drp[hi], a.lcnt[hi], lo);
        if (lane_id() == 0) {
            if (!fh || !fl) atomicOr((unsigned long long*)&a.rcnt[kRcErr], (unsigned long long)kErrMissing);
            lower_end(a, lo);
        }
        return;
    }
    DYN_ITEMS(i, k) {
        bool act = i < k && !ops[i];
        int32_t hi = 0, lo = 0;
        if (act) {
            const int32_t u = edges[2 * i], v = edges[2 * i + 1];
            if (u < 0 || v < 0 || u >= a.n || v >= a.n || u == v) {
                atomicOr((unsigned long long*)&a.rcnt[kRcErr], (unsigned long long)kErrEdge);
                act = false;
            } else {
                hi = a.key[u] > a.key[v] ? u : v;
                lo = hi == u ? v : u;
            }
        }
        const int32_t ch = act ? a.hcnt[lo] : 0, cl = act ? a.lcnt[hi] : 0;
        bool fh = act && ch <= kDynLight && lane_clear(a.hcol + a.drp[lo], ch, hi);
        bool fl = act && cl <= kDynLight && lane_clear(a.lcol + a.drp[hi], cl, lo);
        for (uint64_t hv = ballot(act && ch > kDynLight); hv; hv &= hv - 1) {
            const int l = __builtin_ctzll(hv);
            const int32_t x = __shfl(lo, l, kWave);
            const bool f = wave_clear(a.hcol + a.drp[x], __shfl(ch, l, kWave), __shfl(hi, l, kWave));
            if (lane_id() == l) fh = f;
        }
        for (uint64_t hv = ballot(act && cl > kDynLight); hv; hv &= hv - 1) {
            const int l = __builtin_ctzll(hv);
            const int32_t x = __shfl(hi, l, kWave);
            const bool f = wave_clear(a.lcol + a.drp[x], __shfl(cl, l, kWave), __shfl(lo, l, kWave));
            if (lane_id() == l) fl = f;
        }
        if (act) {
            if (!fh || !fl) atomicOr((unsigned long long*)&a.rcnt[kRcErr], (unsigned long long)kErrMissing);
            lower_end(a, lo);
        }
    }
}

// inserts: append hi to H(lo) and lo to L(hi); a full row gives its slot back
__global__ void k_dyn_insert(DynArgs a, const int32_t* edges, const int8_t* ops, int64_t k) {
    GRID_STRIDE(i, k) {
        if (!ops[i]) continue;
        const int32_t u = edges[2 * i], v = edges[2 * i + 1];
        if (u < 0 || v < 0 || u >= a.n || v >= a.n || u == v) {
            atomicOr((unsigned long long*)&a.rcnt[kRcErr], (unsigned long long)kErrEdge);
            continue;
        }
        const int32_t hi = a.key[u] > a.key[v] ? u : v, lo = hi == u ? v : u;
        const int64_t cap_lo = a.drp[lo + 1] - a.drp[lo], cap_hi = a.drp[hi + 1] - a.drp[hi];
        const int32_t sh = atomicAdd(&a.hcnt[lo], 1);
        if (sh < cap_lo) {
            a.hcol[a.drp[lo] + sh] = hi;
        } else {
            atomicSub(&a.hcnt[lo], 1);
            atomicOr((unsigned long long*)&a.rcnt[kRcErr], (unsigned long long)kErrFull);
        }
        const int32_t sl = atomicAdd(&a.lcnt[hi], 1);
        if (sl < cap_hi) {
            a.lcol[a.drp[hi] + sl] = lo;
        } else {
            atomicSub(&a.lcnt[hi], 1);
            atomicOr((unsigned long long*)&a.rcnt[kRcErr], (unsigned long long)kErrFull);
        }
        lower_end(a, lo);
    }
}

// S from the previous result (one byte per vertex)
__global__ void k_dyn_load(const uint8_t* in_set, int64_t n, uint32_t* S) {
    const int64_t nw = (n + 31) / 32;
    GRID_STRIDE(w, nw) {
        uint32_t x = 0;
        for (int b = 0; b < 32; ++b) {
            const int64_t v = w * 32 + b;
            if (v < n && in_set[v]) x |= 1u << b;
        }
        S[w] = x;
    }
}

// round r, cand: also clears the counters the round's later kernels fill
__global__ void __launch_bounds__(kBlock) k_rep_cand(DynArgs a, int r) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.rcnt[(r + 1) & 1] = 0;
        a.rcnt[kRcDecided] = 0;
        a.rcnt[kRcFlipped] = 0;
    }
    const int32_t* L = a.list[r & 1];
    const int64_t nl = a.rcnt[r & 1];
    int64_t read = 0;
    auto blocks = [&](int32_t u) { return bitv(a.P, u) || bitv(a.S, u); };
    if (nl <= wave_count()) {
        const int64_t i = wave_index();
        if (i >= nl) return;
        const int32_t v = L[i];
        const bool hit = wave_any(a.hcol + a.drp[v], a.hcnt[v], blocks, &read);
        if (!hit && lane_id() == 0) atomicOr(&a.C[v >> 5], 1u << (v & 31));
        return;
    }
    DYN_ITEMS(i, nl) {
        const bool act = i < nl;
        const int32_t v = act ? L[i] : 0;
        const int32_t c = act ? a.hcnt[v] : 0;
        bool cand = act;
        if (act && c <= kDynLight) {
            const int32_t* row = a.hcol + a.drp[v];
            for (int32_t j = 0; j < c && cand; ++j) {
                const int32_t u = row[j];
                if (u >= 0 && blocks(u)) cand = false;
            }
        }
        for (uint64_t hv = ballot(act && c > kDynLight); hv; hv &= hv - 1) {
            const int l = __builtin_ctzll(hv);
            const int32_t x = __shfl(v, l, kWave);
            const bool hit = wave_any(a.hcol + a.drp[x], __shfl(c, l, kWave), blocks, &read);
            if (lane_id() == l) cand = !hit;
        }
        if (cand) atomicOr(&a.C[v >> 5], 1u << (v & 31));
    }
}

// round r, decide: decisions go to the decision list, the undecided to the next list
__global__ void __launch_bounds__(kBlock) k_rep_decide(DynArgs a, int r) {
    const int32_t* L = a.list[r & 1];
    const int64_t nl = a.rcnt[r & 1];
    int64_t work = 0;
    auto excludes = [&](int32_t u) { return bitv(a.C, u) || (!bitv(a.P, u) && bitv(a.S, u)); };
    if (nl <= wave_count()) {
        const int64_t i = wave_index();
        if (i < nl) {
            const int32_t v = L[i];
            if (bitv(a.C, v)) {
                if (lane_id() == 0) a.dec[atomicAdd((unsigned long long*)&a.rcnt[kRcDecided], 1ull)] = v;
            } else {
                const bool out = wave_any(a.hcol + a.drp[v], a.hcnt[v], excludes, &work);
                if (lane_id() == 0) {
                    if (out) a.dec[atomicAdd((unsigned long long*)&a.rcnt[kRcDecided], 1ull)] = ~v;
                    else a.list[(r + 1) & 1][atomicAdd((unsigned long long*)&a.rcnt[(r + 1) & 1], 1ull)] = v;
                }
            }
        }
        if (work) atomicAdd((unsigned long long*)&a.rcnt[kRcWork], (unsigned long long)work);
        return;
    }
    DYN_ITEMS(i, nl) {
        const bool act = i < nl;
        const int32_t v = act ? L[i] : 0;
        const bool in = act && bitv(a.C, v);
        const bool scan = act && !in;
        const int32_t c = scan ? a.hcnt[v] : 0;
        bool out = false;
        if (scan && c <= kDynLight) {
            const int32_t* row = a.hcol + a.drp[v];
            int32_t j = 0;
            for (; j < c && !out; ++j) {
                const int32_t u = row[j];
                if (u >= 0 && excludes(u)) out = true;
            }
            work += j;
        }
        for (uint64_t hv = ballot(scan && c > kDynLight); hv; hv &= hv - 1) {
            const int l = __builtin_ctzll(hv);
            const int32_t x = __shfl(v, l, kWave);
            const bool hit = wave_any(a.hcol + a.drp[x], __shfl(c, l, kWave), excludes, &work);
            if (lane_id() == l) out = hit;
        }
        if (in) a.dec[atomicAdd((unsigned long long*)&a.rcnt[kRcDecided], 1ull)] = v;
        else if (out) a.dec[atomicAdd((unsigned long long*)&a.rcnt[kRcDecided], 1ull)] = ~v;
        else if (act) a.list[(r + 1) & 1][atomicAdd((unsigned long long*)&a.rcnt[(r + 1) & 1], 1ull)] = v;
    }
    if (work) atomicAdd((unsigned long long*)&a.rcnt[kRcWork], (unsigned long long)work);
}

// round r, apply: S and P take the decisions; a changed status is recorded
__global__ void __launch_bounds__(kBlock) k_rep_apply(DynArgs a) {
    const int64_t nd = a.rcnt[kRcDecided];
    GRID_STRIDE(i, nd) {
        const int32_t d = a.dec[i];
        const bool in = d >= 0;
        const int32_t v = in ? d : ~d;
        const uint32_t b = 1u << (v & 31);
        const uint32_t was = in ? atomicOr(&a.S[v >> 5], b) & b : atomicAnd(&a.S[v >> 5], ~b) & b;
        atomicAnd(&a.P[v >> 5], ~b);
        if (in) atomicAnd(&a.C[v >> 5], ~b);
        if ((was != 0) != in) a.flip[atomicAdd((unsigned long long*)&a.rcnt[kRcFlipped], 1ull)] = v;
    }
}

// round r, wake: the lower neighbours of every flipped vertex are pending again
__global__ void __launch_bounds__(kBlock) k_rep_wake(DynArgs a, int r) {
    const int64_t nf = a.rcnt[kRcFlipped];
    int32_t* next = a.list[(r + 1) & 1];
    int64_t* cnt = &a.rcnt[(r + 1) & 1];
    if (nf <= wave_count()) {
        const int64_t i = wave_index();
        if (i >= nf) return;
        const int32_t v = a.flip[i];
        const int32_t c = a.lcnt[v];
        const int32_t* row = a.lcol + a.drp[v];
        for (int32_t j = lane_id(); j < c; j += kWave) {
            const int32_t w = row[j];
            if (w >= 0) make_pending(a, w, next, cnt);
        }
        return;
    }
    DYN_ITEMS(i, nf) {
        const bool act = i < nf;
        const int32_t v = act ? a.flip[i] : 0;
        const int32_t c = act ? a.lcnt[v] : 0;
        if (act && c <= kDynLight) {
            const int32_t* row = a.lcol + a.drp[v];
            for (int32_t j = 0; j < c; ++j) {
                const int32_t w = row[j];
                if (w >= 0) make_pending(a, w, next, cnt);
            }
        }
        for (uint64_t hv = ballot(act && c > kDynLight); hv; hv &= hv - 1) {
            const int l = __builtin_ctzll(hv);
            const int32_t x = __shfl(v, l, kWave), cx = __shfl(c, l, kWave);
            const int32_t* row = a.lcol + a.drp[x];
            for (int32_t k0 = 0; k0 < cx; k0 += kDynUnroll * kWave) {
                int32_t w[kDynUnroll];
                #pragma unroll
                for (int q = 0; q < kDynUnroll; ++q) {
                    const int32_t j = k0 + q * kWave + lane_id();
                    w[q] = j < cx ? row[j] : -1;
                }
                #pragma unroll
                for (int q = 0; q < kDynUnroll; ++q)
                    if (w[q] >= 0) make_pending(a, w[q], next, cnt);
            }
        }
    }
}

// the result bytes and the set size (a workgroup sum, one atomic per workgroup)
__global__ void __launch_bounds__(kBlock) k_dyn_store(const uint32_t* S, int64_t n, uint8_t* in_set, int64_t* n_in) {
    __shared__ int64_t part[kBlock / kWave];
    int64_t cnt = 0;
    GRID_STRIDE(v, n) {
        const uint32_t x = bitv(S, v);
        in_set[v] = (uint8_t)x;
        cnt += x;
    }
    for (int off = kWave / 2; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, kWave);
    if (lane_id() == 0) part[threadIdx.x / kWave] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t sum = 0;
        for (int w = 0; w < kBlock / kWave; ++w) sum += part[w];
        if (sum) atomicAdd((unsigned long long*)n_in, (unsigned long long)sum);
    }
}

DynArgs dyn_args(mis_graph* g) {
    DynArgs a;
    a.drp = g->drp;
    a.hcol = g->hcol;
    a.hcnt = g->hcnt;
    a.lcol = g->lcol;
    a.lcnt = g->lcnt;
    a.key = g->key;
    a.n = g->n;
    a.S = g->rS;
    a.P = g->rP;
    a.C = g->rC;
    a.list[0] = g->rlist[0];
    a.list[1] = g->rlist[1];
    a.dec = g->rdec;
    a.flip = g->rflip;
    a.rcnt = g->rcnt;
    a.claim_h = g->rC;   // free until the repair rounds start
    a.claim_l = g->rS;   // free until the previous result is loaded
    return a;
}

#define DLAUNCH(kernel, work, ...)                                                                            \
    do {                                                                                                      \
        if ((work) > 0) hipLaunchKernelGGL(kernel, dim3(stream_grid(work)), dim3(kBlock), 0, s, __VA_ARGS__); \
        TC_HIP(hipGetLastError());                                                                            \
    } while (0)

}  // namespace

int64_t dyn_counter_words() { return kRcWords; }

}  // namespace tcmis

using namespace tcmis;

extern "C" {

int mis_update_edges(mis_graph* g, const int32_t* edges, const int8_t* ops, int64_t count, uint8_t* in_set,
                     mis_stats* st, void* stream) {
    set_error("");
    if (!g) { set_error("graph is null"); return MIS_EINVAL; }
    if (g->path != MIS_PATH_HYBRID || g->dyn_slack <= 0 || g->count > 0) {
        set_error("edge updates need a single-graph hybrid handle built with dyn_slack > 0");
        return MIS_EINVAL;
    }
    if (count < 0 || (count > 0 && (!edges || !ops))) { set_error("bad edit batch"); return MIS_EINVAL; }
    if (g->n > 0 && !in_set) { set_error("in_set is null"); return MIS_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = g->n, nw = ceil_div(n, 32);
    if (st) {
        st->rounds = 0;
        st->n_in = 0;
    }
    if (n == 0) return MIS_OK;
    DynArgs a = dyn_args(g);
    DLAUNCH(k_dyn_clear, std::max<int64_t>(nw, kRcWords), a.P, a.C, a.S, nw, a.rcnt);
    // a wave per edit (the two kernels take that form when the grid has a wave for each)
    const unsigned egrid = (unsigned)std::min<int64_t>(ceil_div(count, (int64_t)(kBlock / kWave)), 65536);
    if (count > 0) {
        hipLaunchKernelGGL(k_dyn_delete, dim3(egrid), dim3(kBlock), 0, s, a, edges, ops, count);
        hipLaunchKernelGGL(k_dyn_compact, dim3(egrid), dim3(kBlock), 0, s, a, edges, ops, count);
        TC_HIP(hipGetLastError());
    }
    DLAUNCH(k_dyn_unclaim, nw, a.C, nw);
    DLAUNCH(k_dyn_insert, count, a, edges, ops, count);
    DLAUNCH(k_dyn_load, nw, in_set, n, a.S);
    const dim3 grid((unsigned)std::max(1, g->grid_blocks)), blk(kBlock);
    int64_t h[kRcWords] = {};
    TC_HIP(hipMemcpyAsync(h, a.rcnt, sizeof(h), hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    if (h[kRcErr] & kErrEdge) { set_error("an edit names a vertex out of range or a self-loop"); return MIS_EINVAL; }
    if (h[kRcErr] & kErrMissing) { set_error("a deleted edge was not in the graph"); return MIS_EINVAL; }
    if (h[kRcErr] & kErrFull) {
        set_error("a row has no slot left for an inserted edge: rebuild with a larger dyn_slack");
        return MIS_ENOMEM;
    }
    if (h[kRcMaxRow] > kRepairRowMax || h[kRcList1] * kRepairShare > n) {
        mis_stats full = {};
        TC_CHECK(mis_solve(g, in_set, 0, nullptr, 0, &full, stream));
        if (st) {
            st->rounds = full.rounds;
            st->n_in = full.n_in;
            st->units[0] = full.units[0] + full.units[2];
        }
        return MIS_OK;
    }
    int r = 0;
    const int poll = std::max(1, g->poll_rounds);
    for (;;) {
        for (int i = 0; i < poll; ++i) {
            ++r;
            hipLaunchKernelGGL(k_rep_cand, grid, blk, 0, s, a, r);
            hipLaunchKernelGGL(k_rep_decide, grid, blk, 0, s, a, r);
            hipLaunchKernelGGL(k_rep_apply, grid, blk, 0, s, a);
            hipLaunchKernelGGL(k_rep_wake, grid, blk, 0, s, a, r);
        }
        TC_HIP(hipGetLastError());
        TC_HIP(hipMemcpyAsync(h, a.rcnt, sizeof(h), hipMemcpyDeviceToHost, s));
        TC_HIP(hipStreamSynchronize(s));
        if (h[kRcErr] & kErrEdge) { set_error("an edit names a vertex out of range or a self-loop"); return MIS_EINVAL; }
        if (h[kRcErr] & kErrMissing) { set_error("a deleted edge was not in the graph"); return MIS_EINVAL; }
        if (h[kRcErr] & kErrFull) {
            set_error("a row has no slot left for an inserted edge: rebuild with a larger dyn_slack");
            return MIS_ENOMEM;
        }
        if (h[(r + 1) & 1] == 0) break;   // nothing pending for the next round
        if (r > 2 * n + 16) { set_error("repair did not settle"); return MIS_EINTERNAL; }
    }
    TC_HIP(hipMemsetAsync(a.rcnt + kRcIn, 0, 8, s));
    hipLaunchKernelGGL(k_dyn_store, dim3((unsigned)std::min<int64_t>(ceil_div(n, kBlock), 1024)), dim3(kBlock), 0, s,
                       a.S, n, in_set, a.rcnt + kRcIn);
    TC_HIP(hipGetLastError());
    if (st) {
        int64_t nin = 0;
        TC_HIP(hipMemcpyAsync(&nin, a.rcnt + kRcIn, 8, hipMemcpyDeviceToHost, s));
        TC_HIP(hipStreamSynchronize(s));
        st->rounds = r;
        st->n_in = nin;
        st->units[0] = h[kRcWork];
    }
    return MIS_OK;
}

}  // extern "C"
