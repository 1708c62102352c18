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
             kRcWords = 8 };
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

__global__ void k_dyn_clear(uint32_t* P, uint32_t* C, uint32_t* S, int64_t nw, int64_t* rcnt) {
    GRID_STRIDE(w, nw) {
        P[w] = 0;
        C[w] = 0;
        S[w] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x < kRcWords) rcnt[threadIdx.x] = 0;
}

// moves a row's live entries (>= 0) to its front; returns the new count
__device__ inline int32_t compact_row(int32_t* row, int32_t c) {
    int32_t w = 0;
    for (int32_t j = 0; j < c; ++j) {
        const int32_t x = row[j];
        if (x >= 0) row[w++] = x;
    }
    return w;
}

// after the deletes: every row that lost an entry is compacted once (the first
// delete to claim it does it), so rows hold no deleted entries afterwards
__global__ void k_dyn_compact(DynArgs a, const int32_t* edges, const int8_t* ops, int64_t k) {
    GRID_STRIDE(i, k) {
        if (ops[i]) continue;
        const int32_t u = edges[2 * i], v = edges[2 * i + 1];
        if (u < 0 || v < 0 || u >= a.n || v >= a.n || u == v) continue;
        const int32_t hi = a.key[u] > a.key[v] ? u : v, lo = hi == u ? v : u;
        const uint32_t bl = 1u << (lo & 31), bh = 1u << (hi & 31);
        if (!(atomicOr(&a.claim_h[lo >> 5], bl) & bl)) a.hcnt[lo] = compact_row(a.hcol + a.drp[lo], a.hcnt[lo]);
        if (!(atomicOr(&a.claim_l[hi >> 5], bh) & bh)) a.lcnt[hi] = compact_row(a.lcol + a.drp[hi], a.lcnt[hi]);
    }
}

__global__ void k_dyn_unclaim(uint32_t* claim, int64_t nw) { GRID_STRIDE(w, nw) claim[w] = 0; }

// deletes: -1 over the entry in H(lo) and in L(hi)
__global__ void k_dyn_delete(DynArgs a, const int32_t* edges, const int8_t* ops, int64_t k) {
    GRID_STRIDE(i, k) {
        if (ops[i]) continue;
        const int32_t u = edges[2 * i], v = edges[2 * i + 1];
        if (u < 0 || v < 0 || u >= a.n || v >= a.n || u == v) {
            atomicOr((unsigned long long*)&a.rcnt[kRcErr], (unsigned long long)kErrEdge);
            continue;
        }
        const int32_t hi = a.key[u] > a.key[v] ? u : v, lo = hi == u ? v : u;
        bool fh = false, fl = false;
        const int32_t ch = a.hcnt[lo], cl = a.lcnt[hi];
        for (int32_t j = 0; j < ch && !fh; ++j) fh = atomicCAS(&a.hcol[a.drp[lo] + j], hi, -1) == hi;
        for (int32_t j = 0; j < cl && !fl; ++j) fl = atomicCAS(&a.lcol[a.drp[hi] + j], lo, -1) == lo;
        if (!fh || !fl) atomicOr((unsigned long long*)&a.rcnt[kRcErr], (unsigned long long)kErrMissing);
        make_pending(a, lo, a.list[1], &a.rcnt[kRcList1]);
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
        make_pending(a, lo, a.list[1], &a.rcnt[kRcList1]);
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
    GRID_STRIDE(i, nl) {
        const int32_t v = L[i];
        const int64_t e0 = a.drp[v];
        const int32_t c = a.hcnt[v];
        bool cand = true;
        for (int32_t j = 0; j < c && cand; ++j) {
            const int32_t u = a.hcol[e0 + j];
            if (u >= 0 && (bitv(a.P, u) || bitv(a.S, u))) cand = false;
        }
        if (cand) atomicOr(&a.C[v >> 5], 1u << (v & 31));
    }
}

// round r, decide: decisions go to the decision list, the undecided to the next list
__global__ void __launch_bounds__(kBlock) k_rep_decide(DynArgs a, int r) {
    const int32_t* L = a.list[r & 1];
    const int64_t nl = a.rcnt[r & 1];
    int64_t work = 0;
    GRID_STRIDE(i, nl) {
        const int32_t v = L[i];
        if (bitv(a.C, v)) {
            a.dec[atomicAdd((unsigned long long*)&a.rcnt[kRcDecided], 1ull)] = v;
            continue;
        }
        const int64_t e0 = a.drp[v];
        const int32_t c = a.hcnt[v];
        bool out = false;
        int32_t j = 0;
        for (; j < c && !out; ++j) {
            const int32_t u = a.hcol[e0 + j];
            if (u >= 0 && (bitv(a.C, u) || (!bitv(a.P, u) && bitv(a.S, u)))) out = true;
        }
        work += j;
        if (out) a.dec[atomicAdd((unsigned long long*)&a.rcnt[kRcDecided], 1ull)] = ~v;
        else a.list[(r + 1) & 1][atomicAdd((unsigned long long*)&a.rcnt[(r + 1) & 1], 1ull)] = v;
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
    GRID_STRIDE(i, nf) {
        const int32_t v = a.flip[i];
        const int64_t e0 = a.drp[v];
        const int32_t c = a.lcnt[v];
        for (int32_t j = 0; j < c; ++j) {
            const int32_t w = a.lcol[e0 + j];
            if (w >= 0) make_pending(a, w, a.list[(r + 1) & 1], &a.rcnt[(r + 1) & 1]);
        }
    }
}

__global__ void k_dyn_store(const uint32_t* S, int64_t n, uint8_t* in_set, int64_t* n_in) {
    int64_t cnt = 0;
    GRID_STRIDE(v, n) {
        const uint32_t x = bitv(S, v);
        in_set[v] = (uint8_t)x;
        cnt += x;
    }
    for (int off = kWave / 2; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, kWave);
    if (lane_id() == 0 && cnt) atomicAdd((unsigned long long*)n_in, (unsigned long long)cnt);
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
    DLAUNCH(k_dyn_delete, count, a, edges, ops, count);
    DLAUNCH(k_dyn_compact, count, a, edges, ops, count);
    DLAUNCH(k_dyn_unclaim, nw, a.C, nw);
    DLAUNCH(k_dyn_insert, count, a, edges, ops, count);
    DLAUNCH(k_dyn_load, nw, in_set, n, a.S);
    const dim3 grid((unsigned)std::max(1, g->grid_blocks)), blk(kBlock);
    int64_t h[kRcWords] = {};
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
    DLAUNCH(k_dyn_store, n, a.S, n, in_set, a.rcnt + kRcIn);
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
