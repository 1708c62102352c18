// Scalar CSR path: the three phases of Algorithm 2 directly on the adjacency lists.
//
// Per-vertex state: st[v] = 0 while undecided, else (round << 2) | IN/OUT;
// ak[v] = key[v] while undecided, 0 once decided (a decided neighbour, like a
// lower-priority one, never blocks: 0 is the smallest key).
//
// Round r, candidate kernel (Phase 1): an undecided vertex v is a candidate iff no
// neighbour u has ak[u] > key[v] (early exit on the first such neighbour); the
// kernel writes st[v] = IN@r.  ak is not modified in this kernel, so every vertex
// sees the alive set of the round start.
// Round r, exclusion kernel (Phases 2 and 3 fused): a candidate (st == IN@r) is
// retired; an undecided non-candidate scans for a neighbour with st == IN@r
// (N_c(v) > 0, early exit) and becomes OUT@r; the rest go to the next round's
// active list.  Concurrent OUT@r writes never look like IN@r, so the scan reads a
// consistent candidate set without double buffering.
#include "round.hpp"

namespace tcmis {

namespace {

struct CsrArgs {
    const int64_t* rp;
    const int32_t* ci;
    const uint64_t* key;
    uint64_t* ak;
    uint32_t* st;
    Ctrl* ctrl;
    int64_t* stripes;
    TraceRec* trace;
    const int32_t* master[2];   // initial light / heavy lists (round 1)
    const Meta* meta;           // meta->n_light: length of the light list
    int64_t n;
    int32_t* act[2][2];         // [buffer][light, heavy]
};

__device__ inline void round_lists(const CsrArgs& a, int r, const int32_t** in_l, int64_t* n_l,
                                   const int32_t** in_h, int64_t* n_h) {
    if (r == 1) {
        *in_l = a.master[0]; *n_l = a.meta->n_light;
        *in_h = a.master[1]; *n_h = a.n - a.meta->n_light;
    } else {
        const int b = (r - 1) & 1;
        *in_l = a.act[b][0]; *n_l = a.ctrl->n_act[b][0];
        *in_h = a.act[b][1]; *n_h = a.ctrl->n_act[b][1];
    }
}

__device__ void csr_cand(const CsrArgs& a, int r) {
    open_round(a.ctrl, a.stripes, a.trace, r);
    const int32_t *L, *H;
    int64_t nl, nh;
    round_lists(a, r, &L, &nl, &H, &nh);
    if (nl + nh == 0) return;
    const int lane = lane_id();
    const int64_t nthreads = (int64_t)gridDim.x * kBlock;
    const int64_t tid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int64_t n_cand = 0, edges = 0, verts = 0;
    // light vertices: one lane each
    for (int64_t i = tid; i < nl; i += nthreads) {
        const int v = L[i];
        const uint64_t kv = a.key[v];
        const int64_t e1 = a.rp[v + 1];
        bool blocked = false;
        int64_t e = a.rp[v];
        for (; e < e1; ++e) {
            if (a.ak[a.ci[e]] > kv) { blocked = true; ++e; break; }
        }
        edges += e - a.rp[v];
        ++verts;
        if (!blocked) { a.st[v] = tag(r, kIn); ++n_cand; }
    }
    // heavy vertices: one wave each, 64 neighbours per step, ballot early exit
    const int64_t nwaves = nthreads / kWave;
    for (int64_t w = tid / kWave; w < nh; w += nwaves) {
        const int v = H[w];
        const uint64_t kv = a.key[v];
        const int64_t e0 = a.rp[v], e1 = a.rp[v + 1];
        bool blocked = false;
        int64_t e = e0;
        for (; e < e1; e += kWave) {
            const int64_t idx = e + lane;
            const bool b = idx < e1 && a.ak[a.ci[idx]] > kv;
            if (ballot(b)) { blocked = true; e += kWave; break; }
        }
        if (lane == 0) {
            edges += min(e, e1) - e0;
            ++verts;
            if (!blocked) { a.st[v] = tag(r, kIn); ++n_cand; }
        }
    }
    int64_t x[3] = {n_cand, edges, verts};
    block_count(a.stripes, r, {0, 2, 3}, x);
}

__device__ void csr_excl(const CsrArgs& a, int r) {
    __shared__ int32_t lbuf[kBlock / kWave][2][kWave];
    const uint32_t in_r = tag(r, kIn), out_r = tag(r, kOut);
    const int32_t *L, *H;
    int64_t nl, nh;
    round_lists(a, r, &L, &nl, &H, &nh);
    if (nl + nh == 0) return;
    int32_t* nextL = a.act[r & 1][0];
    int32_t* nextH = a.act[r & 1][1];
    int64_t* cntL = &a.ctrl->n_act[r & 1][0];
    int64_t* cntH = &a.ctrl->n_act[r & 1][1];
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    int32_t* bufL = lbuf[wid][0];
    int32_t* bufH = lbuf[wid][1];
    int pendL = 0, pendH = 0;
    const int64_t nthreads = (int64_t)gridDim.x * kBlock;
    const int64_t tid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int64_t n_out = 0, edges = 0, verts = 0;
    const int64_t nl_round = (nl + kWave - 1) / kWave * kWave;   // whole waves iterate together
    for (int64_t i0 = tid; i0 < nl_round; i0 += nthreads) {
        const bool valid = i0 < nl;
        const int v = valid ? L[i0] : 0;
        bool keep = false;
        if (valid) {
            const uint32_t s = a.st[v];
            if (s == in_r) {
                a.ak[v] = 0;
            } else {
                const int64_t e0 = a.rp[v], e1 = a.rp[v + 1];
                bool hit = false;
                int64_t e = e0;
                for (; e < e1; ++e) {
                    if (a.st[a.ci[e]] == in_r) { hit = true; ++e; break; }
                }
                edges += e - e0;
                ++verts;
                if (hit) { a.st[v] = out_r; a.ak[v] = 0; ++n_out; }
                else keep = true;
            }
        }
        lbuf_push(bufL, pendL, nextL, cntL, keep, v);
    }
    lbuf_flush(bufL, pendL, nextL, cntL);
    const int64_t nwaves = nthreads / kWave;
    for (int64_t w = tid / kWave; w < nh; w += nwaves) {
        const int v = H[w];
        const uint32_t s = a.st[v];
        if (s == in_r) {
            if (lane == 0) a.ak[v] = 0;
            continue;
        }
        const int64_t e0 = a.rp[v], e1 = a.rp[v + 1];
        bool hit = false;
        int64_t e = e0;
        for (; e < e1; e += kWave) {
            const int64_t idx = e + lane;
            const bool b = idx < e1 && a.st[a.ci[idx]] == in_r;
            if (ballot(b)) { hit = true; e += kWave; break; }
        }
        if (lane == 0) {
            edges += min(e, e1) - e0;
            ++verts;
            if (hit) { a.st[v] = out_r; a.ak[v] = 0; ++n_out; }
        }
        lbuf_push(bufH, pendH, nextH, cntH, lane == 0 && !hit, v);
    }
    lbuf_flush(bufH, pendH, nextH, cntH);
    int64_t x[3] = {n_out, edges, verts};
    block_count(a.stripes, r, {1, 4, 5}, x);
}

// One kernel per phase; round r = the batch base on the device + ri.
__global__ void __launch_bounds__(kBlock) k_csr_cand(CsrArgs a, int ri) { csr_cand(a, a.ctrl->rbase + ri); }
__global__ void __launch_bounds__(kBlock) k_csr_excl(CsrArgs a, int ri) { csr_excl(a, a.ctrl->rbase + ri); }

// Persistent variant: k rounds in one cooperative launch, a grid barrier after
// every phase; the last round is closed and the base advanced at the end.
__global__ void __launch_bounds__(kBlock) k_csr_rounds(CsrArgs a, int k) {
    const int rb = a.ctrl->rbase;
    for (int ri = 1; ri <= k; ++ri) {
        csr_cand(a, rb + ri);
        grid_barrier(a.ctrl);
        csr_excl(a, rb + ri);
        grid_barrier(a.ctrl);
    }
    finish_rounds(a.ctrl, a.stripes, a.trace, rb, k);
}

__global__ void k_csr_init(const uint64_t* key, uint64_t* ak, uint32_t* st, int64_t n) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        ak[v] = key[v];
        st[v] = 0;
    }
}

// with `gate`: only once every vertex is decided (see k_tile_output)
__global__ void k_csr_output(const Ctrl* gate, const uint32_t* st, int64_t n, uint8_t* in_set) {
    if (gate && gate->alive != 0) return;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        in_set[v] = (st[v] & 3u) == kIn ? 1 : 0;
}

CsrArgs make_args(GraphCore* g) {
    CsrArgs a;
    a.rp = g->row_ptr; a.ci = g->col_idx; a.key = g->key; a.ak = g->ak; a.st = g->st;
    a.ctrl = g->ctrl; a.stripes = g->stripes; a.trace = g->trace;
    a.master[0] = g->light; a.master[1] = g->heavy;
    a.meta = g->meta; a.n = g->n;
    for (int b = 0; b < 2; ++b)
        for (int k = 0; k < 2; ++k) a.act[b][k] = g->act[b][k];
    return a;
}

}  // namespace

// k rounds as one cooperative launch (see k_csr_rounds)
int csr_enqueue_rounds(GraphCore* g, int k, hipStream_t s) {
    CsrArgs a = make_args(g);
    return launch_cooperative((const void*)k_csr_rounds, g, &a, k, s);
}

int csr_init(GraphCore* g, hipStream_t s) {
    if (g->n > 0)
        hipLaunchKernelGGL(k_csr_init, dim3(stream_grid(g->n)), dim3(kBlock), 0, s, g->key, g->ak, g->st, g->n);
    TC_HIP(hipGetLastError());
    return MIS_OK;
}

// phase 0 = candidate kernel, 1 = exclusion kernel (which closes the round)
int csr_enqueue_phase(GraphCore* g, int phase, int r, hipStream_t s) {
    CsrArgs a = make_args(g);
    if (phase == 0) hipLaunchKernelGGL(k_csr_cand, dim3(g->grid_blocks), dim3(kBlock), 0, s, a, r);
    else hipLaunchKernelGGL(k_csr_excl, dim3(g->grid_blocks), dim3(kBlock), 0, s, a, r);
    TC_HIP(hipGetLastError());
    return MIS_OK;
}

int csr_output(GraphCore* g, uint8_t* in_set, bool if_done, hipStream_t s) {
    if (g->n > 0)
        hipLaunchKernelGGL(k_csr_output, dim3(stream_grid(g->n)), dim3(kBlock), 0, s, if_done ? g->ctrl : nullptr,
                           g->st, g->n, in_set);
    TC_HIP(hipGetLastError());
    return MIS_OK;
}

}  // namespace tcmis
