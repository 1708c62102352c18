// Device helpers shared by the round kernels of both paths.
#pragma once
#include "graph.hpp"

namespace tcmis {

// Makes this wave's earlier LDS writes visible to its other lanes and keeps the
// compiler from moving LDS accesses across the point.
__device__ inline void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Sum of a per-lane value over the wave, added with one atomic.
__device__ inline void wave_add(int64_t* p, int64_t x) {
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
    if (lane_id() == 0 && x) atomicAdd((unsigned long long*)p, (unsigned long long)x);
}

// Per-wave LDS staging buffer for list appends: items collect in LDS and are
// written with one atomic per 64 items.  `pend` is wave-uniform.
__device__ inline void lbuf_flush(int32_t* lbuf, int& pend, int32_t* list, int64_t* count) {
    if (pend == 0) return;
    wave_sync_lds();
    unsigned long long base = 0;
    if (lane_id() == 0) base = atomicAdd((unsigned long long*)count, (unsigned long long)pend);
    base = __shfl(base, 0, kWave);
    if (lane_id() < pend) list[base + lane_id()] = lbuf[lane_id()];
    wave_sync_lds();
    pend = 0;
}

__device__ inline void lbuf_push(int32_t* lbuf, int& pend, int32_t* list, int64_t* count, bool keep, int32_t v) {
    const uint64_t b = ballot(keep);
    const int k = __popcll(b);
    if (k == 0) return;
    if (pend + k > kWave) lbuf_flush(lbuf, pend, list, count);
    if (keep) lbuf[pend + __popcll(b & lanes_below())] = v;
    pend += k;
}

__device__ inline int64_t atomic_read(int64_t* p) {
    return (int64_t)__hip_atomic_load((unsigned long long*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Closes round r (one thread): moves its counters into the trace ring and advances
// `round` and `alive`.  A round that is already closed, or that ran after every
// vertex was decided, is left alone.
__device__ inline void close_round(Ctrl* ctrl, TraceRec* trace, int r) {
    if (r < 1 || ctrl->round != r - 1 || ctrl->alive == 0) return;
    int64_t* c = ctrl->cnt[r & 1];
    TraceRec rec;
    rec.c = atomic_read(&c[0]);
    rec.x = atomic_read(&c[1]);
    rec.alive = ctrl->alive - rec.c - rec.x;
    rec.round = r;
    for (int i = 0; i < 4; ++i) rec.u[i] = atomic_read(&c[2 + i]);
    trace[(r - 1) % kTraceCap] = rec;
    for (int i = 0; i < 6; ++i) c[i] = 0;
    ctrl->n_in += rec.c;
    ctrl->alive = rec.alive;
    ctrl->round = r;
}

// Round prologue run by the first thread of round r's candidate kernel: closes
// round r-1 and empties the list that round r's exclusion kernel fills.
__device__ inline void open_round(Ctrl* ctrl, TraceRec* trace, int r) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        close_round(ctrl, trace, r - 1);
        ctrl->n_act[r & 1][0] = 0;
        ctrl->n_act[r & 1][1] = 0;
    }
}

}  // namespace tcmis
