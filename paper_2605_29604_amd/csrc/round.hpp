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

// Called by every workgroup at the end of a round's last kernel.  The workgroup
// that finishes last closes the round: it moves the counters into the trace ring
// and advances the round state, after every other workgroup has exited.
__device__ inline void finish_round(Ctrl* ctrl, TraceRec* trace, int r) {
    __syncthreads();
    if (threadIdx.x != 0) return;
    __threadfence();
    const uint32_t prev = atomicAdd(&ctrl->blocks_done, 1u);
    if (prev != gridDim.x - 1) return;
    __threadfence();
    const int64_t c = (int64_t)atomicAdd((unsigned long long*)&ctrl->cnt_c, 0ull);
    const int64_t x = (int64_t)atomicAdd((unsigned long long*)&ctrl->cnt_x, 0ull);
    const int64_t alive = ctrl->alive - c - x;
    TraceRec rec;
    rec.c = c;
    rec.x = x;
    rec.alive = alive;
    rec.round = r;
    for (int i = 0; i < 4; ++i) rec.u[i] = (int64_t)atomicExch((unsigned long long*)&ctrl->u[i], 0ull);
    trace[(r - 1) % kTraceCap] = rec;
    ctrl->n_in += c;
    ctrl->alive = alive;
    atomicExch((unsigned long long*)&ctrl->cnt_c, 0ull);
    atomicExch((unsigned long long*)&ctrl->cnt_x, 0ull);
    ctrl->round = r;
    atomicExch(&ctrl->blocks_done, 0u);
    __threadfence();
}

}  // namespace tcmis
