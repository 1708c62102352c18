// Device helpers shared by the round kernels of both paths.
#pragma once
#include "graph.hpp"

namespace tcmis {

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

// Adds per-thread counts to round r's counters: a wave sum, a workgroup sum in LDS,
// then one atomic per counter into the workgroup's stripe.  Every thread of the
// workgroup must call it (it synchronises the workgroup).
// (blk: the workgroup's index within the launch, or within its graph's share of a
// launch over several graphs)
template <int N>
__device__ inline void block_count(int64_t* stripes, int r, const int (&idx)[N], int64_t (&x)[N],
                                   int64_t blk = -1) {
    __shared__ int64_t part[kBlock / kWave][N];
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    #pragma unroll
    for (int i = 0; i < N; ++i) {
        for (int off = kWave / 2; off > 0; off >>= 1) x[i] += __shfl_xor(x[i], off, kWave);
        if (lane == 0) part[wid][i] = x[i];
    }
    __syncthreads();
    if (threadIdx.x < N) {
        int64_t sum = 0;
        for (int w = 0; w < kBlock / kWave; ++w) sum += part[w][threadIdx.x];
        const int64_t b = blk < 0 ? (int64_t)blockIdx.x : blk;
        int64_t* st = stripes + ((int64_t)(r & 1) * kStripes + b % kStripes) * kStripeWords;
        if (sum) atomicAdd((unsigned long long*)&st[idx[threadIdx.x]], (unsigned long long)sum);
    }
}

// Closes round r (one full wave, uniform control flow): sums and clears the
// round's counter stripes, writes its trace record and advances `round` and
// `alive`.  A round that is already closed, or that ran after every vertex was
// decided, is left alone.  trace == nullptr: no trace record.
__device__ inline void close_round(Ctrl* ctrl, int64_t* stripes, TraceRec* trace, int r) {
    if (r < 1 || ctrl->round != r - 1 || ctrl->alive == 0) return;
    const int lane = lane_id();
    int64_t v[2 + kUnits];
    #pragma unroll
    for (int i = 0; i < 2 + kUnits; ++i) v[i] = 0;
    for (int s = lane; s < kStripes; s += kWave) {   // kStripes / kWave stripes per lane
        int64_t* st = stripes + ((int64_t)(r & 1) * kStripes + s) * kStripeWords;
        #pragma unroll
        for (int i = 0; i < 2 + kUnits; ++i) v[i] += atomic_read(&st[i]);
        #pragma unroll
        for (int i = 0; i < 2 + kUnits; ++i) st[i] = 0;
    }
    #pragma unroll
    for (int i = 0; i < 2 + kUnits; ++i)
        for (int off = kWave / 2; off > 0; off >>= 1) v[i] += __shfl_xor(v[i], off, kWave);
    if (lane == 0) {
        TraceRec rec;
        rec.c = v[0];
        rec.x = v[1];
        rec.alive = ctrl->alive - rec.c - rec.x;
        rec.round = r;
        for (int i = 0; i < kUnits; ++i) rec.u[i] = v[2 + i];
        if (trace) trace[(r - 1) % kTraceCap] = rec;
        ctrl->n_in += rec.c;
        ctrl->alive = rec.alive;
        ctrl->round = r;
    }
}

// Before round 1: the control block (alive = n, the rest zero), the round's copy of
// the build sizes, and the counter stripes.  Every thread of one workgroup calls it.
__device__ inline void ctrl_reset(Ctrl* ctrl, Meta* smeta, const Meta* meta, int64_t* stripes, int64_t n) {
    if (threadIdx.x == 0) {
        Ctrl c;
        memset(&c, 0, sizeof(c));
        c.alive = n;
        *ctrl = c;
        *smeta = *meta;
    }
    for (int i = threadIdx.x; i < 2 * kStripes * kStripeWords; i += blockDim.x) stripes[i] = 0;
}

// Round prologue run by the first wave of round r's first kernel: closes round
// r-1 and empties the lists that round r's last kernel fills.
__device__ inline void open_round(Ctrl* ctrl, int64_t* stripes, TraceRec* trace, int r, int64_t blk = -1) {
    if ((blk < 0 ? (int64_t)blockIdx.x : blk) == 0 && threadIdx.x < kWave) {
        close_round(ctrl, stripes, trace, r - 1);
        if (threadIdx.x < 4) ctrl->n_act[r & 1][threadIdx.x] = 0;
    }
}

constexpr uint32_t kErrBarrier = 1u << 8;   // Ctrl::error: a grid barrier wait hit its bound
constexpr uint32_t kBarrierSpin = 1u << 22;  // polls (each after a short sleep) before giving up

// Grid-wide barrier of a cooperative launch (every workgroup is co-resident).  The
// arrival counter only grows, so the barrier needs no reset and no generation word:
// the workgroup whose arrival completes a multiple of the grid size releases the
// others.  An agent-scope fence before arriving and after leaving makes every
// workgroup's writes of the phase visible to all workgroups of the next one.  The
// wait is bounded: after kBarrierSpin polls a workgroup raises kErrBarrier and goes
// on, so every wave always reaches the end of the kernel.
__device__ inline void grid_barrier(Ctrl* ctrl) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned long long n = gridDim.x;
        const unsigned long long old = atomicAdd(&ctrl->bar, 1ull);
        const unsigned long long target = (old / n + 1) * n;
        uint32_t spins = 0;
        while (__hip_atomic_load(&ctrl->bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (++spins > kBarrierSpin) {
                atomicOr(&ctrl->error, kErrBarrier);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        __threadfence();
    }
    __syncthreads();
}

// End of a persistent batch of k rounds from base rb (after the last barrier):
// closes round rb + k and moves the base past it.
__device__ inline void finish_rounds(Ctrl* ctrl, int64_t* stripes, TraceRec* trace, int rb, int k) {
    if (blockIdx.x == 0 && threadIdx.x < kWave) {
        close_round(ctrl, stripes, trace, rb + k);
        if (threadIdx.x == 0) ctrl->rbase = rb + k;
    }
}

// Cooperative launch of a persistent round kernel taking (args, k); defined with
// the round loop.
int launch_cooperative(const void* kernel, GraphCore* g, void* args, int k, hipStream_t s);

}  // namespace tcmis
