// Internal helpers shared by the library's HIP sources (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/tcmis.h"

namespace tcmis {

constexpr int kWave = 64;        // CDNA wavefront width
constexpr int kBlock = 256;      // threads per workgroup for streaming kernels

// Per-vertex round state of the CSR path and the tile path's bookkeeping both tag
// decisions with the round that made them: 0 = undecided, else (round << 2) | code.
constexpr uint32_t kIn = 1u, kOut = 2u;
__host__ __device__ inline uint32_t tag(uint32_t round, uint32_t code) { return (round << 2) | code; }

void set_error(const std::string& msg);

#define TC_HIP(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) {                                                        \
            ::tcmis::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));     \
            return MIS_EHIP;                                                           \
        }                                                                              \
    } while (0)

#define TC_CHECK(expr)                          \
    do {                                        \
        int rc_ = (expr);                       \
        if (rc_ != MIS_OK) return rc_;          \
    } while (0)

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// grid for a grid-stride streaming kernel over `work` items
inline unsigned stream_grid(int64_t work, int per_thread = 1) {
    int64_t blocks = ceil_div(work, (int64_t)kBlock * per_thread);
    if (blocks < 1) blocks = 1;
    if (blocks > 65536) blocks = 65536;
    return (unsigned)blocks;
}

#define GRID_STRIDE(i, count) \
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (count); i += (int64_t)gridDim.x * blockDim.x)

// SplitMix64 (Steele, Lea, Flood 2014): output i of the stream seeded with s
__device__ inline uint64_t splitmix_at(uint64_t s, uint64_t i) {
    uint64_t z = s + i * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// ---- wave primitives -------------------------------------------------------
__device__ inline int lane_id() { return (int)__lane_id(); }
__device__ inline uint64_t ballot(bool p) { return __ballot(p); }
__device__ inline uint64_t lanes_below() { return (1ull << lane_id()) - 1ull; }

// Makes this wave's earlier LDS writes visible to its other lanes and keeps the
// compiler from moving LDS accesses across the point.
__device__ inline void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Lanes that share a key I are adjacent (I < 0: none).  ORs each run's masks in
// registers (segmented suffix scan) and lets the run's first lane apply the result
// to dst[I] with one atomic OR.  Every lane of the wave must call it.
__device__ inline void run_or(int32_t I, uint32_t m, uint32_t* dst) {
    const int lane = lane_id();
    #pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t mo = (uint32_t)__shfl_down((int)m, off, kWave);
        const int32_t Io = __shfl_down(I, off, kWave);
        if (lane + off < kWave && Io == I) m |= mo;
    }
    const int32_t Ip = __shfl_up(I, 1, kWave);
    if ((lane == 0 || Ip != I) && I >= 0 && m) atomicOr(&dst[I], m);
}

// Prefix scans (no allocation; `scratch` holds scan_scratch_elems(count) elements
// of the scanned type; d_total, if given, receives the grand total on the device).
int64_t scan_scratch_elems(int64_t count);
int scan_excl_i32(const int32_t* in, int32_t* out, int64_t count, int32_t* d_total, int32_t* scratch, hipStream_t s);
int scan_excl_i64(const int64_t* in, int64_t* out, int64_t count, int64_t* d_total, int64_t* scratch, hipStream_t s);
int scan_incl_max_i32(const int32_t* in, int32_t* out, int64_t count, int32_t* scratch, hipStream_t s);

// Stable LSD radix sort of 64-bit keys on bits [lo_bit, hi_bit), optional uint32
// payload; `keys_alt`/`vals_alt` are same-sized scratch and `scratch` holds
// sort_scratch_bytes(count) bytes.  With `counts` (DEVICE, one per 4096-key block)
// block b of the input holds only its first counts[b] keys and the output is the
// dense sorted sequence of those keys.  *result_in_alt tells which buffer holds the
// sorted data.  count < 2^31.
constexpr int kSortTileKeys = 4096;
size_t sort_scratch_bytes(int64_t count);
int radix_sort_u64(uint64_t* keys, uint64_t* keys_alt, uint32_t* vals, uint32_t* vals_alt, int64_t count,
                   const int32_t* counts, int lo_bit, int hi_bit, void* scratch, bool* result_in_alt, hipStream_t s);

}  // namespace tcmis
