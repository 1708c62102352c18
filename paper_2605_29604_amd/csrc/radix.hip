// Device prefix scans and the LSD radix sort used by the build stage.
//
// No allocation and no host synchronisation: callers pass scratch sized by
// scan_scratch_elems / sort_scratch_bytes, and results stay on the device.
//
// Scans: reduce-then-scan over tiles of 2048 items (256 threads x 8), recursive on
// the tile totals.  Radix sort: 8- to 10-bit digits, five kernels per pass
// (per-block digit histogram stored block-major, chunk sums, a per-digit scan of
// the chunk sums, positions in place of the counts, stable scatter); within a block every wavefront ranks a
// contiguous run of keys with one ballot per digit bit and counters of its own,
// which keeps every pass stable with two block-wide barriers.
#include <algorithm>
#include <utility>

#include "common.hpp"

namespace tcmis {

namespace {

constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;   // 2048
constexpr int kSortIters = 16;
constexpr int kSortTile = kBlock * kSortIters;   // 4096 keys per block
constexpr int kWavesPerBlock = kBlock / kWave;

struct OpAdd {
    template <typename T> __device__ static T apply(T a, T b) { return a + b; }
    template <typename T> __device__ static T identity() { return T(0); }
};
struct OpMax {
    template <typename T> __device__ static T apply(T a, T b) { return a > b ? a : b; }
    template <typename T> __device__ static T identity() { return T(-1); }
};

// inclusive scan of one value per thread over the block; *total = block aggregate
template <typename T, typename Op>
__device__ T block_scan(T x, T* lds_wave, T* total) {
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    for (int off = 1; off < kWave; off <<= 1) {
        T y = __shfl_up(x, off, kWave);
        if (lane >= off) x = Op::apply(x, y);
    }
    if (lane == kWave - 1) lds_wave[wid] = x;
    __syncthreads();
    T before = Op::template identity<T>(), all = Op::template identity<T>();
    for (int w = 0; w < kWavesPerBlock; ++w) {
        T s = lds_wave[w];
        if (w < wid) before = Op::apply(before, s);
        all = Op::apply(all, s);
    }
    __syncthreads();
    *total = all;
    return Op::apply(before, x);
}

template <typename T, typename Op>
__global__ void __launch_bounds__(kBlock) k_scan_reduce(const T* in, int64_t count, T* sums) {
    __shared__ T lds[kWavesPerBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    T s = Op::template identity<T>();
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t idx = base + i;
        if (idx < count) s = Op::apply(s, in[idx]);
    }
    T total;
    block_scan<T, Op>(s, lds, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// exclusive (kIncl = false) or inclusive scan of each tile, seeded with the
// exclusive scan of the tile totals (tile_prefix), or, with tile_sums instead, with
// the total of the tiles before this one, which the block adds up itself (at most
// kScanTile tiles)
template <typename T, typename Op, bool kIncl>
__global__ void __launch_bounds__(kBlock) k_scan_apply(const T* in, T* out, int64_t count, const T* tile_prefix,
                                                       T* d_total, const T* tile_sums) {
    __shared__ T lds[kWavesPerBlock];
    __shared__ T seed;
    if (tile_sums) {
        T part = Op::template identity<T>();
        for (int64_t i = threadIdx.x; i < blockIdx.x; i += kBlock) part = Op::apply(part, tile_sums[i]);
        T all;
        block_scan<T, Op>(part, lds, &all);
        if (threadIdx.x == 0) seed = all;
        __syncthreads();
    }
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    T v[kScanItems];
    T s = Op::template identity<T>();
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t idx = base + i;
        v[i] = idx < count ? in[idx] : Op::template identity<T>();
        s = Op::apply(s, v[i]);
    }
    T total;
    const T incl = block_scan<T, Op>(s, lds, &total);
    // exclusive prefix of this thread's first item = inclusive result of the previous thread
    __shared__ T lds_incl[kBlock];
    lds_incl[threadIdx.x] = incl;
    __syncthreads();
    T run = threadIdx.x == 0 ? Op::template identity<T>() : lds_incl[threadIdx.x - 1];
    if (tile_prefix) run = Op::apply(tile_prefix[blockIdx.x], run);
    if (tile_sums) run = Op::apply(seed, run);
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t idx = base + i;
        if (kIncl) {
            run = Op::apply(run, v[i]);
            if (idx < count) out[idx] = run;
        } else {
            if (idx < count) out[idx] = run;
            run = Op::apply(run, v[i]);
        }
    }
    if (d_total && blockIdx.x == gridDim.x - 1 && threadIdx.x == kBlock - 1) *d_total = run;
}

template <typename T, typename Op, bool kIncl>
int scan_impl(const T* in, T* out, int64_t count, T* d_total, T* scratch, hipStream_t s) {
    if (count <= 0) return MIS_OK;
    const int64_t nb = ceil_div(count, kScanTile);
    if (nb == 1) {
        hipLaunchKernelGGL((k_scan_apply<T, Op, kIncl>), dim3(1), dim3(kBlock), 0, s, in, out, count, (const T*)nullptr,
                           d_total, (const T*)nullptr);
        TC_HIP(hipGetLastError());
        return MIS_OK;
    }
    T* sums = scratch;
    T* rest = scratch + nb;
    hipLaunchKernelGGL((k_scan_reduce<T, Op>), dim3((unsigned)nb), dim3(kBlock), 0, s, in, count, sums);
    TC_HIP(hipGetLastError());
    if (nb <= kScanTile) {   // two kernels: each tile adds up the totals before it
        hipLaunchKernelGGL((k_scan_apply<T, Op, kIncl>), dim3((unsigned)nb), dim3(kBlock), 0, s, in, out, count,
                           (const T*)nullptr, d_total, (const T*)sums);
        TC_HIP(hipGetLastError());
        return MIS_OK;
    }
    TC_CHECK((scan_impl<T, Op, false>(sums, sums, nb, (T*)nullptr, rest, s)));
    hipLaunchKernelGGL((k_scan_apply<T, Op, kIncl>), dim3((unsigned)nb), dim3(kBlock), 0, s, in, out, count,
                       (const T*)sums, d_total, (const T*)nullptr);
    TC_HIP(hipGetLastError());
    return MIS_OK;
}

// ---- radix sort kernels ----
// Keys are processed in blocks of kSortTile; block b holds keys
// [b*kSortTile, b*kSortTile + len_b) with len_b = counts[b] when per-block counts are
// given (compacted producer output), else kSortTile (the last block: the rest).
// (with `dense_total`, a pass after a compacted first pass: the keys are dense and
// their number is on the device)
__device__ inline int block_len(const int32_t* counts, const int32_t* dense_total, int64_t count, int64_t b) {
    if (counts) return counts[b];
    const int64_t c = dense_total ? (int64_t)*dense_total : count;
    const int64_t rest = c - b * kSortTile;
    return (int)(rest < 0 ? 0 : (rest < kSortTile ? rest : kSortTile));
}

// Lanes of the wavefront whose valid key has digit d (d < 2^DB), including this
// lane; empty for an invalid key.  DB ballots, no LDS.
template <int DB>
__device__ inline uint64_t digit_peers(bool valid, int d) {
    const uint64_t v = ballot(valid);
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    #pragma unroll
    for (int b = 0; b < DB; ++b) {
        // the lanes whose bit b equals this lane's: m & ~(ballot ^ s), s = this lane's
        // bit spread over the word, as one three-input logic op per half.  m is the
        // middle operand and the function is symmetric in the outer two, so the truth
        // table (m = 1 and the outer two equal: 0x84) does not depend on which outer
        // operand is the high index bit.
        const uint32_t s = (uint32_t)(((int32_t)((uint32_t)d << (31 - b))) >> 31);
        const uint64_t bb = ballot(s != 0);
        lo = __builtin_amdgcn_bitop3_b32((uint32_t)bb, lo, s, 0x84);
        hi = __builtin_amdgcn_bitop3_b32((uint32_t)(bb >> 32), hi, s, 0x84);
    }
    return valid ? ((uint64_t)hi << 32 | lo) : 0ull;
}

// Keys of a block are split into one contiguous run of kSortTile / 4 keys per
// wavefront (block order = wavefront, iteration, lane), so every wavefront counts
// and ranks its keys with counters of its own and no block-wide barrier.
constexpr int kRunPerWave = kSortTile / kWavesPerBlock;   // 1024
constexpr int kRunIters = kRunPerWave / kWave;            // 16

// Digit histogram of one block: per-wavefront LDS counters.
template <int DB>
__global__ void __launch_bounds__(kBlock) k_radix_hist(const uint64_t* keys, int64_t count, const int32_t* counts,
                                                       const int32_t* dense_total, int shift, int64_t nblocks,
                                                       int32_t* hist) {
    constexpr int D = 1 << DB;
    __shared__ int cnt[kWavesPerBlock][D];
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    for (int i = threadIdx.x; i < kWavesPerBlock * D; i += kBlock) (&cnt[0][0])[i] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    const int len = block_len(counts, dense_total, count, blockIdx.x);
    // every key of the lane is loaded before the first counter update
    uint64_t kk[kRunIters];
    #pragma unroll
    for (int it = 0; it < kRunIters; ++it) {
        const int i = wid * kRunPerWave + it * kWave + lane;
        kk[it] = i < len ? keys[base + i] : 0;
    }
    #pragma unroll
    for (int it = 0; it < kRunIters; ++it)
        if (wid * kRunPerWave + it * kWave + lane < len) atomicAdd(&cnt[wid][(kk[it] >> shift) & (D - 1)], 1);
    __syncthreads();
    for (int d = threadIdx.x; d < D; d += kBlock) {
        int tot = 0;
        for (int w = 0; w < kWavesPerBlock; ++w) tot += cnt[w][d];
        hist[(int64_t)blockIdx.x * D + d] = tot;   // row per block: one coalesced store
    }
}

// The histogram is block-major (row b = block b's digit counts), so every block
// writes and reads its row with coalesced accesses.  Block b's first position for
// digit d is (keys of smaller digits) + (keys of digit d in earlier blocks); the
// second term is split into chunks of `chunk` rows: sums per chunk, a per-digit
// scan of those, then each chunk's rows are turned into positions in place.  The
// chunk grows with the number of blocks (1 .. 16 rows), so that the per-digit scan
// has a few hundred chunks to scan and the chunk kernels enough workgroups.
inline int64_t hist_chunk(int64_t nblocks) { return std::min<int64_t>(16, std::max<int64_t>(1, nblocks / 256)); }

// csum[c * D + d] = digit d's keys in blocks c * chunk .. + chunk - 1
template <int DB>
__global__ void __launch_bounds__(kBlock) k_hist_chunk_sum(const int32_t* hist, int64_t nblocks, int64_t chunk,
                                                           int32_t* csum) {
    constexpr int D = 1 << DB;
    const int64_t c = blockIdx.x, b0 = c * chunk, b1 = min(nblocks, b0 + chunk);
    for (int d = threadIdx.x; d < D; d += kBlock) {
        int sum = 0;
        for (int64_t b = b0; b < b1; ++b) sum += hist[b * D + d];
        csum[c * D + d] = sum;
    }
}

// One workgroup per digit d: column d of csum becomes its exclusive scan over the
// chunks, and dtot[d] the digit's total.
template <int DB>
__global__ void __launch_bounds__(kBlock) k_hist_col_scan(int32_t* csum, int64_t nchunks, int32_t* dtot) {
    constexpr int D = 1 << DB;
    __shared__ int32_t lw[kWavesPerBlock];
    const int d = blockIdx.x;
    const int64_t per = (nchunks + kBlock - 1) / kBlock;
    const int64_t c0 = threadIdx.x * per, c1 = min(nchunks, c0 + per);
    int sum = 0;
    for (int64_t c = c0; c < c1; ++c) sum += csum[c * D + d];
    int total;
    const int incl = block_scan<int, OpAdd>(sum, lw, &total);
    int run = incl - sum;
    for (int64_t c = c0; c < c1; ++c) {
        const int x = csum[c * D + d];
        csum[c * D + d] = run;
        run += x;
    }
    if (threadIdx.x == 0) dtot[d] = total;
}

// One workgroup per chunk: its rows of the histogram become the blocks' first
// positions per digit (in place); workgroup 0 also writes the number of keys.
template <int DB>
__global__ void __launch_bounds__(kBlock) k_hist_apply(int32_t* hist, const int32_t* csum, const int32_t* dtot,
                                                       int64_t nblocks, int64_t chunk, int32_t* dense_out) {
    constexpr int D = 1 << DB;
    constexpr int kPerT = D / kBlock > 0 ? D / kBlock : 1;
    __shared__ int32_t lw[kWavesPerBlock];
    const int t = threadIdx.x;
    const int64_t c = blockIdx.x, b0 = c * chunk, b1 = min(nblocks, b0 + chunk);
    // exclusive scan of the digit totals (digits t * kPerT .. are this thread's)
    int x[kPerT], loc = 0;
    #pragma unroll
    for (int j = 0; j < kPerT; ++j) {
        const int d = t * kPerT + j;
        x[j] = d < D ? dtot[d] : 0;
        loc += x[j];
    }
    int all;
    int run = block_scan<int, OpAdd>(loc, lw, &all) - loc;
    if (dense_out && c == 0 && t == 0) *dense_out = all;
    #pragma unroll
    for (int j = 0; j < kPerT; ++j) {
        const int d = t * kPerT + j;
        if (d < D) {
            int pos = run + csum[c * D + d];
            for (int64_t b = b0; b < b1; ++b) {
                const int n = hist[b * D + d];
                hist[b * D + d] = pos;
                pos += n;
            }
        }
        run += x[j];
    }
}

// Stable scatter of one block.  Each wavefront ranks its run's keys among its own
// earlier keys of the same digit; one pass over the digits then turns the
// per-wavefront counts into first positions (block order: digit, wavefront), the
// keys are placed in LDS in (digit, original order) and written out so that
// consecutive threads write consecutive positions of one digit's run -- coalesced
// stores instead of one scattered 8-byte store per key.
template <int DB, bool kVals>
__global__ void __launch_bounds__(kBlock) k_radix_scatter(const uint64_t* keys, uint64_t* keys_out,
                                                          const uint32_t* vals, uint32_t* vals_out, int64_t count,
                                                          const int32_t* counts, const int32_t* dense_total, int shift,
                                                          int64_t nblocks, const int32_t* offsets) {
    constexpr int D = 1 << DB;
    constexpr int kPerT = D / kBlock > 0 ? D / kBlock : 1;   // digits per thread in the digit pass
    __shared__ uint64_t skey[kSortTile];
    __shared__ uint32_t sval[kVals ? kSortTile : 1];
    __shared__ int32_t wpos[kWavesPerBlock][D];   // per-wavefront counts, then first positions
    __shared__ int32_t gdelta[D];                 // global minus local position of each digit's keys
    __shared__ int32_t wsum[kWavesPerBlock];
    const int t = threadIdx.x, lane = lane_id(), wid = t / kWave;
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    const int len = block_len(counts, dense_total, count, blockIdx.x);
    int32_t* wc = wpos[wid];
    // this block's global first position of each of the thread's digits (its row)
    int gb[kPerT];
    #pragma unroll
    for (int j = 0; j < kPerT; ++j) {
        const int d = t * kPerT + j;
        gb[j] = d < D ? offsets[(int64_t)blockIdx.x * D + d] : 0;
    }
    for (int d = lane; d < D; d += kWave) wc[d] = 0;
    // every key (and value) of the lane is loaded before the ranking pass
    uint64_t kk[kRunIters];
    uint32_t vv[kRunIters];
    #pragma unroll
    for (int it = 0; it < kRunIters; ++it) {
        const int i = wid * kRunPerWave + it * kWave + lane;
        kk[it] = i < len ? keys[base + i] : 0;
        vv[it] = (kVals && i < len) ? vals[base + i] : 0;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // rank of each key among the wavefront's earlier keys of its digit
    int rk[kRunIters];
    #pragma unroll
    for (int it = 0; it < kRunIters; ++it) {
        const int i = wid * kRunPerWave + it * kWave + lane;
        const int d = (int)((kk[it] >> shift) & (D - 1));
        const uint64_t m = digit_peers<DB>(i < len, d);
        const int below = __popcll(m & lanes_below());
        const int prior = m ? wc[d] : 0;
        rk[it] = prior + below;
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (m && below == 0) wc[d] = prior + __popcll(m);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // digit pass: block totals, their exclusive scan, each wavefront's first position
    int tot[kPerT];
    int local = 0;
    #pragma unroll
    for (int j = 0; j < kPerT; ++j) {
        const int d = t * kPerT + j;
        int sum = 0;
        if (d < D)
            for (int w = 0; w < kWavesPerBlock; ++w) sum += wpos[w][d];
        tot[j] = sum;
        local += sum;
    }
    int incl = local;
    for (int off = 1; off < kWave; off <<= 1) {
        const int o = __shfl_up(incl, off, kWave);
        if (lane >= off) incl += o;
    }
    if (lane == kWave - 1) wsum[wid] = incl;
    __syncthreads();
    int before = incl - local;
    for (int w = 0; w < wid; ++w) before += wsum[w];
    #pragma unroll
    for (int j = 0; j < kPerT; ++j) {
        const int d = t * kPerT + j;
        if (d < D) {
            gdelta[d] = gb[j] - before;
            int run = before;
            for (int w = 0; w < kWavesPerBlock; ++w) {
                const int c = wpos[w][d];
                wpos[w][d] = run;
                run += c;
            }
        }
        before += tot[j];
    }
    __syncthreads();
    #pragma unroll
    for (int it = 0; it < kRunIters; ++it) {
        const int i = wid * kRunPerWave + it * kWave + lane;
        if (i < len) {
            const int pos = wc[(int)((kk[it] >> shift) & (D - 1))] + rk[it];
            skey[pos] = kk[it];
            if (kVals) sval[pos] = vv[it];
        }
    }
    __syncthreads();
    // coalesced write-out in (digit, original order)
    for (int j = t; j < len; j += kBlock) {
        const uint64_t k = skey[j];
        const int64_t dst = (int64_t)gdelta[(int)((k >> shift) & (D - 1))] + j;
        keys_out[dst] = k;
        if (kVals) vals_out[dst] = sval[j];
    }
}

template <int DB>
int sort_passes(uint64_t** src, uint64_t** dst, uint32_t** vsrc, uint32_t** vdst, int64_t count,
                const int32_t* counts, int lo_bit, int hi_bit, int32_t* hist, int32_t* csum, int32_t* dtot,
                int32_t* total, bool* alt, hipStream_t s) {
    const int64_t nb = ceil_div(count, kSortTile), chunk = hist_chunk(nb), nchunks = ceil_div(nb, chunk);
    const int32_t* dense = nullptr;
    for (int shift = lo_bit; shift < hi_bit; shift += DB) {
        hipLaunchKernelGGL((k_radix_hist<DB>), dim3((unsigned)nb), dim3(kBlock), 0, s, *src, count, counts, dense, shift,
                           nb, hist);
        TC_HIP(hipGetLastError());
        hipLaunchKernelGGL((k_hist_chunk_sum<DB>), dim3((unsigned)nchunks), dim3(kBlock), 0, s, (const int32_t*)hist,
                           nb, chunk, csum);
        TC_HIP(hipGetLastError());
        hipLaunchKernelGGL((k_hist_col_scan<DB>), dim3(1u << DB), dim3(kBlock), 0, s, csum, nchunks, dtot);
        TC_HIP(hipGetLastError());
        int32_t* dense_out = counts ? total : nullptr;   // the first pass counts the kept keys
        hipLaunchKernelGGL((k_hist_apply<DB>), dim3((unsigned)nchunks), dim3(kBlock), 0, s, hist, (const int32_t*)csum,
                           (const int32_t*)dtot, nb, chunk, dense_out);
        TC_HIP(hipGetLastError());
        if (*vsrc)
            hipLaunchKernelGGL((k_radix_scatter<DB, true>), dim3((unsigned)nb), dim3(kBlock), 0, s, *src, *dst, *vsrc,
                               *vdst, count, counts, dense, shift, nb, (const int32_t*)hist);
        else
            hipLaunchKernelGGL((k_radix_scatter<DB, false>), dim3((unsigned)nb), dim3(kBlock), 0, s, *src, *dst,
                               (const uint32_t*)nullptr, (uint32_t*)nullptr, count, counts, dense, shift, nb,
                               (const int32_t*)hist);
        TC_HIP(hipGetLastError());
        std::swap(*src, *dst);
        std::swap(*vsrc, *vdst);
        *alt = !*alt;
        if (counts) dense = total;   // after a compacted first pass the keys are dense
        counts = nullptr;
    }
    return MIS_OK;
}

}  // namespace

int64_t scan_scratch_elems(int64_t count) {
    int64_t total = 0;
    while (count > kScanTile) {
        count = ceil_div(count, kScanTile);
        total += count;
    }
    return total + 1;
}

int scan_excl_i32(const int32_t* in, int32_t* out, int64_t count, int32_t* d_total, int32_t* scratch, hipStream_t s) {
    return scan_impl<int32_t, OpAdd, false>(in, out, count, d_total, scratch, s);
}
int scan_excl_i64(const int64_t* in, int64_t* out, int64_t count, int64_t* d_total, int64_t* scratch, hipStream_t s) {
    return scan_impl<int64_t, OpAdd, false>(in, out, count, d_total, scratch, s);
}
int scan_incl_max_i32(const int32_t* in, int32_t* out, int64_t count, int32_t* scratch, hipStream_t s) {
    return scan_impl<int32_t, OpMax, true>(in, out, count, (int32_t*)nullptr, scratch, s);
}

// scratch: block-major histogram (nb rows of up to 1024 digits), chunk sums, digit
// totals, the kept-key count
size_t sort_scratch_bytes(int64_t count) {
    const int64_t nb = ceil_div(count > 0 ? count : 1, kSortTile);
    const int64_t h = nb * 1024, c = ceil_div(nb, hist_chunk(nb)) * 1024;
    return (size_t)(h + c + 1024 + 64) * sizeof(int32_t);
}

// 8-bit digits, or 9/10-bit digits when that saves a pass
static int digit_bits(int lo_bit, int hi_bit) {
    const int bits = hi_bit - lo_bit;
    if (bits > 8 && ceil_div(bits, 10) < ceil_div(bits, 8)) return ceil_div(bits, 9) == ceil_div(bits, 10) ? 9 : 10;
    return 8;
}

int radix_sort_u64(uint64_t* keys, uint64_t* keys_alt, uint32_t* vals, uint32_t* vals_alt, int64_t count,
                   const int32_t* counts, int lo_bit, int hi_bit, void* scratch, bool* result_in_alt, hipStream_t s) {
    *result_in_alt = false;
    if (count <= 1 && !counts) return MIS_OK;
    if (hi_bit <= lo_bit) return MIS_OK;
    if (count >= (1ll << 31)) {
        set_error("radix sort is limited to 2^31 keys");
        return MIS_EINVAL;
    }
    const int64_t nb = ceil_div(count, kSortTile);
    int32_t* hist = (int32_t*)scratch;
    int32_t* csum = hist + nb * 1024;
    int32_t* dtot = csum + ceil_div(nb, hist_chunk(nb)) * 1024;
    int32_t* total = dtot + 1024;
    uint64_t *src = keys, *dst = keys_alt;
    uint32_t *vsrc = vals, *vdst = vals_alt;
    const int db = digit_bits(lo_bit, hi_bit);
    if (db == 9)
        return sort_passes<9>(&src, &dst, &vsrc, &vdst, count, counts, lo_bit, hi_bit, hist, csum, dtot,
                              total, result_in_alt, s);
    if (db == 10)
        return sort_passes<10>(&src, &dst, &vsrc, &vdst, count, counts, lo_bit, hi_bit, hist, csum, dtot,
                               total, result_in_alt, s);
    return sort_passes<8>(&src, &dst, &vsrc, &vdst, count, counts, lo_bit, hi_bit, hist, csum, dtot,
                          total, result_in_alt, s);
}

}  // namespace tcmis
