// Device prefix scan and LSD radix sort used by the tile builder.
//
// Radix sort: 8-bit digits, three kernels per pass (per-block digit histogram,
// exclusive scan of the digit-major histogram, stable scatter).  The scatter ranks
// equal digits inside a wavefront with eight ballots (one per digit bit), and
// across the block's wavefronts and iterations through LDS counters, which keeps
// the pass stable.
#include "common.hpp"

namespace tcmis {

namespace {

constexpr int kScanItems = 8;                       // items per thread in the scan
constexpr int kScanTile = kBlock * kScanItems;      // 2048
constexpr int kSortIters = 16;                      // iterations per sort block
constexpr int kSortTile = kBlock * kSortIters;      // 4096 keys per block
constexpr int kDigits = 256;
constexpr int kWavesPerBlock = kBlock / kWave;      // 4

// inclusive scan of one value per thread across the block; returns the block total
__device__ int64_t block_inclusive_scan(int64_t x, int64_t* lds_wave /*[kWavesPerBlock]*/, int64_t& total) {
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    for (int off = 1; off < kWave; off <<= 1) {
        int64_t y = __shfl_up(x, off, kWave);
        if (lane >= off) x += y;
    }
    if (lane == kWave - 1) lds_wave[wid] = x;
    __syncthreads();
    int64_t before = 0;
    total = 0;
    for (int w = 0; w < kWavesPerBlock; ++w) {
        int64_t s = lds_wave[w];
        if (w < wid) before += s;
        total += s;
    }
    __syncthreads();
    return x + before;
}

__global__ void __launch_bounds__(kBlock) k_scan_reduce(const int64_t* in, int64_t count, int64_t* sums) {
    __shared__ int64_t lds[kWavesPerBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t s = 0;
    for (int i = 0; i < kScanItems; ++i) {
        int64_t idx = base + i;
        if (idx < count) s += in[idx];
    }
    int64_t total;
    block_inclusive_scan(s, lds, total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kBlock) k_scan_apply(const int64_t* in, int64_t* out, int64_t count,
                                                       const int64_t* block_offsets, int64_t* d_total,
                                                       int64_t grand_total_index) {
    __shared__ int64_t lds[kWavesPerBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t v[kScanItems];
    int64_t s = 0;
    for (int i = 0; i < kScanItems; ++i) {
        int64_t idx = base + i;
        v[i] = idx < count ? in[idx] : 0;
        s += v[i];
    }
    int64_t total;
    int64_t incl = block_inclusive_scan(s, lds, total);
    int64_t run = incl - s + (block_offsets ? block_offsets[blockIdx.x] : 0);
    for (int i = 0; i < kScanItems; ++i) {
        int64_t idx = base + i;
        if (idx < count) out[idx] = run;
        run += v[i];
    }
    if (d_total && (int64_t)blockIdx.x == grand_total_index && threadIdx.x == kBlock - 1) *d_total = run;
}

// ---- radix sort kernels ----
__global__ void __launch_bounds__(kBlock) k_radix_hist(const uint64_t* keys, int64_t count, int shift,
                                                       int64_t nblocks, int64_t* hist) {
    __shared__ int cnt[kDigits];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int it = 0; it < kSortIters; ++it) {
        int64_t idx = base + (int64_t)it * kBlock + threadIdx.x;
        if (idx < count) atomicAdd(&cnt[(keys[idx] >> shift) & 0xff], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

template <bool kVals>
__global__ void __launch_bounds__(kBlock) k_radix_scatter(const uint64_t* keys, uint64_t* keys_out,
                                                          const uint32_t* vals, uint32_t* vals_out,
                                                          int64_t count, int shift, int64_t nblocks,
                                                          const int64_t* offsets) {
    __shared__ int64_t base_of[kDigits];
    __shared__ int wave_cnt[kWavesPerBlock][kDigits];
    const int t = threadIdx.x, lane = lane_id(), wid = t / kWave;
    base_of[t] = offsets[(int64_t)t * nblocks + blockIdx.x];
    for (int w = 0; w < kWavesPerBlock; ++w) wave_cnt[w][t] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int it = 0; it < kSortIters; ++it) {
        const int64_t idx = base + (int64_t)it * kBlock + t;
        const bool valid = idx < count;
        uint64_t k = valid ? keys[idx] : 0;
        uint32_t val = (kVals && valid) ? vals[idx] : 0;
        const int d = (int)((k >> shift) & 0xff);
        uint64_t match = ballot(valid);
        #pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1;
            const uint64_t bb = ballot(bit);
            match &= bit ? bb : ~bb;
        }
        const int rank = __popcll(match & lanes_below());
        const int leader = match ? __ffsll((unsigned long long)match) - 1 : 0;
        if (valid && lane == leader) wave_cnt[wid][d] = __popcll(match);
        __syncthreads();
        if (valid) {
            int64_t dst = base_of[d] + rank;
            for (int w = 0; w < wid; ++w) dst += wave_cnt[w][d];
            keys_out[dst] = k;
            if (kVals) vals_out[dst] = val;
        }
        __syncthreads();
        int add = 0;
        for (int w = 0; w < kWavesPerBlock; ++w) { add += wave_cnt[w][t]; wave_cnt[w][t] = 0; }
        base_of[t] += add;
        __syncthreads();
    }
}

}  // namespace

int scan_exclusive_i64(const int64_t* in, int64_t* out, int64_t count, int64_t* d_total,
                       hipStream_t stream) {
    if (count <= 0) {
        if (d_total) TC_HIP(hipMemsetAsync(d_total, 0, sizeof(int64_t), stream));
        return MIS_OK;
    }
    const int64_t nb = ceil_div(count, kScanTile);
    if (nb == 1) {
        hipLaunchKernelGGL(k_scan_apply, dim3(1), dim3(kBlock), 0, stream, in, out, count,
                           (const int64_t*)nullptr, d_total, (int64_t)0);
        TC_HIP(hipGetLastError());
        return MIS_OK;
    }
    int64_t* sums = nullptr;
    TC_CHECK(dev_alloc((void**)&sums, (size_t)nb * sizeof(int64_t)));
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kBlock), 0, stream, in, count, sums);
    int rc = hipGetLastError() == hipSuccess ? MIS_OK : MIS_EHIP;
    if (rc == MIS_OK) rc = scan_exclusive_i64(sums, sums, nb, nullptr, stream);
    if (rc == MIS_OK) {
        hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kBlock), 0, stream, in, out, count,
                           (const int64_t*)sums, d_total, nb - 1);
        if (hipGetLastError() != hipSuccess) rc = MIS_EHIP;
    }
    (void)hipStreamSynchronize(stream);
    (void)hipFree(sums);
    if (rc != MIS_OK) set_error("scan_exclusive_i64 launch failed");
    return rc;
}

int radix_sort_u64(uint64_t* keys, uint64_t* keys_alt, uint32_t* vals, uint32_t* vals_alt,
                   int64_t count, int lo_bit, int hi_bit, bool* result_in_alt, hipStream_t stream) {
    *result_in_alt = false;
    if (count <= 1 || hi_bit <= lo_bit) return MIS_OK;
    const int64_t nb = ceil_div(count, kSortTile);
    int64_t* hist = nullptr;
    TC_CHECK(dev_alloc((void**)&hist, (size_t)nb * kDigits * sizeof(int64_t)));
    uint64_t *src = keys, *dst = keys_alt;
    uint32_t *vsrc = vals, *vdst = vals_alt;
    int rc = MIS_OK;
    for (int shift = lo_bit; shift < hi_bit && rc == MIS_OK; shift += 8) {
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nb), dim3(kBlock), 0, stream, src, count, shift, nb, hist);
        if (hipGetLastError() != hipSuccess) { rc = MIS_EHIP; break; }
        rc = scan_exclusive_i64(hist, hist, nb * kDigits, nullptr, stream);
        if (rc != MIS_OK) break;
        if (vals) {
            hipLaunchKernelGGL(k_radix_scatter<true>, dim3((unsigned)nb), dim3(kBlock), 0, stream, src, dst,
                               vsrc, vdst, count, shift, nb, hist);
        } else {
            hipLaunchKernelGGL(k_radix_scatter<false>, dim3((unsigned)nb), dim3(kBlock), 0, stream, src, dst,
                               (const uint32_t*)nullptr, (uint32_t*)nullptr, count, shift, nb, hist);
        }
        if (hipGetLastError() != hipSuccess) { rc = MIS_EHIP; break; }
        uint64_t* t = src; src = dst; dst = t;
        uint32_t* tv = vsrc; vsrc = vdst; vdst = tv;
        *result_in_alt = !*result_in_alt;
    }
    (void)hipStreamSynchronize(stream);
    (void)hipFree(hist);
    if (rc != MIS_OK) set_error("radix_sort_u64 failed");
    return rc;
}

}  // namespace tcmis
