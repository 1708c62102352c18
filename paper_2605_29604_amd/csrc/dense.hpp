// Dense 16-row blocks of the hybrid path: the candidate test, shared by the key
// kernel (which takes a sample of blocks) and the dense-block build.
#pragma once
#include "graph.hpp"

namespace tcmis {

constexpr int kDenseCap = 1024;     // most oriented entries a block may hold to be dense
constexpr int kDenseTiles = 64;     // most tiles of a dense block (one per lane)

// A block is examined exactly only if its whole adjacency looks concentrated: a
// wave ORs a 256-bit signature of its entries' column blocks, and linear counting
// (-256 ln(1 - bits / 256)) estimates its distinct column blocks, i.e. its nonzero
// tiles.  Its higher-priority half must average dense_min entries per tile, so a
// block is a candidate when its entries reach dense_min times that estimate (a factor
// of two of slack) and it has at most 2 * kDenseCap entries.  A sample of blocks
// decides first whether the graph has such blocks at all (at least 1% of the
// sample); if not, the build only writes the empty slot map.  These tests only choose
// the representation; the results never depend on them.
constexpr int kGateSamples = 1024;

// the sample: every stride-th of the nI row-blocks, at most kGateSamples of them
inline int64_t dense_stride(int64_t nI) { return nI / kGateSamples > 1 ? nI / kGateSamples : 1; }
inline int dense_samples(int64_t nI) {
    const int64_t st = dense_stride(nI);
    const int64_t k = (nI + st - 1) / st;
    return (int)(k < kGateSamples ? k : kGateSamples);
}

__device__ inline int sig_index(int64_t J) { return (int)(((uint64_t)J * 0x9E3779B97F4A7C15ull) >> 56); }

// 1 if block I (entries [b0, b1)) is a dense candidate; every lane of the wave calls it
__device__ inline int block_candidate(const int32_t* ci, int64_t b0, int64_t b1, int dense_min) {
    const int64_t tot = b1 - b0;
    if (tot == 0 || tot > 2 * kDenseCap) return 0;
    uint64_t s[4] = {0, 0, 0, 0};
    for (int64_t e = b0 + lane_id(); e < b1; e += 4 * kWave) {
        int32_t u[4];
        #pragma unroll
        for (int j = 0; j < 4; ++j) u[j] = e + j * kWave < b1 ? ci[e + j * kWave] : -1;
        #pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (u[j] < 0) continue;
            const int k = sig_index(u[j] >> 4);
            const uint64_t bit = 1ull << (k & 63);
            if (k < 64) s[0] |= bit;
            else if (k < 128) s[1] |= bit;
            else if (k < 192) s[2] |= bit;
            else s[3] |= bit;
        }
    }
    int bits = 0;
    #pragma unroll
    for (int w = 0; w < 4; ++w) {
        for (int off = kWave / 2; off > 0; off >>= 1) s[w] |= __shfl_xor(s[w], off, kWave);
        bits += __popcll(s[w]);
    }
    if (bits >= 256) return 0;
    const float est = -256.0f * logf(1.0f - (float)bits / 256.0f);
    return est <= 2.0f * kDenseTiles && (float)tot >= (float)dense_min * est ? 1 : 0;
}

// The sample: every stride-th block; a wave takes sample i (its candidate flag into
// samp[i]) for i = wave, wave + waves, ... < samples.  Every lane of the wave calls it.
__device__ inline void dense_sample(const int64_t* rp, const int32_t* ci, int64_t n, int64_t stride, int samples,
                                    int dense_min, int32_t* samp, int64_t wave, int64_t waves) {
    for (int64_t i = wave; i < samples; i += waves) {
        const int64_t I = i * stride;
        const int c = block_candidate(ci, rp[16 * I], rp[min<int64_t>(16 * I + 16, n)], dense_min);
        if (lane_id() == 0) samp[i] = c;
    }
}

}  // namespace tcmis
