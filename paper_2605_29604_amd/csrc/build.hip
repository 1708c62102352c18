// Build stage: validation, priority keys, vertex reordering and the nonzero
// T x T bit tiles (Section 3.2: the adjacency matrix is kept as nonzero tiles in a
// compressed block format), plus the degree-binned vertex lists of the CSR path.
#include <algorithm>
#include <vector>

#include "graph.hpp"

namespace tcmis {

namespace {

enum : uint32_t { kErrRange = 1, kErrLoop = 2, kErrDup = 4, kErrAsym = 8, kErrTie = 16 };

// ---- SplitMix64 (Steele, Lea, Flood 2014): output i of the stream seeded with s
__device__ inline uint64_t splitmix_at(uint64_t s, uint64_t i) {
    uint64_t z = s + i * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// row of entry e: the largest v with row_ptr[v] <= e (row_ptr monotone, e < nnz)
__device__ inline int64_t row_of(const int64_t* rp, int64_t n, int64_t e) {
    int64_t lo = 0, hi = n;
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) >> 1;
        if (rp[mid] <= e) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ void k_validate_rows(const int64_t* rp, int64_t n, int64_t nnz, uint32_t* err) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        int64_t a = rp[v], b = rp[v + 1];
        if (a < 0 || b < a || b > nnz) atomicOr(err, kErrRange);
    }
}

__global__ void k_validate_edges(const int64_t* rp, const int32_t* ci, int64_t n, int64_t nnz,
                                 const uint64_t* key, uint32_t* err) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = row_of(rp, n, e);
        const int64_t u = ci[e];
        if (u < 0 || u >= n) { atomicOr(err, kErrRange); continue; }
        if (u == v) { atomicOr(err, kErrLoop); continue; }
        if (e > rp[v] && (int64_t)ci[e - 1] >= u) atomicOr(err, kErrDup);
        int64_t lo = rp[u], hi = rp[u + 1];
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if ((int64_t)ci[mid] < v) lo = mid + 1; else hi = mid;
        }
        if (lo >= rp[u + 1] || (int64_t)ci[lo] != v) atomicOr(err, kErrAsym);
        if (key && key[u] == key[v]) atomicOr(err, kErrTie);
    }
}

// Default priority key (Eq. 1, discretised): q(deg) << 56 | hash << 24 | v with
// q(d) = floor(255 / (1 + d)) (lower degree wins) and hash = top 32 bits of output
// v+1 of the SplitMix64 stream seeded with `seed` (the random perturbation).
__global__ void k_keys(const int64_t* rp, int64_t n, uint64_t seed, uint64_t* key) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t deg = rp[v + 1] - rp[v];
        const uint64_t q = (uint64_t)(255 / (1 + deg));
        const uint64_t h = splitmix_at(seed, (uint64_t)v + 1) >> 32;
        key[v] = (q << 56) | (h << 24) | (uint64_t)v;
    }
}

__global__ void k_iota_i32(int32_t* out, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (int32_t)i;
}

// sort keys for the degree and priority orders
__global__ void k_order_keys(const int64_t* rp, const uint64_t* key, int64_t n, int mode,
                             uint64_t* sk, uint32_t* payload) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        if (mode == MIS_REORDER_DEGREE) {
            int64_t deg = rp[v + 1] - rp[v];
            uint64_t inv = 0xFFFFFFFFull - (uint64_t)(deg > 0xFFFFFFFFll ? 0xFFFFFFFFll : deg);
            sk[v] = (inv << 32) | (uint64_t)v;       // decreasing degree, then id
        } else {
            sk[v] = ~key[v];                          // decreasing priority
        }
        payload[v] = (uint32_t)v;
    }
}

__global__ void k_scatter_rank(const uint32_t* order, int64_t n, int32_t* new_id) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x)
        new_id[order[p]] = (int32_t)p;
}

// one entry per kept adjacency entry: (I, J, r, c) packed high to low
__global__ void k_tile_entries(const int64_t* rp, const int32_t* ci, int64_t n, int64_t nnz,
                               const int32_t* new_id, const uint64_t* key, int oriented,
                               int tshift, int bj, uint64_t* ent, unsigned long long* n_valid) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t tmask = (1 << tshift) - 1;
    for (int64_t e0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e0 - threadIdx.x < nnz; e0 += stride) {
        const bool in_range = e0 < nnz;
        bool keep = false;
        uint64_t out = ~0ull;
        if (in_range) {
            const int64_t v = row_of(rp, n, e0);
            const int64_t u = ci[e0];
            keep = !oriented || key[u] > key[v];
            if (keep) {
                const uint64_t p = (uint64_t)new_id[v], q = (uint64_t)new_id[u];
                const uint64_t I = p >> tshift, J = q >> tshift;
                out = (I << (bj + 10)) | (J << 10) | ((p & tmask) << 5) | (q & tmask);
            }
            ent[e0] = out;
        }
        const uint64_t b = ballot(keep);
        if (lane_id() == 0 && b) atomicAdd(n_valid, (unsigned long long)__popcll(b));
    }
}

__global__ void k_tile_flags(const uint64_t* ent, int64_t nvalid, int64_t* flag) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nvalid; e += (int64_t)gridDim.x * blockDim.x)
        flag[e] = (e == 0 || (ent[e] >> 10) != (ent[e - 1] >> 10)) ? 1 : 0;
}

__global__ void k_tile_fill(const uint64_t* ent, int64_t nvalid, const int64_t* flag, const int64_t* excl,
                            int tile, int bj, int32_t* tile_col, uint32_t* bits, int64_t* rb_cnt) {
    const uint64_t jmask = (1ull << bj) - 1;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nvalid; e += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t x = ent[e];
        const int64_t t = excl[e] + flag[e] - 1;
        const uint32_t r = (uint32_t)((x >> 5) & 31), c = (uint32_t)(x & 31);
        if (flag[e]) {
            tile_col[t] = (int32_t)((x >> 10) & jmask);
            atomicAdd((unsigned long long*)&rb_cnt[x >> (bj + 10)], 1ull);
        }
        if (tile == 16) atomicOr(&bits[t * 8 + (r >> 1)], 1u << (((r & 1) << 4) | c));
        else atomicOr(&bits[t * 32 + r], 1u << c);
    }
}

__global__ void k_seg_count(const int64_t* rb_ptr, int64_t nI, int64_t* cnt) {
    for (int64_t I = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; I < nI; I += (int64_t)gridDim.x * blockDim.x) {
        int64_t t = rb_ptr[I + 1] - rb_ptr[I];
        int64_t s = (t + kSegTiles - 1) / kSegTiles;
        cnt[I] = s < 1 ? 1 : s;
    }
}

__global__ void k_seg_fill(const int64_t* rb_ptr, const int64_t* seg0, int64_t nI, int64_t n, int tile,
                           int32_t* seg_rb, int64_t* seg_t0, int64_t* seg_t1, int32_t* rb_seg0,
                           int32_t* rb_nseg, uint32_t* alive0) {
    for (int64_t I = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; I < nI; I += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = rb_ptr[I], b = rb_ptr[I + 1];
        const int64_t s0 = seg0[I];
        const int64_t ns = b - a > 0 ? (b - a + kSegTiles - 1) / kSegTiles : 1;
        rb_seg0[I] = (int32_t)s0;
        rb_nseg[I] = (int32_t)ns;
        for (int64_t k = 0; k < ns; ++k) {
            seg_rb[s0 + k] = (int32_t)I;
            seg_t0[s0 + k] = a + k * kSegTiles;
            seg_t1[s0 + k] = min(b, a + (k + 1) * kSegTiles);
        }
        const int64_t rows = min((int64_t)tile, n - I * tile);
        alive0[I] = rows >= 32 ? 0xFFFFFFFFu : ((1u << rows) - 1u);
    }
}

__global__ void k_permute_keys(const uint64_t* key, const int32_t* new_id, int64_t n, uint64_t* key_p) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        key_p[new_id[v]] = key[v];
}

__global__ void k_deg_flags(const int64_t* rp, int64_t n, int heavy, int64_t* flag) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const bool h = rp[v + 1] - rp[v] > kLightDeg;
        flag[v] = (h == (heavy != 0)) ? 1 : 0;
    }
}

__global__ void k_compact_flagged(const int64_t* flag, const int64_t* pos, int64_t n, int32_t* out) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        if (flag[v]) out[pos[v]] = (int32_t)v;
}

int bits_for(int64_t x) {   // bits to hold values 0..x (so x itself is never all ones)
    int b = 1;
    while ((1ll << b) <= x) ++b;
    return b;
}

int galloc(mis_graph* g, void** p, size_t bytes) {
    if (bytes == 0) bytes = 8;
    TC_CHECK(dev_alloc(p, bytes));
    g->owned.push_back(*p);
    g->bytes += bytes;
    return MIS_OK;
}

struct TmpBuf {   // build temporaries, freed on scope exit
    std::vector<void*> ptrs;
    ~TmpBuf() {
        (void)hipDeviceSynchronize();
        for (void* p : ptrs) (void)hipFree(p);
    }
    int alloc(void** p, size_t bytes) {
        if (bytes == 0) bytes = 8;
        TC_CHECK(dev_alloc(p, bytes));
        ptrs.push_back(*p);
        return MIS_OK;
    }
};

template <typename T>
int read_scalar(const T* d, T* h, hipStream_t s) {
    TC_HIP(hipMemcpyAsync(h, d, sizeof(T), hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    return MIS_OK;
}

}  // namespace

int host_rcm(const int64_t* rp, const int32_t* ci, int64_t n, std::vector<int32_t>& new_id);

// ---------------------------------------------------------------------------

int validate_graph(const mis_csr* csr, const uint64_t* user_keys, hipStream_t s) {
    TmpBuf tmp;
    uint32_t* err = nullptr;
    TC_CHECK(tmp.alloc((void**)&err, 4));
    TC_HIP(hipMemsetAsync(err, 0, 4, s));
    int64_t ends[2] = {0, 0};
    TC_HIP(hipMemcpyAsync(&ends[0], csr->row_ptr, 8, hipMemcpyDeviceToHost, s));
    TC_HIP(hipMemcpyAsync(&ends[1], csr->row_ptr + csr->n, 8, hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    if (ends[0] != 0 || ends[1] != csr->nnz) {
        set_error("row_ptr[0] must be 0 and row_ptr[n] must equal nnz");
        return MIS_ERANGE;
    }
    if (csr->n > 0)
        hipLaunchKernelGGL(k_validate_rows, dim3(stream_grid(csr->n)), dim3(kBlock), 0, s, csr->row_ptr, csr->n,
                           csr->nnz, err);
    uint32_t h = 0;
    TC_CHECK(read_scalar(err, &h, s));
    if (h) { set_error("row_ptr is not monotone within [0, nnz]"); return MIS_ERANGE; }
    if (csr->nnz > 0)
        hipLaunchKernelGGL(k_validate_edges, dim3(stream_grid(csr->nnz)), dim3(kBlock), 0, s, csr->row_ptr,
                           csr->col_idx, csr->n, csr->nnz, user_keys, err);
    TC_HIP(hipGetLastError());
    TC_CHECK(read_scalar(err, &h, s));
    if (h & kErrRange) { set_error("column index out of range"); return MIS_ERANGE; }
    if (h & kErrLoop) { set_error("self-loop"); return MIS_ESELFLOOP; }
    if (h & kErrDup) { set_error("duplicate or unsorted adjacency entries"); return MIS_EDUP; }
    if (h & kErrAsym) { set_error("adjacency is not symmetric"); return MIS_ENOTSYM; }
    if (h & kErrTie) { set_error("two adjacent vertices have equal keys"); return MIS_EINVAL; }
    return MIS_OK;
}

int build_keys(mis_graph* g, const mis_build_opts* o, hipStream_t s) {
    TC_CHECK(galloc(g, (void**)&g->key, (size_t)g->n * 8));
    if (g->n == 0) return MIS_OK;
    if (o->keys) {
        TC_HIP(hipMemcpyAsync(g->key, o->keys, (size_t)g->n * 8, hipMemcpyDeviceToDevice, s));
    } else {
        hipLaunchKernelGGL(k_keys, dim3(stream_grid(g->n)), dim3(kBlock), 0, s, g->row_ptr, g->n, o->seed, g->key);
        TC_HIP(hipGetLastError());
    }
    return MIS_OK;
}

int build_csr_lists(mis_graph* g, hipStream_t s) {
    const int64_t n = g->n;
    TmpBuf tmp;
    int64_t *flag = nullptr, *pos = nullptr, *tot = nullptr;
    TC_CHECK(tmp.alloc((void**)&flag, (size_t)n * 8));
    TC_CHECK(tmp.alloc((void**)&pos, (size_t)n * 8));
    TC_CHECK(tmp.alloc((void**)&tot, 8));
    int32_t* lists[2];
    int64_t counts[2];
    for (int heavy = 0; heavy < 2; ++heavy) {
        if (n > 0)
            hipLaunchKernelGGL(k_deg_flags, dim3(stream_grid(n)), dim3(kBlock), 0, s, g->row_ptr, n, heavy, flag);
        TC_CHECK(scan_exclusive_i64(flag, pos, n, tot, s));
        TC_CHECK(read_scalar(tot, &counts[heavy], s));
        TC_CHECK(galloc(g, (void**)&lists[heavy], (size_t)counts[heavy] * 4));
        if (n > 0)
            hipLaunchKernelGGL(k_compact_flagged, dim3(stream_grid(n)), dim3(kBlock), 0, s, flag, pos, n, lists[heavy]);
        TC_HIP(hipGetLastError());
    }
    g->light = lists[0]; g->n_light = counts[0];
    g->heavy = lists[1]; g->n_heavy = counts[1];
    for (int b = 0; b < 2; ++b) {
        TC_CHECK(galloc(g, (void**)&g->act[b][0], (size_t)g->n_light * 4));
        TC_CHECK(galloc(g, (void**)&g->act[b][1], (size_t)g->n_heavy * 4));
    }
    TC_CHECK(galloc(g, (void**)&g->st, (size_t)n * 4));
    TC_CHECK(galloc(g, (void**)&g->ak, (size_t)n * 8));
    TC_HIP(hipStreamSynchronize(s));
    return MIS_OK;
}

int build_order(mis_graph* g, hipStream_t s) {
    const int64_t n = g->n;
    TC_CHECK(galloc(g, (void**)&g->new_id, (size_t)n * 4));
    if (n == 0) return MIS_OK;
    if (g->reorder == MIS_REORDER_NONE) {
        hipLaunchKernelGGL(k_iota_i32, dim3(stream_grid(n)), dim3(kBlock), 0, s, g->new_id, n);
        TC_HIP(hipGetLastError());
        return MIS_OK;
    }
    if (g->reorder == MIS_REORDER_RCM) {
        std::vector<int64_t> rp(n + 1);
        std::vector<int32_t> ci(g->nnz);
        TC_HIP(hipMemcpyAsync(rp.data(), g->row_ptr, (n + 1) * 8, hipMemcpyDeviceToHost, s));
        if (g->nnz) TC_HIP(hipMemcpyAsync(ci.data(), g->col_idx, g->nnz * 4, hipMemcpyDeviceToHost, s));
        TC_HIP(hipStreamSynchronize(s));
        std::vector<int32_t> nid;
        TC_CHECK(host_rcm(rp.data(), ci.data(), n, nid));
        TC_HIP(hipMemcpyAsync(g->new_id, nid.data(), n * 4, hipMemcpyHostToDevice, s));
        TC_HIP(hipStreamSynchronize(s));
        return MIS_OK;
    }
    TmpBuf tmp;
    uint64_t *sk = nullptr, *sk2 = nullptr;
    uint32_t *pl = nullptr, *pl2 = nullptr;
    TC_CHECK(tmp.alloc((void**)&sk, n * 8));
    TC_CHECK(tmp.alloc((void**)&sk2, n * 8));
    TC_CHECK(tmp.alloc((void**)&pl, n * 4));
    TC_CHECK(tmp.alloc((void**)&pl2, n * 4));
    hipLaunchKernelGGL(k_order_keys, dim3(stream_grid(n)), dim3(kBlock), 0, s, g->row_ptr, g->key, n, g->reorder, sk, pl);
    TC_HIP(hipGetLastError());
    bool alt = false;
    TC_CHECK(radix_sort_u64(sk, sk2, pl, pl2, n, 0, 64, &alt, s));
    hipLaunchKernelGGL(k_scatter_rank, dim3(stream_grid(n)), dim3(kBlock), 0, s, alt ? pl2 : pl, n, g->new_id);
    TC_HIP(hipGetLastError());
    TC_HIP(hipStreamSynchronize(s));
    return MIS_OK;
}

int build_tiles(mis_graph* g, hipStream_t s) {
    const int64_t n = g->n, nnz = g->nnz;
    const int T = g->tile;
    const int tshift = T == 16 ? 4 : 5;
    g->nI = ceil_div(n, T);
    const int64_t nI = g->nI;
    const int bj = bits_for(nI), bi = bits_for(nI);

    TmpBuf tmp;
    uint64_t *ent = nullptr, *ent2 = nullptr;
    unsigned long long* d_valid = nullptr;
    TC_CHECK(tmp.alloc((void**)&ent, (size_t)nnz * 8));
    TC_CHECK(tmp.alloc((void**)&ent2, (size_t)nnz * 8));
    TC_CHECK(tmp.alloc((void**)&d_valid, 8));
    TC_HIP(hipMemsetAsync(d_valid, 0, 8, s));
    if (nnz > 0)
        hipLaunchKernelGGL(k_tile_entries, dim3(stream_grid(nnz)), dim3(kBlock), 0, s, g->row_ptr, g->col_idx, n, nnz,
                           g->new_id, g->key, g->orient, tshift, bj, ent, d_valid);
    TC_HIP(hipGetLastError());
    unsigned long long nvalid_u = 0;
    TC_CHECK(read_scalar(d_valid, &nvalid_u, s));
    const int64_t nvalid = (int64_t)nvalid_u;
    bool alt = false;
    TC_CHECK(radix_sort_u64(ent, ent2, nullptr, nullptr, nnz, 10, 10 + bi + bj, &alt, s));
    uint64_t* sorted = alt ? ent2 : ent;

    int64_t *flag = nullptr, *excl = nullptr, *d_tiles = nullptr, *rb_cnt = nullptr;
    TC_CHECK(tmp.alloc((void**)&flag, (size_t)nvalid * 8));
    TC_CHECK(tmp.alloc((void**)&excl, (size_t)nvalid * 8));
    TC_CHECK(tmp.alloc((void**)&d_tiles, 8));
    TC_CHECK(tmp.alloc((void**)&rb_cnt, (size_t)(nI + 1) * 8));
    if (nvalid > 0)
        hipLaunchKernelGGL(k_tile_flags, dim3(stream_grid(nvalid)), dim3(kBlock), 0, s, sorted, nvalid, flag);
    TC_HIP(hipGetLastError());
    TC_CHECK(scan_exclusive_i64(flag, excl, nvalid, d_tiles, s));
    TC_CHECK(read_scalar(d_tiles, &g->ntiles, s));
    const int64_t nt = g->ntiles;
    const int64_t words = (int64_t)T * T / 32;
    TC_CHECK(galloc(g, (void**)&g->tile_col, (size_t)nt * 4));
    TC_CHECK(galloc(g, (void**)&g->tile_bits, (size_t)nt * words * 4));
    TC_CHECK(galloc(g, (void**)&g->rb_ptr, (size_t)(nI + 1) * 8));
    TC_HIP(hipMemsetAsync(g->tile_bits, 0, (size_t)nt * words * 4, s));
    TC_HIP(hipMemsetAsync(rb_cnt, 0, (size_t)(nI + 1) * 8, s));
    if (nvalid > 0)
        hipLaunchKernelGGL(k_tile_fill, dim3(stream_grid(nvalid)), dim3(kBlock), 0, s, sorted, nvalid, flag, excl, T, bj,
                           g->tile_col, g->tile_bits, rb_cnt);
    TC_HIP(hipGetLastError());
    TC_CHECK(scan_exclusive_i64(rb_cnt, g->rb_ptr, nI + 1, nullptr, s));

    // work segments of at most kSegTiles tiles (every row-block has >= 1)
    int64_t *segc = nullptr, *seg0 = nullptr, *d_nseg = nullptr;
    TC_CHECK(tmp.alloc((void**)&segc, (size_t)nI * 8));
    TC_CHECK(tmp.alloc((void**)&seg0, (size_t)nI * 8));
    TC_CHECK(tmp.alloc((void**)&d_nseg, 8));
    if (nI > 0) hipLaunchKernelGGL(k_seg_count, dim3(stream_grid(nI)), dim3(kBlock), 0, s, g->rb_ptr, nI, segc);
    TC_CHECK(scan_exclusive_i64(segc, seg0, nI, d_nseg, s));
    TC_CHECK(read_scalar(d_nseg, &g->nseg, s));
    const int64_t ns = g->nseg;
    TC_CHECK(galloc(g, (void**)&g->seg_rb, (size_t)ns * 4));
    TC_CHECK(galloc(g, (void**)&g->seg_t0, (size_t)ns * 8));
    TC_CHECK(galloc(g, (void**)&g->seg_t1, (size_t)ns * 8));
    TC_CHECK(galloc(g, (void**)&g->rb_seg0, (size_t)nI * 4));
    TC_CHECK(galloc(g, (void**)&g->rb_nseg, (size_t)nI * 4));
    TC_CHECK(galloc(g, (void**)&g->alive0, (size_t)nI * 4));
    if (nI > 0)
        hipLaunchKernelGGL(k_seg_fill, dim3(stream_grid(nI)), dim3(kBlock), 0, s, g->rb_ptr, seg0, nI, n, T, g->seg_rb,
                           g->seg_t0, g->seg_t1, g->rb_seg0, g->rb_nseg, g->alive0);
    TC_HIP(hipGetLastError());
    TC_CHECK(galloc(g, (void**)&g->seg_all, (size_t)ns * 4));
    if (ns > 0) hipLaunchKernelGGL(k_iota_i32, dim3(stream_grid(ns)), dim3(kBlock), 0, s, g->seg_all, ns);

    if (!g->orient) {
        TC_CHECK(galloc(g, (void**)&g->key_p, (size_t)nI * T * 8));
        TC_HIP(hipMemsetAsync(g->key_p, 0, (size_t)nI * T * 8, s));
        if (n > 0) hipLaunchKernelGGL(k_permute_keys, dim3(stream_grid(n)), dim3(kBlock), 0, s, g->key, g->new_id, n, g->key_p);
        TC_HIP(hipGetLastError());
    }
    // per-round state
    TC_CHECK(galloc(g, (void**)&g->alive, (size_t)nI * 4));
    TC_CHECK(galloc(g, (void**)&g->cand, (size_t)nI * 8));
    TC_CHECK(galloc(g, (void**)&g->inmask, (size_t)nI * 4));
    TC_CHECK(galloc(g, (void**)&g->acc, (size_t)nI * 2 * 4));
    TC_CHECK(galloc(g, (void**)&g->done, (size_t)nI * 2 * 4));
    TC_CHECK(galloc(g, (void**)&g->seglist[0], (size_t)ns * 4));
    TC_CHECK(galloc(g, (void**)&g->seglist[1], (size_t)ns * 4));
    TC_HIP(hipMemsetAsync(g->acc, 0, (size_t)nI * 2 * 4, s));
    TC_HIP(hipMemsetAsync(g->done, 0, (size_t)nI * 2 * 4, s));
    TC_HIP(hipStreamSynchronize(s));
    return MIS_OK;
}

}  // namespace tcmis
