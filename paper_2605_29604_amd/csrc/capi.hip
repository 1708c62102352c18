// C ABI: argument checking, option resolution, the handle, and the polled round loop.
#include <algorithm>
#include <mutex>
#include <new>
#include <cstring>
#include <string>
#include <vector>

#include "round.hpp"

namespace tcmis {

int validate_graph(const mis_csr* csr, const uint64_t* user_keys, const int64_t* goff, int64_t count,
                   uint32_t* d_err, hipStream_t s);
int build_keys(mis_graph* g, const mis_build_opts* o, hipStream_t s);
int build_csr_lists(mis_graph* g, hipStream_t s);
int build_order(mis_graph* g, hipStream_t s);
int build_tiles(mis_graph* g, hipStream_t s);
int csr_init(GraphCore* g, hipStream_t s);
int csr_enqueue_phase(GraphCore* g, int phase, int r, hipStream_t s);
int csr_output(GraphCore* g, uint8_t* in_set, bool if_done, hipStream_t s);
int tile_init(GraphCore* g, hipStream_t s);
int tile_enqueue_phase(GraphCore* g, int phase, int r, hipStream_t s);
int tile_output(GraphCore* g, uint8_t* in_set, bool if_done, hipStream_t s);
int tile_enqueue_rounds(GraphCore* g, int k, hipStream_t s);
int csr_enqueue_rounds(GraphCore* g, int k, hipStream_t s);
int build_hybrid(mis_graph* g, hipStream_t s);
int hyb_init(GraphCore* g, hipStream_t s);
int hyb_enqueue_phase(GraphCore* g, int phase, int r, hipStream_t s, bool first);
int hyb_output(GraphCore* g, uint8_t* in_set, bool if_done, hipStream_t s);
int hyb_enqueue_rounds(GraphCore* g, int k, hipStream_t s);

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }

namespace {

int fail(int code, const std::string& msg) {
    set_error(msg);
    return code;
}

// Pinned host staging for the round-loop polls: a mirror of the workspace span that
// holds ctrl, meta and the trace ring (adjacent in the layout), so that one copy
// brings back all three.  Buffers come from a process-wide pool (a solve takes one
// and gives it back), so concurrent solves on different threads never share one.
// Nothing frees them from a static or thread-local destructor: those run inside
// exit(), when the HIP runtime may already be gone.  mis_release_host_buffers()
// frees the idle ones explicitly; whatever is left is returned with the process.
struct Staging {
    char* base = nullptr;
    size_t bytes = 0;
    size_t off_meta = 0, off_trace = 0;
    Ctrl* ctrl = nullptr;
    Meta* meta = nullptr;
    TraceRec* trace = nullptr;
};

struct StagingPool {
    std::mutex mu;
    std::vector<Staging*> idle;
};
// deliberately never destroyed (see above)
StagingPool& staging_pool() {
    static StagingPool* p = new StagingPool();
    return *p;
}

// Takes a staging buffer laid out for g (allocating one if no idle buffer is big
// enough); give it back with staging_put.
int staging_get(const GraphCore* g, Staging** out) {
    const size_t om = (size_t)((const char*)g->smeta - (const char*)g->ctrl);
    const size_t ot = (size_t)((const char*)g->trace - (const char*)g->ctrl);
    const size_t need = ot + sizeof(TraceRec) * kTraceCap;
    Staging* st = nullptr;
    {
        StagingPool& P = staging_pool();
        std::lock_guard<std::mutex> lock(P.mu);
        for (size_t i = 0; i < P.idle.size(); ++i) {
            if (P.idle[i]->bytes >= need) {
                st = P.idle[i];
                P.idle.erase(P.idle.begin() + (std::ptrdiff_t)i);
                break;
            }
        }
    }
    if (!st) {
        st = new (std::nothrow) Staging();
        if (!st) return fail(MIS_ENOMEM, "host allocation failed");
        if (hipHostMalloc((void**)&st->base, need, hipHostMallocDefault) != hipSuccess) {
            delete st;
            return fail(MIS_ENOMEM, "pinned host allocation failed");
        }
        st->bytes = need;
    }
    st->off_meta = om;
    st->off_trace = ot;
    st->ctrl = reinterpret_cast<Ctrl*>(st->base);
    st->meta = reinterpret_cast<Meta*>(st->base + om);
    st->trace = reinterpret_cast<TraceRec*>(st->base + ot);
    *out = st;
    return MIS_OK;
}

void staging_put(Staging* st) {
    if (!st) return;
    StagingPool& P = staging_pool();
    std::lock_guard<std::mutex> lock(P.mu);
    P.idle.push_back(st);
}

__global__ void k_ctrl_init(Ctrl* ctrl, Meta* smeta, const Meta* meta, int64_t* stripes, int64_t n) {
    ctrl_reset(ctrl, smeta, meta, stripes, n);
}

// Checks arguments and resolves automatic options (host-only).
int resolve(const mis_csr* csr, const mis_build_opts* opts, mis_build_opts* o, int32_t count = 0,
            const int64_t* offsets = nullptr) {
    if (!csr) return fail(MIS_EINVAL, "csr is null");
    if (csr->n < 0 || csr->n >= (1ll << 31)) return fail(MIS_EINVAL, "n must be in [0, 2^31)");
    if (csr->nnz < 0 || csr->nnz >= (1ll << 40)) return fail(MIS_EINVAL, "nnz must be in [0, 2^40)");
    if (!csr->row_ptr) return fail(MIS_EINVAL, "row_ptr is null");
    if (csr->nnz > 0 && !csr->col_idx) return fail(MIS_EINVAL, "col_idx is null");
    if (opts) *o = *opts; else mis_default_opts(o);
    if (o->path < MIS_PATH_AUTO || o->path > MIS_PATH_HYBRID) return fail(MIS_EINVAL, "bad path");
    if (o->dense_min < -1) return fail(MIS_EINVAL, "dense_min must be >= -1");
    if (o->key_rule < MIS_KEY_DEGREE || o->key_rule > MIS_KEY_EQ1) return fail(MIS_EINVAL, "bad key_rule");
    if (o->timing < 0 || o->timing > 1) return fail(MIS_EINVAL, "timing must be 0 or 1");
    if (o->tile != 0 && o->tile != 16 && o->tile != 32) return fail(MIS_EINVAL, "tile must be 0, 16 or 32");
    if (o->reorder < MIS_REORDER_AUTO || o->reorder > MIS_REORDER_RCM) return fail(MIS_EINVAL, "bad reorder");
    if (o->orient < -1 || o->orient > 1) return fail(MIS_EINVAL, "orient must be -1, 0 or 1");
    if (o->poll_rounds < 0 || o->poll_rounds > kTraceCap) return fail(MIS_EINVAL, "poll_rounds out of range");
    if (o->launch < MIS_LAUNCH_AUTO || o->launch > MIS_LAUNCH_PERSISTENT) return fail(MIS_EINVAL, "bad launch mode");
    if (o->blocks_per_cu < 0 || o->blocks_per_cu > 32) return fail(MIS_EINVAL, "blocks_per_cu must be in [0, 32]");
    if (count < 0) return fail(MIS_EINVAL, "count must be >= 0");
    if (count > 0) {
        if (!offsets) return fail(MIS_EINVAL, "offsets is null");
        if (offsets[0] != 0 || offsets[count] != csr->n) return fail(MIS_EINVAL, "offsets must run from 0 to n");
        for (int32_t i = 0; i < count; ++i) {
            if (offsets[i + 1] < offsets[i]) return fail(MIS_EINVAL, "offsets must not decrease");
            if (!o->keys && offsets[i + 1] - offsets[i] > (1ll << 24))
                return fail(MIS_EINVAL, "the default key rule needs graphs of at most 2^24 vertices; pass keys");
        }
    } else if (!o->keys && csr->n > (1ll << 24)) {
        return fail(MIS_EINVAL, "the default key rule needs n <= 2^24; pass keys");
    }
    if (o->path == MIS_PATH_AUTO) o->path = MIS_PATH_HYBRID;
    // the tile and CSR paths index adjacency entries with 32-bit offsets; the hybrid
    // path's entry offsets are 64-bit (the caller's row pointer)
    if (o->path != MIS_PATH_HYBRID && csr->nnz >= (1ll << 31))
        return fail(MIS_EINVAL, "the tile and CSR paths need nnz < 2^31 (the hybrid path takes more)");
    if (o->path == MIS_PATH_HYBRID) {
        if (o->tile != 0 && o->tile != 16) return fail(MIS_EINVAL, "the hybrid path uses 16 x 16 tiles");
        if (o->reorder != MIS_REORDER_AUTO && o->reorder != MIS_REORDER_NONE)
            return fail(MIS_EINVAL, "the hybrid path keeps the input order");
        if (o->orient == 0) return fail(MIS_EINVAL, "the hybrid path stores higher-priority edges only");
        o->tile = 16;
        o->reorder = MIS_REORDER_NONE;
        o->orient = 1;
        if (o->dyn_slack < 0) return fail(MIS_EINVAL, "dyn_slack must be >= 0");
        if (o->dyn_slack > 0) {
            if (count > 0) return fail(MIS_EINVAL, "a dynamic handle holds one graph");
            if (o->dense_min > 0) return fail(MIS_EINVAL, "a dynamic handle keeps entry lists only (dense_min -1)");
            o->dense_min = -1;
        }
        if (o->dense_min == 0) o->dense_min = kDenseMinDefault;
    } else if (o->dyn_slack != 0) {
        return fail(MIS_EINVAL, "dyn_slack needs the hybrid path");
    } else if (o->path == MIS_PATH_TILE) {
        if (o->tile == 0) o->tile = 16;
        if (o->reorder == MIS_REORDER_AUTO) o->reorder = MIS_REORDER_KEY;
        if (o->orient < 0) o->orient = 1;
    } else {
        o->tile = 0;
        o->reorder = MIS_REORDER_NONE;
        o->orient = 0;
    }
    if (o->poll_rounds == 0) o->poll_rounds = 4;
    return MIS_OK;
}

}  // namespace

void build_mark(mis_graph* g, hipStream_t s) {
    if (!g->btiming) return;
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return;
    if (hipEventRecord(e, s) != hipSuccess) {
        (void)hipEventDestroy(e);
        return;
    }
    g->bev.push_back(e);
}

namespace {

void configure(GraphCore* g, const mis_csr* csr, const mis_build_opts& o) {
    g->n = csr->n;
    g->nnz = csr->nnz;
    g->row_ptr = csr->row_ptr;
    g->col_idx = csr->col_idx;
    g->path = o.path;
    g->tile = o.tile;
    g->reorder = o.reorder;
    g->orient = o.orient;
    g->poll_rounds = o.poll_rounds;
    g->launch = o.launch;
    g->user_keys = o.keys != nullptr;
    g->seed = o.seed;
    g->btiming = o.timing != 0;
    g->dense_min = o.path == MIS_PATH_HYBRID && o.dense_min > 0 ? o.dense_min : 0;
    g->dyn_slack = o.path == MIS_PATH_HYBRID ? o.dyn_slack : 0;
}

// kernels per round: tile path candidate / exclusion / finalize, CSR and hybrid paths
// candidate / exclusion
int phases(const GraphCore* g) { return g->path == MIS_PATH_TILE ? 3 : 2; }

// first: the phase belongs to the solve's first round (the hybrid path gives it a
// thread per vertex)
int enqueue_phase(GraphCore* g, int phase, int r, hipStream_t s, bool first) {
    if (g->path == MIS_PATH_HYBRID) return hyb_enqueue_phase(g, phase, r, s, first);
    return g->path == MIS_PATH_TILE ? tile_enqueue_phase(g, phase, r, s) : csr_enqueue_phase(g, phase, r, s);
}

// per-graph rounds (largest decision round of its vertices) and set sizes; one
// workgroup of kStatsBlock threads per graph, four consecutive vertices per thread and
// step with their loads in flight together
constexpr int kStatsBlock = 1024;
__global__ void __launch_bounds__(kStatsBlock) k_batch_stats(const int64_t* goff, const uint8_t* in_set,
                                                             const int32_t* new_id, const int32_t* dround,
                                                             const uint32_t* st, int32_t* g_rounds, int64_t* g_in) {
    __shared__ int32_t smax[kStatsBlock / kWave];
    __shared__ int64_t ssum[kStatsBlock / kWave];
    const int64_t g = blockIdx.x;
    const int64_t v1 = goff[g + 1];
    int32_t mx = 0;
    int64_t sum = 0;
    for (int64_t b = goff[g] + 4 * (int64_t)threadIdx.x; b < v1; b += 4 * kStatsBlock) {
        int32_t r[4];
        uint32_t in[4];
        #pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t v = b + j;
            r[j] = 0;
            in[j] = 0;
            if (v < v1) {
                r[j] = new_id ? dround[new_id[v]] : st ? (int32_t)(st[v] >> 2) : dround[v];
                in[j] = in_set[v];
            }
        }
        #pragma unroll
        for (int j = 0; j < 4; ++j) {
            mx = max(mx, r[j]);
            sum += in[j];
        }
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
        mx = max(mx, __shfl_xor(mx, off, kWave));
        sum += __shfl_xor(sum, off, kWave);
    }
    if (lane_id() == 0) { smax[threadIdx.x / kWave] = mx; ssum[threadIdx.x / kWave] = sum; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kStatsBlock / kWave; ++w) { mx = max(mx, smax[w]); sum += ssum[w]; }
        g_rounds[g] = mx;
        g_in[g] = sum;
    }
}

// closes the last round of a batch of k rounds and moves the round base past it
// (one wave)
__global__ void k_close(Ctrl* ctrl, int64_t* stripes, TraceRec* trace, int k) {
    const int rb = ctrl->rbase;
    close_round(ctrl, stripes, trace, rb + k);
    if (threadIdx.x == 0) ctrl->rbase = rb + k;
}

// enqueues a batch of k rounds (round indices 1..k after the device-side base) and
// the close kernel; first: the batch opens the solve
int enqueue_batch(GraphCore* g, int64_t k, hipStream_t s, hipEvent_t* ev, bool first) {
    for (int64_t i = 0; i < k; ++i) {
        const int P = phases(g);
        for (int ph = 0; ph < P; ++ph) {
            if (ev) (void)hipEventRecord(ev[(P + 1) * i + ph], s);
            TC_CHECK(enqueue_phase(g, ph, (int)(i + 1), s, first && i == 0));
        }
        if (ev) (void)hipEventRecord(ev[(P + 1) * i + P], s);
    }
    hipLaunchKernelGGL(k_close, dim3(1), dim3(kWave), 0, s, g->ctrl, g->stripes, g->trace, (int)k);
    TC_HIP(hipGetLastError());
    return MIS_OK;
}

// captures a full batch (poll_rounds rounds) once, on a private stream
bool ensure_graph(mis_graph* g) {
    if (g->graph_exec) return true;
    if (g->graph_failed) return false;
    bool ok = hipStreamCreateWithFlags(&g->cap_stream, hipStreamNonBlocking) == hipSuccess &&
              hipStreamBeginCapture(g->cap_stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
        const int rc = enqueue_batch(g, g->poll_rounds, g->cap_stream, nullptr, false);
        hipGraph_t graph = nullptr;
        ok = hipStreamEndCapture(g->cap_stream, &graph) == hipSuccess && rc == MIS_OK && graph;
        if (ok) {
            g->graph = graph;
            ok = hipGraphInstantiate(&g->graph_exec, graph, nullptr, nullptr, 0) == hipSuccess;
        } else if (graph) {
            (void)hipGraphDestroy(graph);
        }
    }
    if (!ok) {
        (void)hipGetLastError();
        g->graph_failed = true;
    }
    return ok;
}

// bytes the kernels must move per work unit (see TraceRec::u)
int64_t unit_bytes(const GraphCore* g, int k) {
    if (g->path == MIS_PATH_CSR) {
        static const int64_t b[kUnits] = {12, 28, 8, 24, 0, 0, 0, 0};
        return b[k];
    }
    if (g->path == MIS_PATH_HYBRID) {
        // entries read (the 4-byte index; the neighbour's class or status is a
        // per-vertex vector), rows examined (row bounds and key or list slot), tiles
        // multiplied (bitmap + column block), dense blocks examined (list slot, block
        // slot, tile range, its two bitmap words)
        static const int64_t b[kUnits] = {4, 16, 4, 16, 36, 36, 24, 24};
        return b[k];
    }
    // tile path: 4-byte words, bytes, 4-byte words, bitmaps multiplied, row-blocks
    // finalized (alive, blocked, hit read and written), chunk entries written
    const int64_t S = (int64_t)g->tile * g->tile / 8;
    static const int64_t b[kUnits] = {4, 1, 4, 0, 24, 8, 0, 0};
    return k == 3 ? S : b[k];
}

}  // namespace

int solve_begin(GraphCore* g, hipStream_t s) {
    g->enq_rounds = 0;
    if (g->path == MIS_PATH_HYBRID) return hyb_init(g, s);   // resets the control block too
    hipLaunchKernelGGL(k_ctrl_init, dim3(1), dim3(256), 0, s, g->ctrl, g->smeta, g->meta, g->stripes, g->n);
    TC_HIP(hipGetLastError());
    return g->path == MIS_PATH_TILE ? tile_init(g, s) : csr_init(g, s);
}

// Launches a persistent round kernel taking (args, k) on the cooperative grid: every
// workgroup must be resident, at most two per compute unit within what the kernel's
// resources allow (sized from the kernel on each launch, so that concurrent solves
// share no host state).
int launch_cooperative(const void* kernel, GraphCore* g, void* args, int k, hipStream_t s) {
    int dev = 0, cus = 0, per = 0;
    TC_HIP(hipGetDevice(&dev));
    TC_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    TC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, kBlock, 0));
    if (per < 1 || cus < 1) return fail(MIS_EHIP, "the persistent round kernel cannot be resident");
    const int blocks = cus * std::min(per, 2);
    void* kargs[2] = {args, &k};
    TC_HIP(hipLaunchCooperativeKernel(kernel, dim3((unsigned)blocks), dim3(kBlock), kargs, 0, s));
    return MIS_OK;
}

int solve_rounds(GraphCore* g, int64_t k, bool allow_graph, hipStream_t s, mis_graph* owner) {
    const bool first = g->enq_rounds == 0;
    g->enq_rounds += k;
    if (g->launch == MIS_LAUNCH_PERSISTENT) {
        if (g->path == MIS_PATH_HYBRID) return hyb_enqueue_rounds(g, (int)k, s);
        return g->path == MIS_PATH_TILE ? tile_enqueue_rounds(g, (int)k, s) : csr_enqueue_rounds(g, (int)k, s);
    }
    // auto: a handle solved once gains nothing from a capture, which costs more than
    // the launches it replaces; capture when it is solved again (only over the
    // handle's own round state: a captured graph holds its addresses).  The first
    // batch of a solve is always launched directly: its first round has a launch
    // shape of its own.
    const bool graph = owner && (g->launch == MIS_LAUNCH_GRAPH || (g->launch == MIS_LAUNCH_AUTO && owner->solves > 1));
    if (allow_graph && graph && !first && k == g->poll_rounds && ensure_graph(owner)) {
        if (hipGraphLaunch(owner->graph_exec, s) != hipSuccess) return fail(MIS_EHIP, "hipGraphLaunch failed");
        return MIS_OK;
    }
    return enqueue_batch(g, k, s, nullptr, first);
}

int resolve_opts(const mis_csr* csr, const mis_build_opts* opts, mis_build_opts* o, int32_t count,
                 const int64_t* offsets) {
    return resolve(csr, opts, o, count, offsets);
}

void configure_graph(GraphCore* g, const mis_csr* csr, const mis_build_opts& o, int32_t count) {
    configure(g, csr, o);
    g->count = count;
}

int build_into(mis_graph* g, const mis_csr* csr, const mis_build_opts& o, int32_t count, const int64_t* offsets,
               char* ws, size_t need, hipStream_t s) {
    g->ws = ws;
    g->ws_bytes = need;
    layout(g, g->ws);
    int dev = 0, cus = 256;
    TC_HIP(hipGetDevice(&dev));
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    g->cus = std::max(1, cus);
    g->grid_blocks = g->cus * (o.blocks_per_cu ? o.blocks_per_cu : 8);
    int rc = MIS_OK;
    if (count > 0 && hipMemcpyAsync(g->goff, offsets, (size_t)(count + 1) * 8, hipMemcpyHostToDevice, s) != hipSuccess)
        rc = fail(MIS_EHIP, "copy of the batch offsets failed");
    if (rc == MIS_OK && o.validate) rc = validate_graph(csr, o.keys, g->goff, count, &g->ctrl->error, s);
    build_mark(g, s);
    if (rc == MIS_OK) rc = build_keys(g, &o, s);
    build_mark(g, s);
    if (rc == MIS_OK) {
        if (g->path == MIS_PATH_CSR) rc = build_csr_lists(g, s);
        else if (g->path == MIS_PATH_HYBRID) rc = build_hybrid(g, s);
        else {
            rc = build_order(g, s);
            build_mark(g, s);
            if (rc == MIS_OK) rc = build_tiles(g, s);
        }
    }
    build_mark(g, s);
    return rc;
}

int solve_output(GraphCore* g, uint8_t* in_set, hipStream_t s, bool if_done) {
    if (g->path == MIS_PATH_HYBRID) return hyb_output(g, in_set, if_done, s);
    return g->path == MIS_PATH_TILE ? tile_output(g, in_set, if_done, s) : csr_output(g, in_set, if_done, s);
}

}  // namespace tcmis

using namespace tcmis;

extern "C" {

void mis_default_opts(mis_build_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->path = MIS_PATH_AUTO;
    o->tile = 0;
    o->reorder = MIS_REORDER_AUTO;
    o->orient = -1;
    o->validate = 0;
    o->poll_rounds = 0;
    o->seed = 1;
    o->keys = nullptr;
}

const char* mis_status_string(int s) {
    switch (s) {
        case MIS_OK: return "ok";
        case MIS_EINVAL: return "invalid argument";
        case MIS_ENOTSYM: return "adjacency not symmetric";
        case MIS_ESELFLOOP: return "self-loop";
        case MIS_EDUP: return "duplicate or unsorted adjacency entry";
        case MIS_ERANGE: return "index out of range";
        case MIS_ENOMEM: return "out of device memory";
        case MIS_EBUSY: return "busy: no free slot or arena region";
        case MIS_EHIP: return "HIP runtime error";
        case MIS_EINTERNAL: return "internal error";
        default: return "unknown status";
    }
}

const char* mis_last_error(void) { return g_last_error.c_str(); }

const char* mis_version(void) { return "tcmis-hip 0.1 gfx950"; }

int mis_build_bytes(const mis_csr* csr, const mis_build_opts* opts, size_t* bytes) {
    return mis_build_batch_bytes(csr, 0, nullptr, opts, bytes);
}

int mis_build_batch_bytes(const mis_csr* csr, int32_t count, const int64_t* offsets, const mis_build_opts* opts,
                          size_t* bytes) {
    g_last_error.clear();
    if (!bytes) return fail(MIS_EINVAL, "bytes is null");
    mis_build_opts o;
    TC_CHECK(resolve(csr, opts, &o, count, offsets));
    mis_graph g;
    configure(&g, csr, o);
    g.count = count;
    *bytes = layout(&g, nullptr);
    return MIS_OK;
}

int mis_build_tiles(const mis_csr* csr, const mis_build_opts* opts, void* workspace, size_t workspace_bytes,
                    void* stream, mis_graph** out) {
    return mis_build_batch(csr, 0, nullptr, opts, workspace, workspace_bytes, stream, out);
}

int mis_build_batch(const mis_csr* csr, int32_t count, const int64_t* offsets, const mis_build_opts* opts,
                    void* workspace, size_t workspace_bytes, void* stream, mis_graph** out) {
    g_last_error.clear();
    if (!out) return fail(MIS_EINVAL, "out is null");
    *out = nullptr;
    mis_build_opts o;
    TC_CHECK(resolve(csr, opts, &o, count, offsets));
    mis_graph* g = new (std::nothrow) mis_graph();
    if (!g) return fail(MIS_ENOMEM, "host allocation failed");
    configure(g, csr, o);
    g->count = count;
    const size_t need = layout(g, nullptr);
    if (!workspace || workspace_bytes < need || ((uintptr_t)workspace & 255)) {
        delete g;
        return fail(MIS_EINVAL, "workspace must be 256-byte aligned device memory of at least " +
                                    std::to_string(need) + " bytes (mis_build_bytes)");
    }
    const int rc = build_into(g, csr, o, count, offsets, (char*)workspace, need, (hipStream_t)stream);
    if (rc != MIS_OK) {
        delete g;
        return rc;
    }
    *out = g;
    return MIS_OK;
}

int mis_graph_bytes(const mis_graph* g, size_t* bytes) {
    if (!g || !bytes) return fail(MIS_EINVAL, "null argument");
    *bytes = g->ws_bytes;
    return MIS_OK;
}

}  // extern "C"

namespace tcmis {
namespace {

// The round loop of one solve over g's round state (the handle's own when owner is
// the handle: then the loop may replay a captured graph of it; a caller's scratch
// otherwise).
int solve_loop(GraphCore* g, mis_graph* owner, uint8_t* in_set, int32_t max_rounds, mis_stats* st, hipStream_t s) {
    const bool timing = st && st->timing;
    Staging* sg = nullptr;
    TC_CHECK(staging_get(g, &sg));
    struct Give {   // the buffer goes back to the pool on every return path
        Staging* s;
        ~Give() { staging_put(s); }
    } give{sg};
    if (owner) ++owner->solves;
    TC_CHECK(solve_begin(g, s));

    const int P = phases(g);
    std::vector<hipEvent_t> ev;
    if (timing) {
        ev.resize((size_t)(P + 1) * g->poll_rounds);
        for (auto& e : ev) TC_HIP(hipEventCreate(&e));
    }
    double kms[3] = {0.0, 0.0, 0.0};
    int64_t launches = 0;
    int64_t units[kUnits] = {};
    int64_t enq = 0, drained = 0;
    int rc = MIS_OK;
    if (g->n > 0) {
        for (;;) {
            int64_t k = g->poll_rounds;
            if (max_rounds > 0) k = std::min<int64_t>(k, max_rounds - enq);
            if (timing) {
                rc = enqueue_batch(g, k, s, ev.data(), g->enq_rounds == 0);
                g->enq_rounds += k;
            } else {
                rc = solve_rounds(g, k, true, s, owner);
            }
            // the result, written by the device only if this batch decided the last vertex
            if (rc == MIS_OK) rc = solve_output(g, in_set, s, true);
            if (rc != MIS_OK) break;
            // ring slots of rounds drained+1 .. enq (ring order; all slots once it wraps),
            // with ctrl and meta in front of them: one copy
            const int64_t first = drained % kTraceCap, cnt = enq + k - drained;
            enq += k;
            const int64_t slots = std::min<int64_t>(first + cnt, kTraceCap);
            const size_t span = sg->off_trace + (size_t)kTraceCap * sizeof(TraceRec);
            const size_t bytes = std::min(span, (sg->off_trace + (size_t)slots * sizeof(TraceRec) + 255) & ~(size_t)255);
            if (hipMemcpyAsync(sg->base, g->ctrl, bytes, hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                rc = fail(MIS_EHIP, std::string("round loop: ") + hipGetErrorString(hipGetLastError()));
                break;
            }
            if (timing) {
                for (int64_t i = 0; i < k; ++i) {
                    for (int ph = 0; ph < P; ++ph) {
                        float ms = 0.f;
                        (void)hipEventElapsedTime(&ms, ev[(P + 1) * i + ph], ev[(P + 1) * i + ph + 1]);
                        kms[ph] += ms;
                    }
                }
                launches += k;
            }
            const int64_t done_rounds = sg->ctrl->round;
            for (int64_t r = drained + 1; r <= done_rounds; ++r) {
                const TraceRec& t = sg->trace[(r - 1) % kTraceCap];
                if (st && st->trace && r <= st->trace_cap) {
                    st->trace[3 * (r - 1) + 0] = t.c;
                    st->trace[3 * (r - 1) + 1] = t.x;
                    st->trace[3 * (r - 1) + 2] = t.alive;
                }
                for (int i = 0; i < kUnits; ++i) units[i] += t.u[i];
            }
            drained = done_rounds;
            if (sg->ctrl->alive == 0) break;
            if (max_rounds > 0 && enq >= max_rounds) break;
            if (done_rounds > g->n + 1) { rc = fail(MIS_EINTERNAL, "round limit exceeded (equal adjacent keys?)"); break; }
        }
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    if (rc != MIS_OK) return rc;
    if (g->n > 0 && (sg->ctrl->error & kErrBarrier))
        return fail(MIS_EINTERNAL, "a grid barrier of the persistent round kernel timed out");
    // a solve stopped by max_rounds still writes the result of the rounds it ran
    if (g->n > 0 && sg->ctrl->alive != 0) TC_CHECK(solve_output(g, in_set, s));
    if (g->n == 0) {   // nothing ran: no staging contents of this graph
        sg->ctrl->round = 0;
        sg->ctrl->n_in = 0;
        sg->meta->ntiles = 0;
        sg->meta->n_dtiles = 0;
    }
    if (st) {
        st->rounds = sg->ctrl->round;
        st->path = g->path;
        st->tile = g->tile;
        st->reorder = g->reorder;
        st->orient = g->orient;
        st->n_in = sg->ctrl->n_in;
        const int64_t nt = g->path == MIS_PATH_TILE ? sg->meta->ntiles
                           : g->path == MIS_PATH_HYBRID ? sg->meta->n_dtiles : 0;
        st->tiles = nt;
        st->tile_bytes = nt * ((int64_t)g->tile * g->tile / 8 + 4);
        int64_t ab = 0;
        for (int i = 0; i < kUnits; ++i) {
            st->units[i] = units[i];
            ab += units[i] * unit_bytes(g, i);
        }
        st->alg_bytes = ab;
        for (int ph = 0; ph < 3; ++ph) st->kernel_ms[ph] = (float)kms[ph];
        st->launches = (int32_t)launches;
        st->graph = timing ? 0 : g->launch == MIS_LAUNCH_PERSISTENT ? 2
                  : (owner && owner->graph_exec != nullptr && g->launch != MIS_LAUNCH_DIRECT);
    }
    return MIS_OK;
}

}  // namespace
}  // namespace tcmis

extern "C" {

int mis_solve_scratch_bytes(const mis_graph* g, size_t* bytes) {
    if (!g || !bytes) return fail(MIS_EINVAL, "null argument");
    GraphCore v = *g;
    *bytes = layout_state(&v, nullptr);
    return MIS_OK;
}

int mis_solve(mis_graph* g, uint8_t* in_set, int32_t max_rounds, void* scratch, size_t scratch_bytes, mis_stats* st,
              void* stream) {
    g_last_error.clear();
    if (!g) return fail(MIS_EINVAL, "graph is null");
    if (g->n > 0 && !in_set) return fail(MIS_EINVAL, "in_set is null");
    if (max_rounds < 0) return fail(MIS_EINVAL, "max_rounds must be >= 0");
    if (st && st->trace_cap > 0 && !st->trace) return fail(MIS_EINVAL, "stats trace buffer is null");
    if (!scratch) return solve_loop(g, g, in_set, max_rounds, st, (hipStream_t)stream);
    GraphCore v = *g;   // the structure's pointers, the round state in the caller's scratch
    const size_t need = layout_state(&v, nullptr);
    if (((uintptr_t)scratch & 255) || scratch_bytes < need)
        return fail(MIS_EINVAL, "scratch must be 256-byte aligned device memory of at least " + std::to_string(need) +
                                    " bytes (mis_solve_scratch_bytes)");
    layout_state(&v, (char*)scratch);
    return solve_loop(&v, nullptr, in_set, max_rounds, st, (hipStream_t)stream);
}

int mis_solve_union(mis_graph* g, uint8_t* in_set, mis_stats* stats, int32_t* graph_rounds, int64_t* graph_in,
                    void* stream) {
    g_last_error.clear();
    if (!g) return fail(MIS_EINVAL, "batch is null");
    if (g->count <= 0) return fail(MIS_EINVAL, "the handle was not built with mis_build_batch");
    TC_CHECK(mis_solve(g, in_set, 0, nullptr, 0, stats, stream));
    hipStream_t s = (hipStream_t)stream;
    if (g->n > 0) {
        hipLaunchKernelGGL(k_batch_stats, dim3((unsigned)g->count), dim3(kStatsBlock), 0, s, g->goff, in_set,
                           g->path == MIS_PATH_TILE ? g->new_id : nullptr, g->dround,
                           g->path == MIS_PATH_CSR ? g->st : nullptr, g->g_rounds, g->g_in);
        TC_HIP(hipGetLastError());
    } else {
        TC_HIP(hipMemsetAsync(g->g_rounds, 0, (size_t)g->count * 4, s));
        TC_HIP(hipMemsetAsync(g->g_in, 0, (size_t)g->count * 8, s));
    }
    if (graph_rounds) TC_HIP(hipMemcpyAsync(graph_rounds, g->g_rounds, (size_t)g->count * 4, hipMemcpyDeviceToHost, s));
    if (graph_in) TC_HIP(hipMemcpyAsync(graph_in, g->g_in, (size_t)g->count * 8, hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    return MIS_OK;
}

void mis_free_tiles(mis_graph* g) { delete g; }

int mis_build_times(const mis_graph* g, float* ms, int32_t cap, int32_t* count) {
    if (!g || !count || cap < 0 || (cap > 0 && !ms)) return fail(MIS_EINVAL, "bad argument");
    if (!g->btiming) return fail(MIS_EINVAL, "the handle was not built with timing = 1");
    const int32_t k = g->bev.empty() ? 0 : (int32_t)g->bev.size() - 1;
    *count = k;
    if (k > 0) TC_HIP(hipEventSynchronize(g->bev.back()));
    for (int32_t i = 0; i < k && i < cap; ++i) TC_HIP(hipEventElapsedTime(&ms[i], g->bev[i], g->bev[i + 1]));
    return MIS_OK;
}

void mis_release_host_buffers(void) {
    StagingPool& P = staging_pool();
    std::lock_guard<std::mutex> lock(P.mu);
    for (Staging* st : P.idle) {
        (void)hipHostFree(st->base);
        delete st;
    }
    P.idle.clear();
}

}  // extern "C"
