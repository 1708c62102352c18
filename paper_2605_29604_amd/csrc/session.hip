// Serving session: continuous batching of MIS requests on one GPU.
//
// Every admitted request gets a slot (its own default-priority stream, event and
// pinned control-block mirror) and a region of the caller's device arena that holds
// its CSR copy, its solver structure and its output.  The host scheduler never
// blocks on one request: mis_session_progress polls every slot's event, enqueues the
// next `rounds_per_step` rounds of a request whose previous batch has drained, and
// retires finished requests, which frees their slot and arena region for the next
// admission.  Requests that arrive while others are on the device therefore join
// at the next round boundary, and the kernels of all live requests overlap on the
// device.  Each request's rounds read only its own state, so its result is the one
// it gets alone.
#include <chrono>
#include <map>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "arena.hpp"
#include "graph.hpp"

namespace tcmis {
namespace {

enum class Phase { Idle, Rounds, Output };

struct Slot {
    Phase phase = Phase::Idle;
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    Ctrl* h_ctrl = nullptr;       // pinned mirror of the request's control block
    mis_graph* g = nullptr;
    uint64_t tag = 0;
    size_t off = 0, bytes = 0;
    uint8_t* d_out = nullptr;
    uint8_t* h_out = nullptr;
    int64_t n = 0;
    int32_t rounds = 0, status = MIS_OK;
    int64_t n_in = 0;
    double t_admit = 0.0;
};

double now_s(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace
}  // namespace tcmis

struct mis_session {
    mis_session_config cfg{};
    char* base = nullptr;
    tcmis::Arena arena;
    std::vector<tcmis::Slot> slots;
    tcmis::Ctrl* h_ctrl = nullptr;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    int32_t live = 0;
};

using namespace tcmis;

namespace {

int sfail(int code, const std::string& msg) {
    set_error(msg);
    return code;
}

// enqueues the next batch of rounds of a live request and the poll of its control block
int enqueue_step(mis_session* S, Slot& sl) {
    TC_CHECK(solve_rounds(sl.g, S->cfg.rounds_per_step, true, sl.stream));
    TC_HIP(hipMemcpyAsync(sl.h_ctrl, sl.g->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, sl.stream));
    TC_HIP(hipEventRecord(sl.ev, sl.stream));
    sl.phase = Phase::Rounds;
    return MIS_OK;
}

int enqueue_output(Slot& sl) {
    if (sl.n > 0) {
        TC_CHECK(solve_output(sl.g, sl.d_out, sl.stream));
        if (sl.h_out) TC_HIP(hipMemcpyAsync(sl.h_out, sl.d_out, (size_t)sl.n, hipMemcpyDeviceToHost, sl.stream));
    }
    TC_HIP(hipEventRecord(sl.ev, sl.stream));
    sl.phase = Phase::Output;
    return MIS_OK;
}

void retire(mis_session* S, Slot& sl) {
    mis_free_tiles(sl.g);
    sl.g = nullptr;
    S->arena.release(sl.off, sl.bytes);
    sl.phase = Phase::Idle;
    --S->live;
}

}  // namespace

extern "C" {

int mis_session_create(const mis_session_config* cfg, mis_session** out) {
    if (!cfg || !out) return sfail(MIS_EINVAL, "null argument");
    *out = nullptr;
    if (!cfg->arena || ((uintptr_t)cfg->arena & 255) || cfg->arena_bytes < 256)
        return sfail(MIS_EINVAL, "arena must be 256-byte aligned device memory of at least 256 bytes");
    if (cfg->max_live < 1 || cfg->max_live > 256) return sfail(MIS_EINVAL, "max_live must be in [1, 256]");
    if (cfg->rounds_per_step < 0 || cfg->rounds_per_step > 1024)
        return sfail(MIS_EINVAL, "rounds_per_step must be in [0, 1024]");
    if (cfg->opts.launch == MIS_LAUNCH_PERSISTENT)
        return sfail(MIS_EINVAL, "a session does not run persistent (cooperative) launches");
    mis_session* S = new (std::nothrow) mis_session();
    if (!S) return sfail(MIS_ENOMEM, "host allocation failed");
    S->cfg = *cfg;
    if (S->cfg.rounds_per_step == 0) S->cfg.rounds_per_step = 4;
    S->cfg.opts.poll_rounds = S->cfg.rounds_per_step;
    S->base = (char*)cfg->arena;
    S->arena.init(cfg->arena_bytes);
    S->slots.resize((size_t)cfg->max_live);
    int rc = MIS_OK;
    if (hipHostMalloc((void**)&S->h_ctrl, sizeof(Ctrl) * (size_t)cfg->max_live, hipHostMallocDefault) != hipSuccess)
        rc = sfail(MIS_ENOMEM, "pinned host allocation failed");
    for (size_t i = 0; rc == MIS_OK && i < S->slots.size(); ++i) {
        Slot& sl = S->slots[i];
        sl.h_ctrl = S->h_ctrl + i;
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess)
            rc = sfail(MIS_EHIP, "stream or event creation failed");
    }
    if (rc != MIS_OK) {
        mis_session_destroy(S);
        return rc;
    }
    *out = S;
    return MIS_OK;
}

int mis_session_admit(mis_session* S, const mis_csr* csr, int32_t csr_on_host, const mis_build_opts* opts,
                      uint8_t* d_out, uint8_t* h_out, uint64_t tag) {
    if (!S || !csr) return sfail(MIS_EINVAL, "null argument");
    if (!d_out && !h_out) return sfail(MIS_EINVAL, "either d_out or h_out is required");
    mis_build_opts o = opts ? *opts : S->cfg.opts;
    o.poll_rounds = S->cfg.rounds_per_step;
    // every live request runs on its own stream; cooperative grids sized to fill the
    // device could not all be resident at once
    if (o.launch == MIS_LAUNCH_PERSISTENT)
        return sfail(MIS_EINVAL, "a session does not run persistent (cooperative) launches");
    size_t build_bytes = 0;
    TC_CHECK(mis_build_bytes(csr, &o, &build_bytes));
    const int64_t n = csr->n, nnz = csr->nnz;
    size_t need = round256(build_bytes);
    const size_t rp_off = need;
    if (csr_on_host) need += round256((size_t)(n + 1) * 8) + round256((size_t)nnz * 4);
    const size_t out_off = need;
    if (!d_out) need += round256((size_t)std::max<int64_t>(n, 1));
    if (need > S->arena.capacity())
        return sfail(MIS_EINVAL, "request needs " + std::to_string(need) + " bytes, more than the session arena");
    Slot* sl = nullptr;
    for (Slot& s : S->slots)
        if (s.phase == Phase::Idle) { sl = &s; break; }
    if (!sl) return sfail(MIS_EBUSY, "every slot is live");
    size_t off = 0;
    if (!S->arena.alloc(need, &off)) return sfail(MIS_EBUSY, "no arena region of " + std::to_string(need) + " bytes free");
    char* region = S->base + off;
    mis_csr dcsr = *csr;
    int rc = MIS_OK;
    if (csr_on_host) {
        int64_t* rp = (int64_t*)(region + rp_off);
        int32_t* ci = (int32_t*)(region + rp_off + round256((size_t)(n + 1) * 8));
        if (hipMemcpyAsync(rp, csr->row_ptr, (size_t)(n + 1) * 8, hipMemcpyHostToDevice, sl->stream) != hipSuccess ||
            (nnz > 0 &&
             hipMemcpyAsync(ci, csr->col_idx, (size_t)nnz * 4, hipMemcpyHostToDevice, sl->stream) != hipSuccess))
            rc = sfail(MIS_EHIP, "copy of the request's CSR failed");
        dcsr.row_ptr = rp;
        dcsr.col_idx = nnz > 0 ? ci : nullptr;
    }
    mis_graph* g = nullptr;
    if (rc == MIS_OK) rc = mis_build_tiles(&dcsr, &o, region, round256(build_bytes), sl->stream, &g);
    if (rc == MIS_OK) rc = solve_begin(g, sl->stream);
    sl->g = g;
    sl->tag = tag;
    sl->off = off;
    sl->bytes = need;
    sl->d_out = d_out ? d_out : (uint8_t*)(region + out_off);
    sl->h_out = h_out;
    sl->n = n;
    sl->rounds = 0;
    sl->n_in = 0;
    sl->status = MIS_OK;
    sl->t_admit = now_s(S->t0);
    if (rc == MIS_OK) rc = n > 0 ? enqueue_step(S, *sl) : enqueue_output(*sl);
    if (rc != MIS_OK) {
        // nothing of this request may still run on the device when its region is reused
        (void)hipStreamSynchronize(sl->stream);
        if (g) mis_free_tiles(g);
        sl->g = nullptr;
        S->arena.release(off, need);
        sl->phase = Phase::Idle;
        return rc;
    }
    ++S->live;
    return MIS_OK;
}

}  // extern "C"

namespace {

// One pass over the slots.  step: a request whose last batch of rounds has drained
// gets its next batch, or its output once it is done.  poll: a request whose output
// has landed is retired into done (at most cap).  Returns through *moved whether
// anything changed.
int session_pass(mis_session* S, bool step, bool poll, mis_done* done, int32_t cap, int32_t* n_done, int32_t* moved) {
    for (Slot& sl : S->slots) {
        if (sl.phase == Phase::Idle) continue;
        if (sl.phase == Phase::Rounds && !step) continue;
        if (sl.phase == Phase::Output && (!poll || *n_done >= cap)) continue;
        const hipError_t q = hipEventQuery(sl.ev);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) return sfail(MIS_EHIP, std::string("request event: ") + hipGetErrorString(q));
        if (sl.phase == Phase::Rounds) {
            sl.rounds = sl.h_ctrl->round;
            sl.n_in = sl.h_ctrl->n_in;
            if (sl.h_ctrl->error != 0) {
                sl.status = MIS_EINTERNAL;   // a device-side invariant check failed
                TC_CHECK(enqueue_output(sl));
            } else if (sl.h_ctrl->alive == 0) {
                TC_CHECK(enqueue_output(sl));
            } else if (sl.h_ctrl->round > sl.n + 1) {
                sl.status = MIS_EINTERNAL;   // a strict key order decides a vertex every round
                TC_CHECK(enqueue_output(sl));
            } else {
                TC_CHECK(enqueue_step(S, sl));
            }
        } else {
            mis_done& d = done[(*n_done)++];
            d.tag = sl.tag;
            d.status = sl.status;
            d.rounds = sl.rounds;
            d.n = sl.n;
            d.n_in = sl.n_in;
            d.admit_s = sl.t_admit;
            d.done_s = now_s(S->t0);
            retire(S, sl);
        }
        ++*moved;
    }
    return MIS_OK;
}

bool any_in(const mis_session* S, Phase p) {
    for (const Slot& sl : S->slots)
        if (sl.phase == p) return true;
    return false;
}

}  // namespace

extern "C" {

int mis_session_step(mis_session* S, int32_t* advanced) {
    if (!S) return sfail(MIS_EINVAL, "session is null");
    int32_t moved = 0, nd = 0;
    TC_CHECK(session_pass(S, true, false, nullptr, 0, &nd, &moved));
    if (advanced) *advanced = moved;
    return MIS_OK;
}

int mis_session_poll(mis_session* S, int32_t wait, mis_done* done, int32_t cap, int32_t* n_done) {
    if (!S || !n_done || cap < 0 || (cap > 0 && !done)) return sfail(MIS_EINVAL, "bad argument");
    *n_done = 0;
    for (;;) {
        int32_t moved = 0;
        TC_CHECK(session_pass(S, false, true, done, cap, n_done, &moved));
        if (!wait || *n_done > 0 || *n_done >= cap || !any_in(S, Phase::Output)) break;
        if (!moved) std::this_thread::yield();
    }
    return MIS_OK;
}

int mis_session_progress(mis_session* S, int32_t wait, mis_done* done, int32_t cap, int32_t* n_done) {
    if (!S || !n_done || cap < 0 || (cap > 0 && !done)) return sfail(MIS_EINVAL, "bad argument");
    *n_done = 0;
    for (;;) {
        int32_t moved = 0;
        TC_CHECK(session_pass(S, true, true, done, cap, n_done, &moved));
        if (!wait || *n_done > 0 || S->live == 0 || *n_done >= cap) break;
        if (!moved) std::this_thread::yield();
    }
    return MIS_OK;
}

int mis_session_query(const mis_session* S, int32_t* live, size_t* bytes_in_use, size_t* largest_free) {
    if (!S) return sfail(MIS_EINVAL, "session is null");
    if (live) *live = S->live;
    if (bytes_in_use) *bytes_in_use = S->arena.used();
    if (largest_free) *largest_free = S->arena.largest_free();
    return MIS_OK;
}

void mis_session_destroy(mis_session* S) {
    if (!S) return;
    for (Slot& sl : S->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.g) mis_free_tiles(sl.g);
        if (sl.ev) (void)hipEventDestroy(sl.ev);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    if (S->h_ctrl) (void)hipHostFree(S->h_ctrl);
    delete S;
}

}  // extern "C"
