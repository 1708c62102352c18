// Build + solve without any allocation, for callers that cannot allocate (code under
// graph capture, tight serving loops, harnesses that forbid it).
//
// The solver structure and the round state live in `scratch`, a file-scope device
// array of kScratchBytes.  Each GPU holds its own copy of it at its own address
// until the process ends; that address is looked up once per device with
// hipGetSymbolAddress, with the device current, and only that address is ever
// passed to kernels or copies (the array's name is a host-side stand-in in host
// code).  Every call on a GPU reuses that GPU's array: the build writes or clears
// everything a solve reads, as it does for any fresh workspace, and calls that
// overlap on one GPU (other threads, or streams without ordering between them) race
// on the array.  The round loop polls its control block with small copies into
// host stack memory instead of the pooled pinned buffers, and launches its rounds
// directly (no captured graph).
#include <mutex>

#include "graph.hpp"

namespace tcmis {
namespace {

constexpr size_t kScratchBytes = 64ull << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// this device's copy of `scratch` (looked up on the device's first call)
int scratch_on_device(char** out) {
    int dev = 0;
    TC_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device index beyond the no-allocation entry point's table");
        return MIS_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            return MIS_EHIP;
        }
        g_scratch_ptr[dev] = (char*)p;
    }
    *out = g_scratch_ptr[dev];
    return MIS_OK;
}

}  // namespace
}  // namespace tcmis

using namespace tcmis;

extern "C" {

size_t mis_noalloc_max_bytes(void) { return kScratchBytes; }

int mis_solve_noalloc(const mis_csr* csr, const mis_build_opts* opts, uint8_t* in_set, int32_t* rounds,
                      int64_t* n_in, void* stream) {
    set_error("");
    mis_build_opts o;
    TC_CHECK(resolve_opts(csr, opts, &o, 0, nullptr));
    if (csr->n > 0 && !in_set) {
        set_error("in_set is null");
        return MIS_EINVAL;
    }
    if (o.reorder == MIS_REORDER_RCM || o.timing || (o.launch != MIS_LAUNCH_AUTO && o.launch != MIS_LAUNCH_DIRECT)) {
        set_error("the no-allocation entry point takes no RCM order (host buffers), no build timing (events) "
                  "and launches rounds directly");
        return MIS_EINVAL;
    }
    o.launch = MIS_LAUNCH_DIRECT;
    mis_graph g;   // host stack: no heap allocation either
    configure_graph(&g, csr, o, 0);
    const size_t need = layout(&g, nullptr);
    if (need > kScratchBytes) {
        set_error("the graph needs " + std::to_string(need) + " bytes of solver state; the no-allocation scratch "
                  "holds " + std::to_string(kScratchBytes));
        return MIS_EINVAL;
    }
    char* ws = nullptr;
    TC_CHECK(scratch_on_device(&ws));
    hipStream_t s = (hipStream_t)stream;
    TC_CHECK(build_into(&g, csr, o, 0, nullptr, ws, need, s));
    int32_t r = 0;
    int64_t in = 0;
    if (g.n > 0) {
        TC_CHECK(solve_begin(&g, s));
        for (;;) {
            TC_CHECK(solve_rounds(&g, g.poll_rounds, false, s));
            TC_CHECK(solve_output(&g, in_set, s, true));
            Ctrl c;
            TC_HIP(hipMemcpyAsync(&c, g.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
            TC_HIP(hipStreamSynchronize(s));
            r = c.round;
            in = c.n_in;
            if (c.error) {
                set_error("a device-side check of the round kernels failed");
                return MIS_EINTERNAL;
            }
            if (c.alive == 0) break;
            if (c.round > g.n + 1) {
                set_error("round limit exceeded (equal adjacent keys?)");
                return MIS_EINTERNAL;
            }
        }
    }
    if (rounds) *rounds = r;
    if (n_in) *n_in = in;
    return MIS_OK;
}

}  // extern "C"
