// Host runtime pieces shared by every entry point: error reporting, stream
// handles, device properties and the device error word.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>

#include <string.h>

#include <mutex>
#include <vector>

#include "common.hpp"

namespace sfg {

static thread_local char t_last_error[512] = "";

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(t_last_error, sizeof(t_last_error), fmt, ap);
    va_end(ap);
    return code;
}

int check_launch(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SFG_EDEVICE, "%s: %s", what, hipGetErrorString(e));
    return SFG_OK;
}

hipStream_t as_stream(void *s) { return static_cast<hipStream_t>(s); }

static constexpr int kMaxDevices = 64;

int device_cu_count() {
    static int cache[kMaxDevices] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 256;
    if (cache[dev] == 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        cache[dev] = cus;
    }
    return cache[dev];
}

// One error word per device; each device holds its own copy of the variable.
static __device__ uint32_t d_error_word;

uint32_t *device_error_word() {
    static uint32_t *addr[kMaxDevices] = {nullptr};
    static std::mutex mu;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(d_error_word)) != hipSuccess) return nullptr;
        addr[dev] = static_cast<uint32_t *>(p);
    }
    return addr[dev];
}

// ----------------------------------------------------------------- launch timing
namespace {
struct ProfRecord {
    const char *name;
    hipEvent_t start, stop;
    bool open;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRecord> g_prof;  // events are reused across resets
size_t g_prof_used = 0;
}  // namespace

// SFGEN_DEBUG_SYNC=1: synchronise after every launch and report the first
// kernel after which the device error word is set (diagnostics only).
static bool debug_sync() {
    static const bool on = [] {
        const char *e = getenv("SFGEN_DEBUG_SYNC");
        return e && e[0] == '1';
    }();
    return on;
}

// Launches recorded into a graph (stream capture) are not timed: an event
// recorded during capture belongs to the graph, not to a launch.
static bool capturing(hipStream_t s) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(s, &st) == hipSuccess && st != hipStreamCaptureStatusNone;
}

ProfScope::ProfScope(const char *name, hipStream_t s) : stream(s), kname(name) {
    std::lock_guard<std::mutex> lock(g_prof_mu);
    if (!g_prof_on || capturing(s)) return;
    if (g_prof_used == g_prof.size()) {
        ProfRecord r{nullptr, nullptr, nullptr, false};
        if (hipEventCreate(&r.start) != hipSuccess || hipEventCreate(&r.stop) != hipSuccess) return;
        g_prof.push_back(r);
    }
    slot = (int)g_prof_used++;
    g_prof[slot].name = name;
    g_prof[slot].open = true;
    (void)hipEventRecord(g_prof[slot].start, s);
}

ProfScope::~ProfScope() {
    if (debug_sync() && !capturing(stream)) {
        uint32_t v = 0;
        uint32_t *w = device_error_word();
        if (hipStreamSynchronize(stream) != hipSuccess)
            fprintf(stderr, "sfgen debug: %s: %s\n", kname, hipGetErrorString(hipGetLastError()));
        else if (w && hipMemcpy(&v, w, sizeof(v), hipMemcpyDeviceToHost) == hipSuccess && v)
            fprintf(stderr, "sfgen debug: device error word %u after %s\n", v, kname);
    }
    if (slot < 0) return;
    std::lock_guard<std::mutex> lock(g_prof_mu);
    (void)hipEventRecord(g_prof[slot].stop, stream);
    g_prof[slot].open = false;
}

}  // namespace sfg

extern "C" {

int sfg_profile_enable(int on) {
    std::lock_guard<std::mutex> lock(sfg::g_prof_mu);
    sfg::g_prof_on = on != 0;
    return SFG_OK;
}

int sfg_profile_reset(void) {
    std::lock_guard<std::mutex> lock(sfg::g_prof_mu);
    sfg::g_prof_used = 0;
    return SFG_OK;
}

int sfg_profile_query(const char *name, uint64_t *launches, double *total_ms) {
    if (!name || !launches || !total_ms) return sfg::fail(SFG_EINVAL, "sfg_profile_query: NULL argument");
    std::lock_guard<std::mutex> lock(sfg::g_prof_mu);
    uint64_t n = 0;
    double ms = 0.0;
    for (size_t i = 0; i < sfg::g_prof_used; ++i) {
        const auto &r = sfg::g_prof[i];
        if (r.open || strcmp(r.name, name) != 0) continue;
        if (hipEventSynchronize(r.stop) != hipSuccess) return sfg::check_launch("sfg_profile_query");
        float t = 0.0f;
        if (hipEventElapsedTime(&t, r.start, r.stop) != hipSuccess) return sfg::check_launch("sfg_profile_query");
        ms += t;
        ++n;
    }
    *launches = n;
    *total_ms = ms;
    return SFG_OK;
}


const char *sfg_last_error(void) { return sfg::t_last_error; }

int sfg_abi_version(void) { return 1; }

int sfg_device_error(void *stream, uint32_t *code) {
    if (!code) return sfg::fail(SFG_EINVAL, "sfg_device_error: code is NULL");
    uint32_t *w = sfg::device_error_word();
    if (!w) return sfg::fail(SFG_EDEVICE, "sfg_device_error: no device error word");
    hipStream_t s = sfg::as_stream(stream);
    uint32_t v = 0;
    if (hipStreamSynchronize(s) != hipSuccess) return sfg::check_launch("sfg_device_error: synchronize");
    if (hipMemcpy(&v, w, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess)
        return sfg::check_launch("sfg_device_error: read");
    if (v != 0) {
        const uint32_t zero = 0;
        if (hipMemcpy(w, &zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess)
            return sfg::check_launch("sfg_device_error: clear");
    }
    *code = v;
    return SFG_OK;
}

}  // extern "C"
