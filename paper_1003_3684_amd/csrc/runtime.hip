// Host runtime pieces shared by every entry point: error reporting, stream
// handles, device properties and the device error word.
#include <stdarg.h>
#include <stdio.h>

#include <mutex>

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

}  // namespace sfg

extern "C" {

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
