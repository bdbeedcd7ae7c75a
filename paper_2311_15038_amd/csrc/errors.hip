// Error reporting and device-property cache for the C ABI.
#include <atomic>
#include <cstring>

#include "common.h"

namespace vr {

namespace {
thread_local char g_msg[512] = {0};

constexpr int kMaxDevices = 64;
std::atomic<int> g_cus[kMaxDevices];
}  // namespace

int fail(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_msg, sizeof(g_msg), fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { g_msg[0] = 0; }

int check_launch(const char* what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(VR_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
    return VR_OK;
}

int num_cus()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return 256;
    if (dev < kMaxDevices) {
        int c = g_cus[dev].load(std::memory_order_relaxed);
        if (c > 0) return c;
    }
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
        n = 256;
    if (dev < kMaxDevices) g_cus[dev].store(n, std::memory_order_relaxed);
    return n;
}

}  // namespace vr

extern "C" const char* vr_last_error(void) { return vr::g_msg; }

extern "C" const char* vr_version(void) { return "vr 0.1 gfx950"; }
