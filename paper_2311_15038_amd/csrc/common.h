// Internal helpers shared by the library's translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>

#include "vr.h"

namespace vr {

// Records the message for vr_last_error() on this host thread and returns `code`.
int fail(int code, const char* fmt, ...);
// Clears the message (called at the start of every entry point).
void clear_error();
// Checks hipGetLastError() after launches; returns VR_OK or VR_ERR_HIP.
int check_launch(const char* what);

// Compute units of the current device (cached per device).
int num_cus();

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

template <typename T>
__host__ __device__ inline T ceil_div(T a, T b) { return (a + b - 1) / b; }

}  // namespace vr

#define VR_REQUIRE(cond, code, ...)              \
    do {                                         \
        if (!(cond)) return ::vr::fail((code), __VA_ARGS__); \
    } while (0)
