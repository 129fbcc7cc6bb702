// Internal helpers shared by the libann translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>

#include "../../include/ann.h"

namespace ann {

// Records the message for ann_last_error() and returns `s`.
ann_status fail(ann_status s, const char *fmt, ...);

// Enqueues a kernel that zeroes the work counter of a persistent launch.
ann_status reset_work_counter(uint32_t *c, hipStream_t st);

// Number of compute units of the current device (cached per device).
int device_cus();
int device_lds_bytes();   // LDS bytes one workgroup may allocate

// True when p is aligned to `a` bytes.
inline bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

inline size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace ann

#define ANN_HIP(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return ::ann::fail(ANN_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define ANN_REQUIRE(cond, ...)                                  \
    do {                                                        \
        if (!(cond)) return ::ann::fail(ANN_EINVAL, __VA_ARGS__); \
    } while (0)

#define ANN_SUPPORTED(cond, ...)                                  \
    do {                                                          \
        if (!(cond)) return ::ann::fail(ANN_ENOTSUP, __VA_ARGS__); \
    } while (0)

// Launch-error check right after a kernel launch.
#define ANN_LAUNCHED() ANN_HIP(hipGetLastError())
