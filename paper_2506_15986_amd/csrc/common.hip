// Error text, version and device facts for libann.
#include "common.h"

#include <cstring>
#include <mutex>

namespace ann {

// The persistent kernels take work from a counter that must start at zero.
// One kernel in one translation unit: every code object of the library must
// export distinct kernel symbols.
__global__ void ann_work_counter_reset(uint32_t *c) { *c = 0u; }

ann_status reset_work_counter(uint32_t *c, hipStream_t st)
{
    hipLaunchKernelGGL(ann_work_counter_reset, dim3(1), dim3(1), 0, st, c);
    ANN_LAUNCHED();
    return ANN_OK;
}

static thread_local char g_err[512] = "";

ann_status fail(ann_status s, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return s;
}

int device_cus()
{
    static int cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cache[dev] == 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
            cus = 256;
        cache[dev] = cus;
    }
    return cache[dev];
}

}  // namespace ann

extern "C" const char *ann_last_error(void) { return ann::g_err; }

extern "C" int32_t ann_version(void) { return 100; }
