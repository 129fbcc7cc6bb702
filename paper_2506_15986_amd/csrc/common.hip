// Error text, version and device facts for libann.
#include "common.h"

#include <cstring>
#include <mutex>

namespace ann {

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
