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

// max |x| over an array; non-negative float bits order like unsigned ints
__global__ void ann_max_abs_kernel(const float *x, int64_t count, unsigned int *out)
{
    unsigned int m = 0u;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        unsigned int b = __float_as_uint(fabsf(x[i]));
        m = b > m ? b : m;
    }
    atomicMax(out, m);
}

__global__ void ann_zero_u32_kernel(unsigned int *p) { *p = 0u; }

static thread_local char g_err[512] = "";

ann_status fail(ann_status s, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return s;
}

int device_lds_bytes()
{
    static int cache[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 65536;
    if (cache[dev] == 0) {
        int b = 0;
        if (hipDeviceGetAttribute(&b, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
                hipSuccess ||
            b <= 0)
            b = 65536;
        cache[dev] = b;
    }
    return cache[dev];
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

extern "C" ann_status ann_max_abs(const float *x, int64_t count, float *result, void *workspace,
                                  size_t ws_bytes, void *stream)
{
    ANN_REQUIRE(x && result && workspace, "a required pointer is NULL");
    ANN_REQUIRE(count >= 1, "count must be >= 1");
    ANN_REQUIRE(ws_bytes >= 4, "workspace too small");
    hipStream_t st = static_cast<hipStream_t>(stream);
    unsigned int *d = static_cast<unsigned int *>(workspace);
    hipLaunchKernelGGL(ann::ann_zero_u32_kernel, dim3(1), dim3(1), 0, st, d);
    ANN_LAUNCHED();
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(ann::ann_max_abs_kernel, dim3((unsigned)blocks), dim3(256), 0, st, x, count, d);
    ANN_LAUNCHED();
    unsigned int h = 0;
    ANN_HIP(hipMemcpyAsync(&h, d, 4, hipMemcpyDeviceToHost, st));
    ANN_HIP(hipStreamSynchronize(st));
    float f;
    memcpy(&f, &h, sizeof(f));
    *result = f;
    return ANN_OK;
}
