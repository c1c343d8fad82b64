// Device memory of the library's own objects: the caller's allocator
// callbacks when given, else HIP's stream-ordered pool allocator.  Every
// allocation and free is enqueued on a stream, and none synchronises the
// host.
#include <hip/hip_runtime.h>

#include <mutex>

#include "cwt_internal.hpp"

namespace cwtrt {

namespace {

// Whether the device supports stream-ordered pool allocation (looked up once
// per device).  Devices without it get hipMalloc, and their frees wait for
// the stream first (the only way a plain hipFree can be ordered after the
// work that used the block).
constexpr int kMaxDev = 64;
std::once_flag g_pool_once[kMaxDev];
bool g_pool_ok[kMaxDev];

bool pools_supported()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) return false;
    std::call_once(g_pool_once[dev], [dev] {
        int v = 0;
        g_pool_ok[dev] = hipDeviceGetAttribute(&v, hipDeviceAttributeMemoryPoolsSupported, dev) ==
                             hipSuccess &&
                         v != 0;
    });
    return g_pool_ok[dev];
}

}  // namespace

int check_dev_mem(const DevMem &m)
{
    if ((m.alloc == nullptr) != (m.free == nullptr))
        return fail(CWT_E_INVALID, "alloc and free must be given together");
    return CWT_OK;
}

int dev_alloc(const DevMem &m, void **p, size_t bytes, hipStream_t s, const char *what)
{
    *p = nullptr;
    const size_t n = bytes < 256 ? 256 : bytes;
    if (m.alloc) {
        *p = m.alloc(n, (void *)s, m.ctx);
        if (!*p) return fail(CWT_E_NOMEM, "allocator returned NULL for %s (%zu bytes)", what, n);
        return CWT_OK;
    }
    hipError_t e = pools_supported() ? hipMallocAsync(p, n, s) : hipMalloc(p, n);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(CWT_E_NOMEM, "device allocation of %s (%zu bytes) failed: %s", what, n,
                    hipGetErrorName(e));
    }
    return CWT_OK;
}

void dev_free(const DevMem &m, void *p, size_t bytes, hipStream_t s)
{
    if (!p) return;
    const size_t n = bytes < 256 ? 256 : bytes;
    if (m.free) {
        m.free(p, n, (void *)s, m.ctx);
    } else if (pools_supported()) {
        (void)hipFreeAsync(p, s);
    } else {
        (void)hipStreamSynchronize(s);
        (void)hipFree(p);
    }
}

int plan_alloc(cwt_plan &P, void **p, size_t bytes, hipStream_t s, const char *what)
{
    int rc = dev_alloc(P.mem, p, bytes, s, what);
    if (rc != CWT_OK) return rc;
    P.blocks.push_back({*p, bytes < 256 ? 256 : bytes});  // the size asked of the allocator
    return CWT_OK;
}

void plan_free_all(cwt_plan &P, hipStream_t s)
{
    for (const auto &b : P.blocks) dev_free(P.mem, b.p, b.n, s);
    P.blocks.clear();
}

}  // namespace cwtrt
