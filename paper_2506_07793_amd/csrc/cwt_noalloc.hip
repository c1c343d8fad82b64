// cwt_execute_noalloc: cwt_execute for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc).  The workspace cwt_execute takes from its caller (the
// channels' half spectra between the forward FFT and the transform kernel)
// lives here in a file-scope device array instead, one copy per GPU, held
// until the process ends.
//
// Host code never passes `scratch` itself to a kernel: on the host that name
// is a stand-in, not a device address.  The first call on each device looks
// up that device's copy with hipGetSymbolAddress (with the device current)
// and keeps the address; every launch takes that address.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "../../include/cwt.h"
#include "cwt_internal.hpp"

using namespace cwtrt;

static __device__ __align__(256) unsigned char scratch[CWT_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;

struct ScratchSlot {
    std::once_flag once;
    void *ptr = nullptr;
    hipError_t err = hipSuccess;
};

ScratchSlot g_slots[kMaxDevices];

// Device address of the current device's scratch array (looked up once per
// device), or an error code with the message set.
int scratch_address(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice in cwt_execute_noalloc");
    if (dev < 0 || dev >= kMaxDevices)
        return fail(CWT_E_UNSUPPORTED, "device %d is beyond the %d devices this entry point serves",
                    dev, kMaxDevices);
    ScratchSlot &s = g_slots[dev];
    std::call_once(s.once, [&s] {
        void *p = nullptr;
        s.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (s.err == hipSuccess) s.ptr = p;
    });
    if (s.err != hipSuccess) return hip_fail(s.err, "hipGetSymbolAddress(scratch)");
    if (!s.ptr) return fail(CWT_E_HIP, "hipGetSymbolAddress(scratch) returned no address");
    *out = s.ptr;
    return CWT_OK;
}

}  // namespace

extern "C" int cwt_execute_noalloc(const cwt_plan *P, const float *x, int64_t C, void *out,
                                   void *stream)
{
    clear_error();
    if (!P) return fail(CWT_E_INVALID, "cwt_execute_noalloc: plan is NULL");
    if (P->n_seg)
        return fail(CWT_E_UNSUPPORTED,
                    "segmented plans (padded length above %d) run through cwt_execute",
                    CWT_MAX_LEN);
    if (C < 0 || C > (int64_t)1 << 24) return fail(CWT_E_INVALID, "C out of range");
    if (C == 0) return CWT_OK;
    const size_t need = cwt_workspace_size(P, C);
    if (need > (size_t)CWT_NOALLOC_SCRATCH_BYTES)
        return fail(CWT_E_UNSUPPORTED,
                    "%lld channels need %zu bytes of workspace, above the %u-byte static scratch "
                    "of cwt_execute_noalloc; split C or use cwt_execute with a workspace",
                    (long long)C, need, (unsigned)CWT_NOALLOC_SCRATCH_BYTES);
    void *ws = nullptr;
    int rc = scratch_address(&ws);
    if (rc != CWT_OK) return rc;
    rc = check_exec_args(P, x, true, C, out, true, ws, need);
    if (rc != CWT_OK) return rc;
    // Nothing in the scratch needs to start at zero: the forward stage writes
    // every half-spectrum element before the transform reads it.
    if (P->opts.precision != CWT_PREC_FP32)
        return enqueue_execute_split(*P, x, C, P->n, out, ws, (hipStream_t)stream);
    return enqueue_execute(*P, x, C, P->n, out, ws, (hipStream_t)stream);
}
