// Split-precision (hi + lo) DFT-as-GEMM path on MFMA.  Not built yet: plans
// asking for it are refused with CWT_E_UNSUPPORTED.
#include "cwt_internal.hpp"

namespace cwtrt {

bool split_precision_available() { return false; }
int prepare_split_precision(cwt_plan &, hipStream_t) { return CWT_E_UNSUPPORTED; }
void release_split_precision(cwt_plan &) {}
size_t split_workspace_bytes(const cwt_plan &, int64_t) { return 0; }
int enqueue_execute_split(const cwt_plan &, const float *, int64_t, int64_t, void *, void *,
                          hipStream_t)
{
    return CWT_E_UNSUPPORTED;
}
int enqueue_transform_split(const cwt_plan &, int64_t, void *, void *, hipStream_t)
{
    return CWT_E_UNSUPPORTED;
}

}  // namespace cwtrt
