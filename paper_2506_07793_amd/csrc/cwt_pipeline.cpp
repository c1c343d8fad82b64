// cwt_execute_batches: many batches of C channels with one plan.
//
// Plans with a register-resident transform kernel run one launch per batch
// on the caller's stream: the transform of batch i and the forward FFT of
// batch i + 1 share the launch (launch_fused_reg), the forward writing the
// other half of a double-buffered workspace.  Stream order alone separates
// a half's writer from its reader, so there are no events and no second
// stream.  Other plans run forward then transform per batch.
#include <hip/hip_runtime.h>

#include "cwt_internal.hpp"

using namespace cwtk;
using namespace cwtrt;

namespace {

FwdParams forward_params(const cwt_plan &P, const float *x, int64_t C, void *ws)
{
    FwdParams fp{};
    fp.x = x;
    fp.C = (int)C;
    fp.N = (int)P.n;
    fp.x_stride = P.n;
    fp.Xh = reinterpret_cast<float2 *>(ws);
    fp.Lh = P.L / 2 + 1;
    fp.tw = P.d_tw;
    fp.rp = P.rp;
    return fp;
}

MainParams transform_params(const cwt_plan &P, int64_t C, void *out, void *ws)
{
    MainParams mp{};
    mp.Xh = reinterpret_cast<const float2 *>(ws);
    mp.Lh = P.L / 2 + 1;
    mp.H = P.d_H;
    mp.Hc = P.d_Hc;
    mp.band = P.d_band;
    mp.tw = P.d_tw;
    mp.out = out;
    mp.out_mode = P.opts.out;
    mp.N = (int)P.n;
    mp.F = P.F;
    mp.C = (int)C;
    mp.n_rows = (P.opts.out == CWT_OUT_BANDPOWER_F32) ? P.n_bands : P.F;
    mp.grp_freq = P.d_grp_freq;
    mp.grp_off = P.d_grp_off;
    mp.rp = P.rp;
    mp.variant = P.variant;
    return mp;
}

}  // namespace

extern "C" size_t cwt_batches_workspace_size(const cwt_plan *P, int64_t C)
{
    return 2 * cwt_workspace_size(P, C);
}

extern "C" int cwt_execute_batches(const cwt_plan *P, const float *x, int64_t x_batch_stride,
                                   int32_t n_batches, int64_t C, void *out,
                                   int64_t out_batch_stride, void *ws, size_t ws_bytes,
                                   void *stream)
{
    clear_error();
    if (!P) return fail(CWT_E_INVALID, "cwt_execute_batches: plan is NULL");
    if (P->n_seg)
        return fail(CWT_E_UNSUPPORTED,
                    "segmented plans (padded length above %d) run through cwt_execute",
                    CWT_MAX_LEN);
    if (n_batches < 0) return fail(CWT_E_INVALID, "n_batches %d < 0", (int)n_batches);
    if (x_batch_stride < 0 || out_batch_stride < 0)
        return fail(CWT_E_INVALID, "negative batch stride");
    if ((out_batch_stride & 7) != 0)
        return fail(CWT_E_INVALID, "out_batch_stride %lld is not a multiple of 8 bytes",
                    (long long)out_batch_stride);
    const size_t half = cwt_workspace_size(P, C);
    if (C > 0 && ws_bytes < 2 * half)
        return fail(CWT_E_INVALID, "workspace too small: %zu < %zu bytes", ws_bytes, 2 * half);
    int rc = check_exec_args(P, x, true, C, out, true, ws, half);
    if (rc != CWT_OK || C == 0 || n_batches == 0) return rc;

    hipStream_t s = (hipStream_t)stream;
    char *ws_half[2] = {static_cast<char *>(ws), static_cast<char *>(ws) + half};
    auto xb = [&](int32_t i) { return x + (int64_t)i * x_batch_stride; };
    auto ob = [&](int32_t i) { return static_cast<char *>(out) + (int64_t)i * out_batch_stride; };

    if (P->opts.precision != CWT_PREC_FP32 || !P->use_fixed) {
        for (int32_t i = 0; i < n_batches; ++i) {
            rc = (P->opts.precision != CWT_PREC_FP32)
                     ? enqueue_execute_split(*P, xb(i), C, P->n, ob(i), ws_half[i & 1], s)
                     : enqueue_execute(*P, xb(i), C, P->n, ob(i), ws_half[i & 1], s);
            if (rc != CWT_OK) return rc;
        }
        return CWT_OK;
    }
    rc = enqueue_forward(*P, xb(0), C, P->n, ws_half[0], s);
    if (rc != CWT_OK) return rc;
    for (int32_t i = 0; i < n_batches; ++i) {
        const MainParams mp = transform_params(*P, C, ob(i), ws_half[i & 1]);
        if (i + 1 < n_batches) {
            const FwdParams fp = forward_params(*P, xb(i + 1), C, ws_half[(i + 1) & 1]);
            hipError_t e = launch_fused_reg(mp, fp, s, next_launch_events(*P));
            if (e != hipSuccess) return hip_fail(e, "fused transform + forward launch");
        } else {
            rc = enqueue_transform(*P, C, ob(i), ws_half[i & 1], s);
            if (rc != CWT_OK) return rc;
        }
    }
    return CWT_OK;
}
