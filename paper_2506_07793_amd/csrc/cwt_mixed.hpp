// Register-resident kernels for padded lengths that are not powers of two,
// and the dispatch over both register-resident families.
#pragma once

#include "cwt_kernels.hpp"

namespace cwtk {

bool mixed_main_available(int L);
// Pass radices (returned count, into radix[]) and threads per workgroup of the
// register-resident transform kernel of length L, in band-power mode or not;
// 0 when L has none.
int reg_schedule(int L, bool band, int *radix, int *threads);
// Threads per workgroup of the mixed-radix kernels at length L (every mode).
int mixed_block_threads(int L);
hipError_t launch_main_mixed(const MainParams &p, hipStream_t s, LaunchEvents ev = {});
hipError_t launch_forward_mixed(const FwdParams &p, hipStream_t s);
hipError_t launch_fused_mixed(const MainParams &p, const FwdParams &f, hipStream_t s,
                              LaunchEvents ev = {});

// Either register-resident family: the power-of-two kernels (cwt_fixed.hip)
// or the mixed-radix ones, by the plan's padded length.
inline bool reg_main_available(int L) { return fixed_main_available(L) || mixed_main_available(L); }
// Work-items per output row, for the launch-size check: one transform of L / 16
// threads per row for the power-of-two kernels (as the check always counted
// them), a whole workgroup for the mixed-radix ones (an upper bound).
inline int reg_row_threads(int L)
{
    return fixed_main_available(L) ? L / 16 : mixed_block_threads(L);
}
inline hipError_t launch_main_reg(const MainParams &p, hipStream_t s, LaunchEvents ev = {})
{
    return fixed_main_available(p.rp.L) ? launch_main_fixed(p, s, ev) : launch_main_mixed(p, s, ev);
}
inline hipError_t launch_forward_reg(const FwdParams &p, hipStream_t s)
{
    return fixed_main_available(p.rp.L) ? launch_forward_fixed(p, s) : launch_forward_mixed(p, s);
}
inline hipError_t launch_fused_reg(const MainParams &p, const FwdParams &f, hipStream_t s,
                                   LaunchEvents ev = {})
{
    return fixed_main_available(p.rp.L) ? launch_fused_fixed(p, f, s, ev)
                                        : launch_fused_mixed(p, f, s, ev);
}

}  // namespace cwtk
