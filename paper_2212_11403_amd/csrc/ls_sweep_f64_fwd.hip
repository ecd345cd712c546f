// Sweep kernels for one precision and direction (see ls_sweep.h).
#include "ls_sweep.h"

namespace lsk {

template <int NSLOT>
static hipError_t launch_one(const SweepPtrs &p, const SweepArgs &a, int nwaves, hipStream_t st) {
    using PT = PrecF64;
    const int vps = sweep_slot_vgprs(PT::vgpr_per_slot, p.prior != nullptr);
    if (nwaves < 1 || nwaves > max_waves_for(NSLOT, vps, p.prior != nullptr))
        return hipErrorInvalidValue;
    if (a.nblk < 1 || a.r0 < 0 || a.r0 + a.nblk > a.R) return hipErrorInvalidValue;
    if (p.prior && p.emis)
        hipLaunchKernelGGL((sweep_kernel<PT, NSLOT, 0, false, true, true>), dim3(a.nblk),
                           dim3(64 * nwaves), 0, st, p.Hr, (const PT::T *)p.emis, p.lu_prefix,
                           p.prior, p.rho, p.coef, p.recipients, (PT::ST *)p.state, p.log_scale,
                           p.status, (PT::IO *)p.snap, a);
    else if (p.prior)
        hipLaunchKernelGGL((sweep_kernel<PT, NSLOT, 0, false, false, true>), dim3(a.nblk),
                           dim3(64 * nwaves), 0, st, p.Hr, nullptr, nullptr, p.prior, p.rho,
                           p.coef, p.recipients, (PT::ST *)p.state, p.log_scale, p.status,
                           (PT::IO *)p.snap, a);
    else if (p.emis)
        hipLaunchKernelGGL((sweep_kernel<PT, NSLOT, 0, false, true>), dim3(a.nblk),
                           dim3(64 * nwaves), 0, st, p.Hr, (const PT::T *)p.emis, p.lu_prefix, nullptr,
                           p.rho, p.coef, p.recipients, (PT::ST *)p.state, p.log_scale, p.status,
                           (PT::IO *)p.snap, a);
    else
        hipLaunchKernelGGL((sweep_kernel<PT, NSLOT, 0>), dim3(a.nblk), dim3(64 * nwaves), 0, st,
                           p.Hr, nullptr, nullptr, nullptr, p.rho, p.coef, p.recipients, (PT::ST *)p.state,
                           p.log_scale, p.status, (PT::IO *)p.snap, a);
    return hipGetLastError();
}

hipError_t launch_sweep_f64_fwd(const SweepPtrs &p, const SweepArgs &a, Shape shape, hipStream_t st) {
    switch (shape.nslot) {
#define LS_CASE(n) \
    case n:        \
        return launch_one<n>(p, a, shape.nwaves, st);
        LS_MENU_F64(LS_CASE)
#undef LS_CASE
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace lsk
