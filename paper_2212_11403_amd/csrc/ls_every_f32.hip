// The keep-alpha forward sweep of the gradient's segment recompute:
// FP32, over the gradient's slot menu.
#include "ls_grad_kernel.h"

namespace lsk {

template <int NSLOT>
static hipError_t launch_every_one(const SweepPtrs &p, const SweepArgs &a, int nwaves,
                                   hipStream_t st) {
    using PT = PrecF32;
    const int vps = sweep_slot_vgprs(PT::vgpr_per_slot, p.prior != nullptr);
    if (nwaves < 1 || nwaves > max_waves_for(NSLOT, vps, p.prior != nullptr))
        return hipErrorInvalidValue;
    if (a.nblk < 1 || a.r0 < 0 || a.r0 + a.nblk > a.R) return hipErrorInvalidValue;
    if (p.emis && p.prior)
        hipLaunchKernelGGL((sweep_kernel<PT, NSLOT, 0, true, true, true>), dim3(a.nblk),
                           dim3(64 * nwaves), 0, st, p.Hr, (const typename PT::T *)p.emis,
                           p.lu_prefix, p.prior, p.rho, p.coef, p.recipients,
                           (typename PT::ST *)p.state, p.log_scale, p.status,
                           (typename PT::IO *)p.snap, a);
    else if (p.prior)
        hipLaunchKernelGGL((sweep_kernel<PT, NSLOT, 0, true, false, true>), dim3(a.nblk),
                           dim3(64 * nwaves), 0, st, p.Hr, nullptr, nullptr, p.prior, p.rho,
                           p.coef, p.recipients, (typename PT::ST *)p.state, p.log_scale,
                           p.status, (typename PT::IO *)p.snap, a);
    else if (p.emis)
        hipLaunchKernelGGL((sweep_kernel<PT, NSLOT, 0, true, true>), dim3(a.nblk),
                           dim3(64 * nwaves), 0, st, p.Hr, (const typename PT::T *)p.emis,
                           p.lu_prefix, nullptr, p.rho, p.coef, p.recipients, (typename PT::ST *)p.state,
                           p.log_scale, p.status, (typename PT::IO *)p.snap, a);
    else
        hipLaunchKernelGGL((sweep_kernel<PT, NSLOT, 0, true>), dim3(a.nblk), dim3(64 * nwaves), 0,
                           st, p.Hr, nullptr, nullptr, nullptr, p.rho, p.coef, p.recipients,
                           (typename PT::ST *)p.state, p.log_scale, p.status,
                           (typename PT::IO *)p.snap, a);
    return hipGetLastError();
}

hipError_t launch_every_f32(const SweepPtrs &p, const SweepArgs &a, Shape sh, hipStream_t st) {
    switch (sh.nslot) {
#define LS_CASE(n) \
    case n:        \
        return launch_every_one<n>(p, a, sh.nwaves, st);
        LS_MENU_GRAD(LS_CASE)
#undef LS_CASE
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace lsk
