// Adjoint kernels of the gradient: FP64, narrow variant, over the slot menu.
#include "ls_grad_kernel.h"

namespace lsk {

hipError_t grad_seg_f64_narrow(const GradArgs &ga, const GradSegArgs &sa, Shape sh, hipStream_t st) {
    switch (sh.nslot) {
#define LS_CASE(n)                                                          \
    case n:                                                                 \
        return launch_grad_seg<PrecF64, n, true>(ga, sa, sh.nwaves, st);
        LS_MENU_GRAD(LS_CASE)
#undef LS_CASE
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace lsk
