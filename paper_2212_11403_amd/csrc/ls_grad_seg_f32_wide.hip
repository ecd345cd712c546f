// Adjoint kernels of the gradient: FP32, wide variant, over the slot menu.
#include "ls_grad_kernel.h"

namespace lsk {

hipError_t grad_seg_f32_wide(const GradArgs &ga, const GradSegArgs &sa, Shape sh, hipStream_t st) {
    switch (sh.nslot) {
#define LS_CASE(n)                                                          \
    case n:                                                                 \
        if constexpr (grad_wide_needed<PrecF32, n>())                           \
            return launch_grad_seg<PrecF32, n, false>(ga, sa, sh.nwaves, st); \
        else                                                                \
            return hipErrorInvalidValue;
        LS_MENU_GRAD(LS_CASE)
#undef LS_CASE
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace lsk
