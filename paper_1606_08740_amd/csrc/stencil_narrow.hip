// Launch entry points of the sweep and Anderson-residual passes with an FP64
// iterate and an FP32 or bfloat16 history ring, single and batched.
#include "stencil_kernels.h"

namespace aar {

hipError_t launch_stencil_f64_narrow(int mode, Prec hist, int radius, bool conv, const TileShape &ts,
                                     StencilArgs<double> a, int *blocks_out, hipStream_t s)
{
    if (mode != kSweep && mode != kFk)
        return hipErrorInvalidValue;
    if (paired_layout(ts, a.st.n0, conv, mode)) {
        if (hist == Prec::F32)
            return mode == kSweep ? launch_paired<double, float, kSweep>(radius, a, ts, blocks_out, s)
                                  : launch_paired<double, float, kFk>(radius, a, ts, blocks_out, s);
        if (hist == Prec::F32_BF16)
            return mode == kSweep ? launch_paired<double, bf16_t, kSweep>(radius, a, ts, blocks_out, s)
                                  : launch_paired<double, bf16_t, kFk>(radius, a, ts, blocks_out, s);
        return hipErrorInvalidValue;
    }
    if (hist == Prec::F32)
        return mode == kSweep ? launch_radius<double, float, kSweep>(radius, conv, a, ts, blocks_out, s)
                              : launch_radius<double, float, kFk>(radius, conv, a, ts, blocks_out, s);
    if (hist == Prec::F32_BF16)
        return mode == kSweep ? launch_radius<double, bf16_t, kSweep>(radius, conv, a, ts, blocks_out, s)
                              : launch_radius<double, bf16_t, kFk>(radius, conv, a, ts, blocks_out, s);
    return hipErrorInvalidValue;
}

hipError_t launch_stencil_batched_f64_narrow(int mode, Prec hist, int radius, bool conv, int ry,
                                             const BatchStencilArgs<double> &a, int grid, hipStream_t s)
{
    if (mode != kSweep && mode != kFk)
        return hipErrorInvalidValue;
    if (hist == Prec::F32)
        return mode == kSweep ? launch_batched_radius<double, float, kSweep>(radius, conv, ry, a, grid, s)
                              : launch_batched_radius<double, float, kFk>(radius, conv, ry, a, grid, s);
    if (hist == Prec::F32_BF16)
        return mode == kSweep ? launch_batched_radius<double, bf16_t, kSweep>(radius, conv, ry, a, grid, s)
                              : launch_batched_radius<double, bf16_t, kFk>(radius, conv, ry, a, grid, s);
    return hipErrorInvalidValue;
}

}  // namespace aar
