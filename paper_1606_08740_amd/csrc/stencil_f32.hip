// Launch entry points of the stencil passes with an FP32 iterate (the inner
// solves of the mixed-precision refinement), single and batched.
#include "stencil_kernels.h"

namespace aar {

hipError_t launch_stencil_f32(int mode, Prec hist, int radius, bool conv, const TileShape &ts,
                              StencilArgs<float> a, int *blocks_out, hipStream_t s)
{
    if (paired_layout(ts, a.st.n0, conv, mode)) {
        const bool bf = hist == Prec::F32_BF16;
        if (mode == kSweep)
            return bf ? launch_paired<float, bf16_t, kSweep>(radius, a, ts, blocks_out, s)
                      : launch_paired<float, float, kSweep>(radius, a, ts, blocks_out, s);
        return bf ? launch_paired<float, bf16_t, kFk>(radius, a, ts, blocks_out, s)
                  : launch_paired<float, float, kFk>(radius, a, ts, blocks_out, s);
    }
    if (mode == kSweep || mode == kFk) {
        const bool bf = hist == Prec::F32_BF16;
        if (mode == kSweep)
            return bf ? launch_radius<float, bf16_t, kSweep>(radius, conv, a, ts, blocks_out, s)
                      : launch_radius<float, float, kSweep>(radius, conv, a, ts, blocks_out, s);
        return bf ? launch_radius<float, bf16_t, kFk>(radius, conv, a, ts, blocks_out, s)
                  : launch_radius<float, float, kFk>(radius, conv, a, ts, blocks_out, s);
    }
    if (mode == kApply)
        return launch_radius<float, float, kApply>(radius, conv, a, ts, blocks_out, s);
    return hipErrorInvalidValue;
}

hipError_t launch_stencil_batched_f32(int mode, Prec hist, int radius, bool conv, int ry,
                                      const BatchStencilArgs<float> &a, int grid, hipStream_t s)
{
    const bool bf = hist == Prec::F32_BF16;
    switch (mode) {
    case kSweep:
        return bf ? launch_batched_radius<float, bf16_t, kSweep>(radius, conv, ry, a, grid, s)
                  : launch_batched_radius<float, float, kSweep>(radius, conv, ry, a, grid, s);
    case kFk:
        return bf ? launch_batched_radius<float, bf16_t, kFk>(radius, conv, ry, a, grid, s)
                  : launch_batched_radius<float, float, kFk>(radius, conv, ry, a, grid, s);
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace aar
