// Launch entry points of the stencil passes with an FP64 iterate and FP64
// history (sweep, Anderson residual, refinement residual, operator apply),
// single and batched, and the tile grid helper.  Narrow-history variants are
// in stencil_narrow.hip, FP32 iterates in stencil_f32.hip.
#include "stencil_kernels.h"

namespace aar {

void stencil_grid(int n0, int n1, int n2, const TileShape &ts, int *tx, int *ty, int *tz, int *blocks, bool paired)
{
    // paired layout: 2 lane rows per wave, 4 << (pair - 1) waves
    const int TY = (paired ? 2 * (kWY << (ts.pair - 1)) : kWY) * ts.ry;
    *tx = (n0 + kTX - 1) / kTX;
    *ty = (n1 + TY - 1) / TY;
    *tz = (n2 + ts.cz - 1) / ts.cz;
    *blocks = *tx * *ty * *tz;
}

hipError_t launch_stencil_f64(int mode, Prec hist, int radius, bool conv, const TileShape &ts,
                              StencilArgs<double> a, int *blocks_out, hipStream_t s)
{
    if (paired_layout(ts, a.st.n0, conv, mode)) {
        if (hist != Prec::F64)
            return launch_stencil_f64_narrow(mode, hist, radius, conv, ts, a, blocks_out, s);
        return mode == kSweep ? launch_paired<double, double, kSweep>(radius, a, ts, blocks_out, s)
                              : launch_paired<double, double, kFk>(radius, a, ts, blocks_out, s);
    }
    if (hist != Prec::F64 && (mode == kSweep || mode == kFk))
        return launch_stencil_f64_narrow(mode, hist, radius, conv, ts, a, blocks_out, s);
    switch (mode) {
    case kSweep:
        return launch_radius<double, double, kSweep>(radius, conv, a, ts, blocks_out, s);
    case kFk:
        return launch_radius<double, double, kFk>(radius, conv, a, ts, blocks_out, s);
    case kResid:
        return launch_radius<double, double, kResid>(radius, conv, a, ts, blocks_out, s);
    case kApply:
        return launch_radius<double, double, kApply>(radius, conv, a, ts, blocks_out, s);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_stencil_batched_f64(int mode, Prec hist, int radius, bool conv, int ry,
                                      const BatchStencilArgs<double> &a, int grid, hipStream_t s)
{
    if (hist != Prec::F64 && (mode == kSweep || mode == kFk))
        return launch_stencil_batched_f64_narrow(mode, hist, radius, conv, ry, a, grid, s);
    switch (mode) {
    case kSweep:
        return launch_batched_radius<double, double, kSweep>(radius, conv, ry, a, grid, s);
    case kFk:
        return launch_batched_radius<double, double, kFk>(radius, conv, ry, a, grid, s);
    case kResid:
        return launch_batched_radius<double, double, kResid>(radius, conv, ry, a, grid, s);
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace aar
