// Launch entry points of the temporal blocks of Richardson steps (residual
// recursion, one-point tiles), FP64 and FP32 iterates with a ring of the same
// type.
#include "tblock_kernels.h"

namespace aar {

namespace {

constexpr size_t kLdsLimit = 160 * 1024;

template <typename T, int R, bool CONV, int TY>
hipError_t launch_tb_one(StencilArgs<T> a, const TileShape &ts, int j0, int nt, bool last_fk, hipStream_t s)
{
    const size_t bytes = tblock_lds_bytes(R, nt, TY, sizeof(T));
    if (bytes + 256 > kLdsLimit)
        return hipErrorInvalidValue;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_tblock<T, R, CONV, TY>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)(kLdsLimit - 256));
        if (e != hipSuccess)
            return e;
        attr_set = true;
    }
    int tx, ty, tz, blocks;
    stencil_grid(a.st.n0, a.st.n1, a.st.n2, ts, &tx, &ty, &tz, &blocks);
    a.tiles_x = tx;
    a.tiles_y = ty;
    a.tiles_z = tz;
    a.cz = ts.cz;
    a.order = ts.order;
    a.j = j0;
    hipLaunchKernelGGL((k_tblock<T, R, CONV, TY>), dim3(blocks), dim3(kTX, kWY), bytes, s, a, nt, last_fk ? 1 : 0);
    return hipGetLastError();
}

template <typename T, int R, bool CONV>
hipError_t launch_tb_ty(StencilArgs<T> a, const TileShape &ts, int j0, int nt, bool last_fk, hipStream_t s)
{
    switch (ts.ry) {
    case 1:
        return launch_tb_one<T, R, CONV, kWY>(a, ts, j0, nt, last_fk, s);
    case 2:
        return launch_tb_one<T, R, CONV, 2 * kWY>(a, ts, j0, nt, last_fk, s);
    case 4:
        return launch_tb_one<T, R, CONV, 4 * kWY>(a, ts, j0, nt, last_fk, s);
    default:
        return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_tb(int radius, bool conv, const TileShape &ts, StencilArgs<T> a, int j0, int nt, bool last_fk,
                     hipStream_t s)
{
    if (nt < 1 || nt > kTbMaxStages || j0 < 1 || ts.pair != 0)
        return hipErrorInvalidValue;
    if (conv)
        return radius == 1 ? launch_tb_ty<T, 1, true>(a, ts, j0, nt, last_fk, s) : hipErrorInvalidValue;
    switch (radius) {
    case 1:
        return launch_tb_ty<T, 1, false>(a, ts, j0, nt, last_fk, s);
    case 2:
        return launch_tb_ty<T, 2, false>(a, ts, j0, nt, last_fk, s);
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace

bool tblock_fits(int radius, bool conv, const TileShape &ts, int nt, bool f64)
{
    if (nt < 1 || nt > kTbMaxStages || ts.pair != 0 || radius > 2 || (conv && radius != 1))
        return false;
    if (ts.ry != 1 && ts.ry != 2 && ts.ry != 4)
        return false;
    return tblock_lds_bytes(radius, nt, kWY * ts.ry, f64 ? 8 : 4) + 256 <= kLdsLimit;
}

hipError_t launch_tblock_f64(int radius, bool conv, const TileShape &ts, StencilArgs<double> a, int j0, int nt,
                             bool last_fk, hipStream_t s)
{
    return launch_tb<double>(radius, conv, ts, a, j0, nt, last_fk, s);
}

hipError_t launch_tblock_f32(int radius, bool conv, const TileShape &ts, StencilArgs<float> a, int j0, int nt,
                             bool last_fk, hipStream_t s)
{
    return launch_tb<float>(radius, conv, ts, a, j0, nt, last_fk, s);
}

}  // namespace aar
