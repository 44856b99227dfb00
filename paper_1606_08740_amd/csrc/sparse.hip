// General sparse A in compressed sparse rows, with the Jacobi or the
// block-Jacobi ILU(0) preconditioner (Sec. 3.1: nonsymmetric systems with
// Jacobi and ILU(0); Secs. 3.2-3.3: block Jacobi with ILU(0) on each block,
// the parallel preconditioner of the Helmholtz and Poisson runs), on gfx950.
//
// One workgroup owns one block of contiguous rows.  A Richardson sweep
// (Eq. 3 first case, Eq. 6) is one pass per block: the residual
// r = b - A x of the block's rows (the rows read x anywhere, so sweeps
// ping-pong x), then for ILU(0) the forward substitution L y = r and the
// backward substitution U z = y on the block's values held in LDS, row by
// row in level order (the rows of one level depend only on rows of earlier
// levels; the driver computes the levels once), then f = z into its history
// slot and x + omega f.  Jacobi blocks are plain row chunks: f = r / a_ii.
//
// The arithmetic follows the definitions in stored column order with no
// contraction of products into fused multiply-adds, so the product A x, the
// factors and the substitutions equal a plain sequential evaluation bit for
// bit.
#include "aar_device.h"

namespace aar {

namespace {

template <int MODE, bool ILU> __global__ __launch_bounds__(kThreads) void k_csr(const CsrArgs a)
{
#pragma clang fp contract(off)
    extern __shared__ __align__(16) double w[];
    __shared__ double red[kWY];
    const CsrDev &c = a.c;
    const int tid = threadIdx.x + kTX * threadIdx.y;
    double *f = a.out;
    if constexpr (MODE == kSweep || MODE == kFk) {
        const InstState *sp = a.state;
        if (sp->status != kRunning)
            return;
        const int64_t k = sp->cycle * a.p + a.j;
        if (k >= sp->max_iter)
            return;
        f = static_cast<double *>(a.fring) + (k % a.nslots) * a.slot_stride;
    }
    const int t = blockIdx.x;
    const int64_t lo = c.bstart[t], hi = c.bstart[t + 1];
    double acc = 0.0;

    // the block's residual (or, for the preconditioner alone, its input)
    for (int64_t i = lo + tid; i < hi; i += kThreads) {
        double r;
        if constexpr (MODE == kPrecond) {
            r = a.x[i];
        } else {
            double s = 0.0;
            for (int64_t e = c.rowptr[i]; e < c.rowptr[i + 1]; ++e)
                s += c.val[e] * a.x[c.col[e]];
            if constexpr (MODE == kApply) {
                a.out[i] = s;
                continue;
            }
            r = a.b[i] - s;
            if constexpr (MODE == kFk)
                acc += r * r;
        }
        if constexpr (ILU) {
            w[i - lo] = r;
        } else {
            const double fi = r / c.val[c.dpos[i]];
            f[i] = fi;
            if constexpr (MODE == kSweep)
                a.xout[i] = a.x[i] + a.omega * fi;
        }
    }
    if constexpr (ILU && MODE != kApply) {
        __syncthreads();
        // L y = r (unit diagonal), level by level
        for (int lv = c.blev_l[t]; lv < c.blev_l[t + 1]; ++lv) {
            for (int q = c.lptr[lv] + tid; q < c.lptr[lv + 1]; q += kThreads) {
                const int64_t i = c.lrows[q];
                double y = w[i - lo];
                for (int64_t e = c.rowptr[i]; e < c.dpos[i]; ++e) {
                    const int64_t j = c.col[e];
                    if (j >= lo)
                        y -= c.lu[e] * w[j - lo];
                }
                w[i - lo] = y;
            }
            __syncthreads();
        }
        // U z = y, level by level
        for (int lv = c.blev_u[t]; lv < c.blev_u[t + 1]; ++lv) {
            for (int q = c.uptr[lv] + tid; q < c.uptr[lv + 1]; q += kThreads) {
                const int64_t i = c.urows[q];
                const int64_t d = c.dpos[i];
                double z = w[i - lo];
                for (int64_t e = d + 1; e < c.rowptr[i + 1]; ++e) {
                    const int64_t j = c.col[e];
                    if (j >= hi)
                        break;
                    z -= c.lu[e] * w[j - lo];
                }
                w[i - lo] = z / c.lu[d];
            }
            __syncthreads();
        }
        for (int64_t i = lo + tid; i < hi; i += kThreads) {
            const double fi = w[i - lo];
            f[i] = fi;
            if constexpr (MODE == kSweep)
                a.xout[i] = a.x[i] + a.omega * fi;
        }
    }
    if constexpr (MODE == kFk) {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1)
            acc += __shfl_down(acc, o, 64);
        if (threadIdx.x == 0)
            red[threadIdx.y] = acc;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            for (int v = 0; v < kWY; ++v)
                s += red[v];
            a.partial[t] = s;
        }
    }
}

// ILU(0) of each diagonal block in place (lu holds a copy of A's values on
// entry): row by row in level order, for each k < i of row i's pattern in
// the block, l_ik = a_ik / u_kk and a_ij -= l_ik u_kj for every later j of row
// i's pattern in the block that row k's pattern holds (fill outside the
// pattern dropped).  Rows of one level are independent; row k is final
// before any row that depends on it starts.  bad[0] is set when a pivot is
// zero or not finite.
__global__ __launch_bounds__(kThreads) void k_ilu0(const CsrDev c, int *bad)
{
#pragma clang fp contract(off)
    const int tid = threadIdx.x + kTX * threadIdx.y;
    const int t = blockIdx.x;
    const int64_t lo = c.bstart[t], hi = c.bstart[t + 1];
    for (int lv = c.blev_l[t]; lv < c.blev_l[t + 1]; ++lv) {
        for (int q = c.lptr[lv] + tid; q < c.lptr[lv + 1]; q += kThreads) {
            const int64_t i = c.lrows[q];
            const int64_t end = c.rowptr[i + 1];
            for (int64_t e = c.rowptr[i]; e < c.dpos[i]; ++e) {
                const int64_t k = c.col[e];
                if (k < lo)
                    continue;
                const double lik = c.lu[e] / c.lu[c.dpos[k]];
                c.lu[e] = lik;
                // walk row k's upper part beside row i's later entries
                int64_t ek = c.dpos[k] + 1;
                const int64_t kend = c.rowptr[k + 1];
                for (int64_t e2 = e + 1; e2 < end; ++e2) {
                    const int64_t j = c.col[e2];
                    if (j >= hi)
                        break;
                    while (ek < kend && c.col[ek] < j)
                        ++ek;
                    if (ek < kend && c.col[ek] == j)
                        c.lu[e2] -= lik * c.lu[ek];
                }
            }
            const double u = c.lu[c.dpos[i]];
            if (u == 0.0 || !isfinite(u))
                bad[0] = 1;
        }
        __syncthreads();
    }
}

template <int MODE, bool ILU> hipError_t launch_one(const CsrArgs &a, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL((k_csr<MODE, ILU>), dim3(a.c.nblocks), dim3(kTX, kWY), ILU ? lds : 0, s, a);
    return hipGetLastError();
}

template <int MODE> hipError_t allow_lds()
{
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_csr<MODE, true>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)kCsrMaxLds);
}

}  // namespace

hipError_t prepare_csr_kernels()
{
    hipError_t e;
    if ((e = allow_lds<kSweep>()) != hipSuccess || (e = allow_lds<kFk>()) != hipSuccess ||
        (e = allow_lds<kPrecond>()) != hipSuccess)
        return e;
    return hipSuccess;
}

hipError_t launch_csr(int mode, const CsrArgs &a, hipStream_t s)
{
    const size_t lds = (size_t)a.c.max_block_rows * sizeof(double);
    if (a.c.ilu && lds > kCsrMaxLds)
        return hipErrorInvalidValue;
    switch (mode) {
    case kSweep:
        return a.c.ilu ? launch_one<kSweep, true>(a, lds, s) : launch_one<kSweep, false>(a, lds, s);
    case kFk:
        return a.c.ilu ? launch_one<kFk, true>(a, lds, s) : launch_one<kFk, false>(a, lds, s);
    case kApply:
        return launch_one<kApply, false>(a, 0, s);
    case kPrecond:
        return a.c.ilu ? launch_one<kPrecond, true>(a, lds, s) : launch_one<kPrecond, false>(a, lds, s);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_ilu0(const CsrDev &c, int *bad, hipStream_t s)
{
    hipLaunchKernelGGL(k_ilu0, dim3(c.nblocks), dim3(kTX, kWY), 0, s, c, bad);
    return hipGetLastError();
}

}  // namespace aar
