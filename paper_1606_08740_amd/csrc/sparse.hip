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

// The block's substitutions L y = r (unit diagonal) and U z = y on its
// values in LDS, level by level, walking the CSR arrays: row i of a level
// reads its entries through rowptr, dpos, col and lu.
template <int TPB>
__device__ inline void substitute_csr(const CsrDev &c, double *w, int t, int tid, int64_t lo, int64_t hi)
{
#pragma clang fp contract(off)
    for (int lv = c.blev_l[t]; lv < c.blev_l[t + 1]; ++lv) {
        for (int q = c.lptr[lv] + tid; q < c.lptr[lv + 1]; q += TPB) {
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
    for (int lv = c.blev_u[t]; lv < c.blev_u[t + 1]; ++lv) {
        for (int q = c.uptr[lv] + tid; q < c.uptr[lv + 1]; q += TPB) {
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
}

// One packed record: block-local row and KP (column, value) slots.
template <int KP> struct PackedRow {
    int row;
    int col[KP];
    double val[KP];
};

template <int KP>
__device__ __attribute__((always_inline)) inline void load_packed(const int16_t *rows, const int16_t *cols, const double *vals, int q, bool ok,
                                   PackedRow<KP> &r)
{
    r.row = -1;
    if (ok) {
        r.row = rows[q];
#pragma unroll
        for (int s = 0; s < KP; ++s) {
            r.col[s] = cols[(int64_t)q * KP + s];
            r.val[s] = vals[(int64_t)q * KP + s];
        }
    }
}

// One triangular sweep over packed records, level by level.  A thread's
// records for its first row of level lv are loaded D levels ahead into a
// register ring (they do not depend on the values being computed), and the
// level bounds come from LDS when they fit, so no level waits on a global
// load once the ring is deep enough; what remains per level is its chain of
// LDS reads, dependent FP64 updates and the LDS write.  Deeper rings hold
// more registers; the driver picks D per matrix by timing.
// UPPER: divide by u_ii (diag) after the subtractions.

// ptr[lv - pbase] is the first record of level lv.
template <int KP, bool UPPER>
__device__ __attribute__((always_inline)) inline void fetch_packed(const int16_t *rows, const int16_t *cols, const double *vals, const double *diag,
                                    const int32_t *ptr, int pbase, int lv, int l1, int tid, PackedRow<KP> &r,
                                    double &d)
{
    r.row = -1;
    if (lv < l1) {
        const int q = ptr[lv - pbase] + tid;
        if (q < ptr[lv + 1 - pbase]) {
            load_packed<KP>(rows, cols, vals, q, true, r);
            if (UPPER)
                d = diag[q];
        }
    }
}

template <int KP, bool UPPER, int D, int TPB>
__device__ __attribute__((always_inline)) inline void sweep_packed(const int16_t *rows, const int16_t *cols, const double *vals, const double *diag,
                                    const int32_t *ptr, int pbase, int l0, int l1, double *w, int tid)
{
#pragma clang fp contract(off)
    PackedRow<KP> ring[D];
    double dg[D];
#pragma unroll
    for (int u = 0; u < D; ++u) {
        dg[u] = 1.0;
        fetch_packed<KP, UPPER>(rows, cols, vals, diag, ptr, pbase, l0 + u, l1, tid, ring[u], dg[u]);
    }
    for (int lv = l0; lv < l1; lv += D) {
#pragma unroll
        for (int u = 0; u < D; ++u) {
            const int l = lv + u;
            if (l >= l1)
                break;   // uniform
            const PackedRow<KP> &cur = ring[u];
            if (cur.row >= 0) {
                double v = w[cur.row];
#pragma unroll
                for (int s = 0; s < KP; ++s)
                    if (cur.col[s] >= 0)
                        v -= cur.val[s] * w[cur.col[s]];
                w[cur.row] = UPPER ? v / dg[u] : v;
            }
            // rows of the level beyond the first TPB (loaded as needed)
            for (int q = ptr[l - pbase] + tid + TPB; q < ptr[l + 1 - pbase]; q += TPB) {
                PackedRow<KP> r;
                load_packed<KP>(rows, cols, vals, q, true, r);
                double v = w[r.row];
#pragma unroll
                for (int s = 0; s < KP; ++s)
                    if (r.col[s] >= 0)
                        v -= r.val[s] * w[r.col[s]];
                w[r.row] = UPPER ? v / diag[q] : v;
            }
            __syncthreads();
            fetch_packed<KP, UPPER>(rows, cols, vals, diag, ptr, pbase, l + D, l1, tid, ring[u], dg[u]);
        }
    }
}

// Both substitutions of block t.  The block's level bounds are staged in
// LDS after its values (lev, sized by the driver) when they fit; otherwise
// they are read from global memory.
template <int KP, int D, int TPB>
__device__ __attribute__((always_inline)) inline void substitute_packed(const CsrDev &c, double *w, int32_t *lev, int t, int tid)
{
    const int l0 = c.blev_l[t], l1 = c.blev_l[t + 1];
    const int u0 = c.blev_u[t], u1 = c.blev_u[t + 1];
    // level lv's bound is ptr[lv - base]; no pointer is ever formed outside
    // its array.  The two branches keep each pointer's memory (LDS or
    // global) known to the compiler: a pointer that may be either becomes a
    // flat access, whose completion is counted with the record loads in
    // flight and would wait for them.
    if (lev) {
        const int nl = l1 - l0 + 1, nu = u1 - u0 + 1;
        for (int v = tid; v < nl; v += TPB)
            lev[v] = c.lptr[l0 + v];
        for (int v = tid; v < nu; v += TPB)
            lev[nl + v] = c.uptr[u0 + v];
        __syncthreads();
        sweep_packed<KP, false, D, TPB>(c.frow, c.fcol, c.fval, nullptr, lev, l0, l0, l1, w, tid);
        sweep_packed<KP, true, D, TPB>(c.brow, c.bcol, c.bval, c.bdiag, lev + nl, u0, u0, u1, w, tid);
    } else {
        sweep_packed<KP, false, D, TPB>(c.frow, c.fcol, c.fval, nullptr, c.lptr, 0, l0, l1, w, tid);
        sweep_packed<KP, true, D, TPB>(c.brow, c.bcol, c.bval, c.bdiag, c.uptr, 0, u0, u1, w, tid);
    }
}

// TPB threads per workgroup: 256, or 64 (one wave) for block ILU(0) with
// many small blocks (launch_one gives the rule).
template <int MODE, bool ILU, int TPB> __global__ __launch_bounds__(TPB) void k_csr(const CsrArgs a)
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
    for (int64_t i = lo + tid; i < hi; i += TPB) {
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
        int32_t *lev = c.lev_lds ? reinterpret_cast<int32_t *>(w + c.max_block_rows) : nullptr;
        if (c.kp == 4 && c.depth == 1) {
            substitute_packed<4, 1, TPB>(c, w, lev, t, tid);
        } else if (c.kp == 4 && c.depth == 2) {
            substitute_packed<4, 2, TPB>(c, w, lev, t, tid);
        } else if (c.kp == 4) {
            substitute_packed<4, 4, TPB>(c, w, lev, t, tid);
        } else if (c.kp == 8 && c.depth == 1) {
            substitute_packed<8, 1, TPB>(c, w, lev, t, tid);
        } else if (c.kp == 8) {
            substitute_packed<8, 2, TPB>(c, w, lev, t, tid);
        } else {
            substitute_csr<TPB>(c, w, t, tid, lo, hi);
        }
        for (int64_t i = lo + tid; i < hi; i += TPB) {
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
            for (int v = 0; v < TPB / kTX; ++v)
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

// Block ILU(0) passes are latency chains (one level after another), so the
// time of a pass is set by how many blocks run at once: with many small
// blocks (2048 or more, eight or more per CU) one-wave workgroups all stay
// resident and win (1024-row blocks of a 128^3 seven-point matrix: 315
// against 489 us); with fewer, larger blocks 256 threads win (2048-row
// blocks: 299 against 365 us).
constexpr int kIluSmallBlocks = 2048;

template <int MODE, bool ILU, int TPB> hipError_t launch_tpb(const CsrArgs &a, size_t lds, hipStream_t s)
{
    hipLaunchKernelGGL((k_csr<MODE, ILU, TPB>), dim3(a.c.nblocks), dim3(kTX, TPB / kTX), ILU ? lds : 0, s, a);
    return hipGetLastError();
}

template <int MODE, bool ILU> hipError_t launch_one(const CsrArgs &a, size_t lds, hipStream_t s)
{
    if (ILU && a.c.nblocks >= kIluSmallBlocks)
        return launch_tpb<MODE, ILU, kTX>(a, lds, s);
    return launch_tpb<MODE, ILU, kThreads>(a, lds, s);
}

template <int MODE> hipError_t allow_lds()
{
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_csr<MODE, true, kThreads>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kCsrMaxLds);
    if (e != hipSuccess)
        return e;
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_csr<MODE, true, kTX>),
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
    const size_t lds = csr_lds_bytes(a.c);
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

namespace {
__global__ void k_pack_factors(const CsrDev c, const int32_t *fe, const int32_t *be, double *fval, double *bval,
                               double *bdiag)
{
    const int64_t slots = (int64_t)c.n * c.kp;
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < slots; s += (int64_t)gridDim.x * blockDim.x) {
        fval[s] = fe[s] >= 0 ? c.lu[fe[s]] : 0.0;
        bval[s] = be[s] >= 0 ? c.lu[be[s]] : 0.0;
        if (s < c.n)
            bdiag[s] = c.lu[c.dpos[c.urows[s]]];
    }
}
}  // namespace

hipError_t launch_pack_factors(const CsrDev &c, const int32_t *fe, const int32_t *be, double *fval, double *bval,
                               double *bdiag, hipStream_t s)
{
    hipLaunchKernelGGL(k_pack_factors, dim3(1024), dim3(256), 0, s, c, fe, be, fval, bval, bdiag);
    return hipGetLastError();
}

hipError_t launch_ilu0(const CsrDev &c, int *bad, hipStream_t s)
{
    hipLaunchKernelGGL(k_ilu0, dim3(c.nblocks), dim3(kTX, kWY), 0, s, c, bad);
    return hipGetLastError();
}

}  // namespace aar
