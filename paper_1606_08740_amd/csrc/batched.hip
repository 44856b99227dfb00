// Batched AAR: many independent systems advanced together.
//
// All running systems execute the same phase of the AAR cycle in one launch
// per phase (p-1 Richardson sweeps, the Anderson residual pass, the Gram
// products, one least-squares wave per system, the update).  The work of a
// launch is a list of items, (system, stencil tile) for the stencil passes and
// (system, chunk of kChunk points) for the streaming passes; a compaction
// kernel rebuilds the lists from the per-system masks, so converged systems
// cost nothing.  Each system keeps its own run state (convergence, iteration
// count, history window), exactly as a single solve does.  Mixed precision
// adds a per-system FP64 refinement step, taken by the systems whose inner
// FP32 solve has ended; the host replays a graph of cycles and runs the
// (device-masked) refinement pass between replays.
#include <math.h>

#include "aar_device.h"
#include "anderson_core.h"

namespace aar {

// ---------------------------------------------------------------------------
// Work-item compaction (one workgroup)
// ---------------------------------------------------------------------------
constexpr int kCompactThreads = 1024;

__device__ inline int compact_active(const CompactArgs &a, int i)
{
    if (a.mode == 0)
        return a.ctl[i].phase == kPhaseInner && a.state[i].status == kRunning;
    if (a.mode == 1)
        return a.refine[i] != 0;
    return 1;
}

__global__ __launch_bounds__(kCompactThreads) void k_compact(const CompactArgs a)
{
    __shared__ int scan_s[kCompactThreads], scan_c[kCompactThreads];
    const int tid = threadIdx.x;
    int carry_s = 0, carry_c = 0;
    for (int base = 0; base < a.count; base += kCompactThreads) {
        const int i = base + tid;
        const int act = i < a.count ? compact_active(a, i) : 0;
        const int ts = act ? a.ntiles[i] : 0;
        const int cs = act ? a.nchunks[i] : 0;
        scan_s[tid] = ts;
        scan_c[tid] = cs;
        __syncthreads();
        for (int off = 1; off < kCompactThreads; off <<= 1) {   // inclusive scan (Hillis-Steele)
            const int vs = tid >= off ? scan_s[tid - off] : 0;
            const int vc = tid >= off ? scan_c[tid - off] : 0;
            __syncthreads();
            scan_s[tid] += vs;
            scan_c[tid] += vc;
            __syncthreads();
        }
        const int es = carry_s + scan_s[tid] - ts, ec = carry_c + scan_c[tid] - cs;
        if (i < a.count) {
            a.sbase[i] = act ? es : -1;
            a.cbase[i] = act ? ec : -1;
            for (int t = 0; t < ts; ++t)
                a.sitems[es + t] = make_int2(i, t);
            for (int c = 0; c < cs; ++c)
                a.citems[ec + c] = make_int2(i, c);
        }
        carry_s += scan_s[kCompactThreads - 1];
        carry_c += scan_c[kCompactThreads - 1];
        __syncthreads();
    }
    if (tid == 0) {
        *a.nsitems = carry_s;
        *a.ncitems = carry_c;
    }
}

hipError_t launch_compact(const CompactArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_compact, dim3(1), dim3(kCompactThreads), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gram products per (system, chunk)
// ---------------------------------------------------------------------------
template <typename H, int MC>
__global__ __launch_bounds__(kThreads) void k_gram_batched(const BatchGramArgs a)
{
    constexpr int NP = MC * (MC + 1) / 2;
    constexpr int NE = NP + MC;
    constexpr int V = VecWidth<H>::value;
    __shared__ double red[kThreads / 64][NE];
    const int nitems = *a.nitems;
    for (int w = blockIdx.x; w < nitems; w += gridDim.x) {
        const int2 it = a.items[w];
        const InstState *s = a.state + it.x;
        if (s->status != kRunning)
            continue;
        const int64_t k = s->cycle * a.p + a.p - 1;
        if (k >= s->max_iter)
            continue;
        const int l = (int)(k < a.m ? k : a.m);
        const int64_t N = a.sizes[it.x];
        const H *ring = reinterpret_cast<const H *>(a.fring) + a.offs[it.x];
        const H *slot[MC + 1];
#pragma unroll
        for (int t = 0; t <= MC; ++t) {
            const int tt = t <= l ? t : l;
            slot[t] = ring + (int64_t)((k - l + tt) % a.nslots) * a.slot_stride;
        }
        double acc[NE];
#pragma unroll
        for (int e = 0; e < NE; ++e)
            acc[e] = 0.0;
        const int64_t lo = (int64_t)it.y * kChunk;
        const int64_t hi = lo + kChunk < N ? lo + kChunk : N;
        const int64_t vhi = lo + (hi - lo) / V * V;
        for (int64_t i = lo + (int64_t)threadIdx.x * V; i < vhi; i += (int64_t)blockDim.x * V) {
            double fv[MC + 1][V];
#pragma unroll
            for (int t = 0; t <= MC; ++t) {
                if (t <= l)
                    load_vec<H, V>(slot[t], i, fv[t]);
                else
#pragma unroll
                    for (int u = 0; u < V; ++u)
                        fv[t][u] = 0.0;
            }
#pragma unroll
            for (int u = 0; u < V; ++u) {
                double col[MC + 1];
#pragma unroll
                for (int t = 0; t <= MC; ++t)
                    col[t] = fv[t][u];
                gram_point<MC>(col, l, acc);
            }
        }
        for (int64_t i = vhi + threadIdx.x; i < hi; i += blockDim.x) {
            double col[MC + 1];
#pragma unroll
            for (int t = 0; t <= MC; ++t)
                col[t] = t <= l ? (double)Hist<H>::load(slot[t], i) : 0.0;
            gram_point<MC>(col, l, acc);
        }
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        wave_sums_to<NE>(acc, red[wave]);   // red[wave][e]: this wave's total of entry e
        __syncthreads();
        for (int e = threadIdx.x; e < NE; e += blockDim.x)
            a.partial[(int64_t)w * NE + e] = red[0][e] + red[1][e] + red[2][e] + red[3][e];
        __syncthreads();
    }
}

template <typename H>
static hipError_t launch_gram_batched_h(const BatchGramArgs &a, int grid, hipStream_t s)
{
    switch (a.m) {
#define AAR_GB_CASE(MC)                                                                              \
    case MC:                                                                                         \
        hipLaunchKernelGGL((k_gram_batched<H, MC>), dim3(grid), dim3(kThreads), 0, s, a);            \
        return hipGetLastError();
        AAR_GB_CASE(1)
        AAR_GB_CASE(2)
        AAR_GB_CASE(3)
        AAR_GB_CASE(4)
        AAR_GB_CASE(5)
        AAR_GB_CASE(6)
        AAR_GB_CASE(7)
        AAR_GB_CASE(8)
        AAR_GB_CASE(9)
        AAR_GB_CASE(10)
        AAR_GB_CASE(11)
        AAR_GB_CASE(12)
#undef AAR_GB_CASE
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_gram_batched(Prec prec, const BatchGramArgs &a, int grid, hipStream_t s)
{
    switch (prec) {
    case Prec::F64:
        return launch_gram_batched_h<double>(a, grid, s);
    case Prec::F32:
        return launch_gram_batched_h<float>(a, grid, s);
    case Prec::F32_BF16:
        return launch_gram_batched_h<bf16_t>(a, grid, s);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Least squares: one wave per system
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kLsqThreads) void k_lsq_batched(const LsqArgs base, const BatchLsqArgs b)
{
    __shared__ double gv[kMaxM * (kMaxM + 1) / 2 + kMaxM];
    const int i = blockIdx.x;
    InstState *st = b.state + i;
    if (st->status != kRunning)
        return;
    const int sb = b.sbase[i], cb = b.cbase[i];
    if (sb < 0 || cb < 0)
        return;   // not in the current lists (cannot happen while running)
    const int tid = threadIdx.x;
    double r = 0.0;
    for (int t = tid; t < b.ntiles[i]; t += kLsqThreads)
        r += b.rho_partial[sb + t];
    r = __shfl(wave_sum_a(r), 0, 64);
    const int ne = base.ne;
    const int nch = b.nchunks[i];
    for (int e0 = 0; e0 < ne; e0 += 32) {
        double acc[32];
#pragma unroll
        for (int j = 0; j < 32; ++j)
            acc[j] = 0.0;
        for (int c = tid; c < nch; c += kLsqThreads) {
            const double *row = b.gram_partial + (int64_t)(cb + c) * ne + e0;
#pragma unroll
            for (int j = 0; j < 32; ++j)
                if (e0 + j < ne)
                    acc[j] += row[j];
        }
#pragma unroll
        for (int j = 0; j < 32; ++j) {
            const double v = wave_sum_a(acc[j]);
            if (tid == 0 && e0 + j < ne)
                gv[e0 + j] = v;
        }
    }
    __syncthreads();
    LsqArgs a = base;
    a.state = st;
    a.log = base.log ? base.log + (int64_t)i * base.log_cap : nullptr;
    lsq_core(a, st, r, gv);
}

hipError_t launch_lsq_batched(const LsqArgs &base, const BatchLsqArgs &b, int count, hipStream_t s)
{
    hipLaunchKernelGGL(k_lsq_batched, dim3(count), dim3(kLsqThreads), 0, s, base, b);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Update per (system, chunk)
// ---------------------------------------------------------------------------
template <typename T, typename H>
__global__ __launch_bounds__(kThreads) void k_update_batched(const BatchUpdateArgs<T> a)
{
    constexpr int V = 16 / (int)sizeof(T);
    __shared__ const H *fs[kMaxSlots];
    __shared__ T al[kMaxSlots];
    using D = typename DxOf<T, H>::type;
    __shared__ const D *ds[kMaxM];
    __shared__ T de[kMaxM];
    __shared__ int nf_s, nd_s, ws_s;
    const int nitems = *a.nitems;
    for (int w = blockIdx.x; w < nitems; w += gridDim.x) {
        const int2 it = a.items[w];
        const InstState *st = a.state + it.x;
        if (st->status != kRunning)
            continue;
        const int64_t off = a.offs[it.x];
        const H *ring = reinterpret_cast<const H *>(a.fring) + off;
        if (threadIdx.x == 0) {
            nf_s = st->nf;
            nd_s = st->nd;
            ws_s = st->wslot;
        }
        if (threadIdx.x < kMaxSlots && (int)threadIdx.x < st->nf) {
            fs[threadIdx.x] = ring + (int64_t)st->fslot[threadIdx.x] * a.slot_stride;
            al[threadIdx.x] = (T)st->alpha[threadIdx.x];
        }
        if (threadIdx.x < kMaxM && (int)threadIdx.x < st->nd) {
            ds[threadIdx.x] = reinterpret_cast<const D *>(a.dxring) + off + (int64_t)st->dslot[threadIdx.x] * a.dx_stride;
            de[threadIdx.x] = (T)st->delta[threadIdx.x];
        }
        __syncthreads();
        const int nf = nf_s, nd = nd_s;
        // residual recursion: positions tr0 .. nf - 2 are the cycle's Richardson steps
        const int tr0 = a.p_rich > 0 ? nf - a.p_rich : nf;
        const int t1 = tr0 < nf - 1 ? tr0 : nf - 1;
        D *dxw = ws_s >= 0 ? reinterpret_cast<D *>(a.dxring) + off + (int64_t)ws_s * a.dx_stride : nullptr;
        const T *xin = a.xin + off;
        T *xout = a.xout + off;
        const T *fk_ptr = a.fcur ? a.fcur + off : nullptr;
        const int64_t N = a.sizes[it.x];
        const int64_t lo = (int64_t)it.y * kChunk;
        const int64_t hi = lo + kChunk < N ? lo + kChunk : N;
        const int64_t vhi = lo + (hi - lo) / V * V;
        for (int64_t i = lo + (int64_t)threadIdx.x * V; i < vhi; i += (int64_t)blockDim.x * V) {
            T d[V], dr[V];
#pragma unroll
            for (int u = 0; u < V; ++u) {
                d[u] = T(0);
                dr[u] = T(0);
            }
            for (int t = 0; t < t1; ++t) {
                const Pack<H, V> h = *reinterpret_cast<const Pack<H, V> *>(fs[t] + i);
#pragma unroll
                for (int u = 0; u < V; ++u)
                    d[u] += al[t] * (T)Hist<H>::load(h.v, u);
            }
            for (int t = t1; t < nf - 1; ++t) {
                const Pack<H, V> h = *reinterpret_cast<const Pack<H, V> *>(fs[t] + i);
#pragma unroll
                for (int u = 0; u < V; ++u) {
                    const T fv = (T)Hist<H>::load(h.v, u);
                    d[u] += al[t] * fv;
                    dr[u] += fv;
                }
            }
            T fk[V];
            if (fk_ptr) {
                const Pack<T, V> h = *reinterpret_cast<const Pack<T, V> *>(fk_ptr + i);
#pragma unroll
                for (int u = 0; u < V; ++u)
                    fk[u] = h.v[u];
            } else {
                const Pack<H, V> h = *reinterpret_cast<const Pack<H, V> *>(fs[nf - 1] + i);
#pragma unroll
                for (int u = 0; u < V; ++u)
                    fk[u] = (T)Hist<H>::load(h.v, u);
            }
#pragma unroll
            for (int u = 0; u < V; ++u)
                d[u] += al[nf - 1] * fk[u];
            for (int t = 0; t < nd; ++t) {
                const Pack<D, V> h = *reinterpret_cast<const Pack<D, V> *>(ds[t] + i);
#pragma unroll
                for (int u = 0; u < V; ++u)
                    d[u] += de[t] * (T)h.v[u];
            }
            const Pack<T, V> xc = *reinterpret_cast<const Pack<T, V> *>(xin + i);
            Pack<T, V> xn;
            Pack<D, V> dx;
#pragma unroll
            for (int u = 0; u < V; ++u) {
                const T xk = xc.v[u] + a.omega_rich * dr[u];
                xn.v[u] = xk + d[u];
                dx.v[u] = (D)(xn.v[u] - xk);
            }
            *reinterpret_cast<Pack<T, V> *>(xout + i) = xn;
            if (dxw)
                *reinterpret_cast<Pack<D, V> *>(dxw + i) = dx;
        }
        for (int64_t i = vhi + threadIdx.x; i < hi; i += blockDim.x) {
            T d = 0, dr = 0;
            for (int t = 0; t < nf - 1; ++t) {
                const T fv = (T)Hist<H>::load(fs[t], i);
                d += al[t] * fv;
                if (t >= t1)
                    dr += fv;
            }
            const T fk = fk_ptr ? fk_ptr[i] : (T)Hist<H>::load(fs[nf - 1], i);
            d += al[nf - 1] * fk;
            for (int t = 0; t < nd; ++t)
                d += de[t] * (T)ds[t][i];
            const T xk = xin[i] + a.omega_rich * dr;
            const T xn = xk + d;
            xout[i] = xn;
            if (dxw)
                dxw[i] = (D)(xn - xk);
        }
        __syncthreads();
    }
}

hipError_t launch_update_batched(Prec prec, const BatchUpdateArgs<double> *a64, const BatchUpdateArgs<float> *a32,
                                 int grid, hipStream_t s)
{
    if (a64) {   // FP64 iterate; the history is FP64, FP32 or bfloat16
        switch (prec) {
        case Prec::F64:
            hipLaunchKernelGGL((k_update_batched<double, double>), dim3(grid), dim3(kThreads), 0, s, *a64);
            break;
        case Prec::F32:
            hipLaunchKernelGGL((k_update_batched<double, float>), dim3(grid), dim3(kThreads), 0, s, *a64);
            break;
        case Prec::F32_BF16:
            hipLaunchKernelGGL((k_update_batched<double, bf16_t>), dim3(grid), dim3(kThreads), 0, s, *a64);
            break;
        }
        return hipGetLastError();
    }
    switch (prec) {
    case Prec::F64:
        return hipErrorInvalidValue;
    case Prec::F32:
        hipLaunchKernelGGL((k_update_batched<float, float>), dim3(grid), dim3(kThreads), 0, s, *a32);
        break;
    case Prec::F32_BF16:
        hipLaunchKernelGGL((k_update_batched<float, bf16_t>), dim3(grid), dim3(kThreads), 0, s, *a32);
        break;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Per-system control: starting runs, refinement, results
// ---------------------------------------------------------------------------
// Where the last iterate of a finished run sits: 0 = xa, 1 = xb.
__device__ inline int final_buffer(const InstState &st, int p)
{
    if (st.status == kConverged || st.status == kStagnated || st.status == kBreakdown)
        return ((p - 1) & 1) ? 1 : 0;
    const int64_t done = st.max_iter;
    const int64_t j = (done - 1) % p;
    if (j == p - 1)
        return 0;
    return ((j + 1) & 1) ? 1 : 0;
}

// Streaming pass over (system, chunk) items.  op:
//   kOpGather   x_packed[i] = src_user[uoff + i]            (FP64 in)
//   kOpScatter  dst_user[uoff + i] = x_packed[i]            (FP64 out)
//   kOpNorm     partial = sum v^2                            (v FP64)
//   kOpSum      partial = sum v                              (v FP64)
//   kOpCorrect  x64 += rnorm * d32 (d from xa32/xb32 by dsel; with the
//               residual recursion xa32 + omega * the unfinished cycle's f)
//   kOpScatterSel / kOpScatterRecur   as kOpScatter from the run's final
//               buffer / plus omega * the unfinished cycle's f (FP64)
//   kOpDeflate  x64 += mean / sigma; r64 -= mean; partial = ||r64||^2
//   kOpPrepare  rhs32 = r64 / rnorm; xa32 = 0; partial = ||rhs32||^2
//   kOpZero64   v = 0
// Residual recursion: number of Richardson steps of the run's last cycle
// that the cycle-start iterate does not include yet (0 while running).
__device__ inline int64_t pending_steps(const InstState &st, int p)
{
    if (st.status == kRunning)
        return 0;
    const int64_t n = (st.status == kMaxIter ? st.iters : st.iters - 1) - st.cycle * p;
    return n < p - 1 ? n : p - 1;
}

__global__ __launch_bounds__(kThreads) void k_stream_batched(const BatchStreamArgs a)
{
    __shared__ double red[kThreads / 64];
    const int nitems = *a.nitems;
    for (int w = blockIdx.x; w < nitems; w += gridDim.x) {
        const int2 it = a.items[w];
        const int sys = it.x;
        if (a.mask && a.mask[sys] < a.mask_min)
            continue;
        const BatchCtl &c = a.ctl[sys];
        if (a.op == kOpCorrect && c.outer < 1)
            continue;
        const int64_t off = a.offs[sys];
        const int64_t N = a.sizes[sys];
        const int64_t lo = (int64_t)it.y * kChunk;
        const int64_t hi = lo + kChunk < N ? lo + kChunk : N;
        double acc = 0.0;
        for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
            switch (a.op) {
            case kOpGather:
                a.v64[off + i] = a.user[a.uoffs[sys] + i];
                break;
            case kOpScatter:
                a.user[a.uoffs[sys] + i] = c.zero ? 0.0 : a.v64[off + i];
                break;
            case kOpScatterSel:
                a.user[a.uoffs[sys] + i] = c.zero ? 0.0 : (c.dsel ? a.x64 : a.v64)[off + i];
                break;
            case kOpScatterRecur: {
                // x at the end of the run: the cycle-start iterate plus omega
                // times the f's of the Richardson steps taken in the last cycle
                const InstState &st = a.state[sys];
                const int64_t base = st.cycle * a.p, n = pending_steps(st, a.p);
                double v = a.v64[off + i];
                for (int64_t k = 0; k < n; ++k) {
                    const int64_t at = ((base + k) % a.nslots) * a.slot_stride + off + i;
                    v += a.omega * (a.ring_f32 ? (double)static_cast<const float *>(a.fring)[at]
                                               : static_cast<const double *>(a.fring)[at]);
                }
                a.user[a.uoffs[sys] + i] = c.zero ? 0.0 : v;
                break;
            }
            case kOpNorm: {
                const double v = a.v64[off + i];
                acc += v * v;
                break;
            }
            case kOpSum:
                acc += a.v64[off + i];
                break;
            case kOpCorrect: {
                float d;
                if (a.recur) {
                    const InstState &st = a.state[sys];
                    const float *ring = static_cast<const float *>(a.fring);
                    const float om = (float)a.omega;
                    const int64_t base = st.cycle * a.p, n = pending_steps(st, a.p);
                    d = a.xa32[off + i];
                    for (int64_t k = 0; k < n; ++k)
                        d += om * ring[((base + k) % a.nslots) * a.slot_stride + off + i];
                } else {
                    d = (c.dsel ? a.xb32 : a.xa32)[off + i];
                }
                a.v64[off + i] += c.rnorm * (double)d;
                break;
            }
            case kOpDeflate: {
                a.x64[off + i] += c.mean * a.inv_shift[sys];
                const double v = a.v64[off + i] - c.mean;
                a.v64[off + i] = v;
                acc += v * v;
                break;
            }
            case kOpPrepare: {
                const float v = (float)(a.v64[off + i] * (1.0 / c.rnorm));
                a.rhs32[off + i] = v;
                a.xa32[off + i] = 0.0f;
                acc += (double)v * (double)v;
                break;
            }
            case kOpZero64:
                a.v64[off + i] = 0.0;
                break;
            default:
                break;
            }
        }
        if (a.partial) {
            acc = wave_sum_a(acc);
            if ((threadIdx.x & 63) == 0)
                red[threadIdx.x >> 6] = acc;
            __syncthreads();
            if (threadIdx.x == 0)
                a.partial[w] = red[0] + red[1] + red[2] + red[3];
            __syncthreads();
        }
    }
}

hipError_t launch_stream_batched(const BatchStreamArgs &a, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_stream_batched, dim3(grid), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

// Sum of a system's item partials [base, base + n) in a fixed order.
__device__ inline double item_sum(const double *partial, int base, int n)
{
    double r = 0.0;
    for (int t = threadIdx.x; t < n; t += 64)
        r += partial[base + t];
    return __shfl(wave_sum_a(r), 0, 64);
}

// Per-system control step (one wave per system).  step:
//   kCtlSelect   decide which systems take a refinement step now (refine = 1);
//                finished inner runs record their iterations and result buffer
//   kCtlNormB    nb64 = sqrt(sum of the norm partials of b)
//   kCtlMean     mean = (sum partials) / N
//   kCtlDecide   rel = ||r|| / ||b||: done, or start an inner run (refine = 2)
//   kCtlStart    initialise the run state of systems with refine == 2 from the
//                norm partials of their right-hand side
__global__ __launch_bounds__(64) void k_ctl_batched(const BatchCtlArgs a)
{
    const int i = blockIdx.x;
    BatchCtl &c = a.ctl[i];
    InstState &st = a.state[i];
    const int tid = threadIdx.x;
    switch (a.step) {
    case kCtlSelect: {
        if (tid != 0)
            return;
        int r = 0;
        if (c.phase == kPhaseStart) {
            r = 1;
        } else if (c.phase == kPhaseInner && st.status != kRunning) {
            const int64_t done = st.status == kMaxIter ? st.max_iter : st.iters;
            c.used += done;
            c.iters_last = done;
            c.dsel = final_buffer(st, a.p);
            if (st.status == kBreakdown) {
                c.phase = kPhaseDone;
                c.status = 2;
            } else if (!a.mixed) {
                c.phase = kPhaseDone;
                c.status = st.status == kConverged ? 0 : 1;
                c.rel = st.last_r;
            } else {
                r = 1;
            }
        }
        a.refine[i] = r;
        if (c.phase != kPhaseDone)
            atomicAdd(a.remaining, 1);
        return;
    }
    case kCtlNormB: {
        if (a.refine[i] == 0)
            return;
        const double s = item_sum(a.partial, a.cbase[i], a.nchunks[i]);
        if (tid == 0)
            c.nb64 = sqrt(s);
        return;
    }
    case kCtlMean: {
        if (a.refine[i] == 0)
            return;
        const double s = item_sum(a.partial, a.cbase[i], a.nchunks[i]);
        if (tid == 0)
            c.mean = s / (double)a.sizes[i];
        return;
    }
    case kCtlDecide: {
        if (a.refine[i] == 0)
            return;
        if (!a.mixed) {   // FP64 runs start directly on b
            if (tid == 0) {
                c.phase = kPhaseInner;
                a.refine[i] = 2;
            }
            return;
        }
        const int base = a.deflate ? a.cbase[i] : a.sbase[i];
        const int n = a.deflate ? a.nchunks[i] : a.ntiles[i];
        const double s = item_sum(a.partial, base, n);
        if (tid != 0)
            return;
        const double rn = sqrt(s);
        if (c.nb64 == 0.0) {
            c.phase = kPhaseDone;
            c.status = 0;
            c.rel = 0.0;
            c.zero = 1;
            a.refine[i] = 0;
            return;
        }
        const double rel = rn / c.nb64;
        c.rel = rel;
        if (!isfinite(rel)) {
            c.phase = kPhaseDone;
            c.status = 2;
            a.refine[i] = 0;
        } else if (rel < a.tol) {
            c.phase = kPhaseDone;
            c.status = 0;
            a.refine[i] = 0;
        } else if (c.outer >= a.max_outer || c.used >= a.max_iter) {
            c.phase = kPhaseDone;
            c.status = 1;
            a.refine[i] = 0;
        } else {
            c.phase = kPhaseInner;
            c.outer += 1;
            c.rnorm = rn;
            a.refine[i] = 2;
        }
        return;
    }
    case kCtlStart: {
        if (a.refine[i] != 2)
            return;
        const double s = item_sum(a.partial, a.cbase[i], a.nchunks[i]);
        if (tid != 0)
            return;
        st.cycle = 0;
        st.iters = 0;
        st.max_iter = a.max_iter - c.used;
        st.tol = a.mixed ? inner_tolerance(a.inner_tol, a.tol, c.rel) : a.tol;
        st.status = kRunning;
        st.rank = 0;
        st.nb = sqrt(s);
        st.last_r = 0.0;
        st.best_r = INFINITY;
        st.since_best = 0;
        st.log_count = 0;
        st.nf = 0;
        st.nd = 0;
        st.wslot = -1;
        st.restart_pos = 0;
        if (!(st.nb > 0.0)) {       // b = 0: x = 0 after zero iterations
            st.status = kConverged;
            c.phase = kPhaseDone;
            c.status = st.nb == 0.0 ? 0 : 2;
            c.zero = st.nb == 0.0;
            c.rel = 0.0;
        }
        return;
    }
    default:
        return;
    }
}

hipError_t launch_ctl_batched(const BatchCtlArgs &a, int count, hipStream_t s)
{
    hipLaunchKernelGGL(k_ctl_batched, dim3(count), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace aar
