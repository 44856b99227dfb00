// Anderson-step kernels of the AAR iteration on gfx950.
//
//   k_gram    the tall-skinny products of the extrapolation step (Eq. 3):
//             G = F_k^T F_k and c = F_k^T f_k, with the columns of F_k
//             (Eq. 5) formed in registers as differences of consecutive
//             history slots and every product accumulated in FP64.  One
//             partial per workgroup; no atomics, so the sums are
//             deterministic.  Together with the residual norm of the kFk
//             stencil pass this is the single global reduction per Anderson
//             step of Secs. 3.2-3.3.
//   k_gram_finish  sums each entry's per-workgroup partials (fixed order).
//   k_lsq     one wave: finishes the residual norm (and, after the fused
//             Gram pass, the Gram entries), tests convergence on
//             ||b - A x_k|| / ||b|| (Sec. 2), solves gamma = (F^T F)^+ F^T f_k
//             (Moore-Penrose pseudoinverse, Sec. 3.2) and writes the update
//             as a linear combination of history slots.  The pseudoinverse
//             drops eigenvalues <= rcond * l * lambda_max; when a Cholesky
//             factor proves all eigenvalues exceed that threshold it is the
//             inverse and the Cholesky solve is used, otherwise a parallel
//             (round-robin ordered) Jacobi eigendecomposition.
//   k_update  x_{k+1} = x_k + beta f_k - (X_k + beta F_k) gamma, streamed.
//             X_k columns of Richardson steps are omega f_j (their exact
//             increment); those of Anderson steps come from a small ring of
//             stored increments.
#include <math.h>

#include "aar_device.h"
#include "anderson_core.h"

namespace aar {


int stream_blocks(int64_t N)
{
    int64_t b = (N + kThreads * 4 - 1) / (kThreads * 4);
    if (b < 1)
        b = 1;
    if (b > 2048)
        b = 2048;
    return (int)b;
}

// Workgroups of the Gram pass: enough waves to cover HBM latency, few enough
// that the one-workgroup solve reads its partial table in one pass.
// Workgroups of the Gram pass: enough to cover N in 8-point strides, capped
// at what the chip holds at once for the history length m (the register
// footprint of the m(m+3)/2 accumulators sets 3 waves per SIMD at m = 7 and
// 2 beyond), so no workgroup waits for a second round.
int gram_blocks(int64_t N, int m)
{
    const int64_t cap = m <= 6 ? 1024 : m == 7 ? 768 : m <= kFastGramM ? 512 : 1024;
    int64_t b = (N + kThreads * 8 - 1) / (kThreads * 8);
    if (b < 1)
        b = 1;
    if (b > cap)
        b = cap;
    return (int)b;
}

// ---------------------------------------------------------------------------
// Gram products
// ---------------------------------------------------------------------------
template <typename H, int MC>
__global__ __launch_bounds__(kThreads) void k_gram(const GramArgs a)
{
    constexpr int NP = MC * (MC + 1) / 2;
    constexpr int NE = NP + MC;
    constexpr int V = VecWidth<H>::value;
    __shared__ double red[kThreads / 64][NE];
    const InstState *s = a.state;
    if (s->status != kRunning)
        return;
    const int64_t k = s->cycle * a.p + a.p - 1;
    if (k >= s->max_iter)
        return;
    const int l = (int)(k < a.m ? k : a.m);
    const H *ring = reinterpret_cast<const H *>(a.fring);
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

    auto accumulate = [&](const double *fv) {
        double fk = 0.0;   // f_k sits at position l
#pragma unroll
        for (int t = 0; t <= MC; ++t)
            fk = t == l ? fv[t] : fk;
        double d[MC];
#pragma unroll
        for (int c = 0; c < MC; ++c)
            d[c] = c < l ? fv[c + 1] - fv[c] : 0.0;
        int e = 0;
#pragma unroll
        for (int c = 0; c < MC; ++c) {
#pragma unroll
            for (int c2 = c; c2 < MC; ++c2)
                acc[e++] += d[c] * d[c2];
        }
#pragma unroll
        for (int c = 0; c < MC; ++c)
            acc[NP + c] += d[c] * fk;
    };

    // slot bases are padded to 8 elements, so every V-aligned index is aligned
    const int64_t nvec = a.N / V;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (l == MC) {
        // Full history (every cycle after the first m iterations): all slots
        // are read, and the loads of the next vector index are issued before
        // the products of the current one, so each wave keeps its loads in
        // flight while it computes.
        using P = Pack<H, V>;
        P cur[MC + 1], nxt[MC + 1];
        int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        if (v < nvec) {
#pragma unroll
            for (int t = 0; t <= MC; ++t)
                cur[t] = *reinterpret_cast<const P *>(slot[t] + v * V);
        }
        for (; v < nvec; v += stride) {
            const int64_t vn = v + stride;
            if (vn < nvec) {
#pragma unroll
                for (int t = 0; t <= MC; ++t)
                    nxt[t] = *reinterpret_cast<const P *>(slot[t] + vn * V);
            }
#pragma unroll
            for (int u = 0; u < V; ++u) {
                double col[MC + 1];
#pragma unroll
                for (int t = 0; t <= MC; ++t)
                    col[t] = (double)Hist<H>::load(cur[t].v, u);
                // l == MC: f_k is the last column and every difference is live
                double d[MC];
#pragma unroll
                for (int c = 0; c < MC; ++c)
                    d[c] = col[c + 1] - col[c];
                int e = 0;
#pragma unroll
                for (int c = 0; c < MC; ++c) {
#pragma unroll
                    for (int c2 = c; c2 < MC; ++c2)
                        acc[e++] += d[c] * d[c2];
                }
#pragma unroll
                for (int c = 0; c < MC; ++c)
                    acc[NP + c] += d[c] * col[MC];
            }
#pragma unroll
            for (int t = 0; t <= MC; ++t)
                cur[t] = nxt[t];
        }
    }
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < MC && v < nvec; v += stride) {
        double fv[MC + 1][V];
#pragma unroll
        for (int t = 0; t <= MC; ++t) {
            if (t <= l)
                load_vec<H, V>(slot[t], v * V, fv[t]);
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
            accumulate(col);
        }
    }
    for (int64_t i = nvec * V + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.N; i += stride) {
        double col[MC + 1];
#pragma unroll
        for (int t = 0; t <= MC; ++t)
            col[t] = t <= l ? (double)Hist<H>::load(slot[t], i) : 0.0;
        accumulate(col);
    }

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    wave_sums_to<NE>(acc, red[wave]);   // red[wave][e]: this wave's total of entry e
    __syncthreads();
    // transposed partial table: entry-major, one column per workgroup
    for (int e = threadIdx.x; e < NE; e += blockDim.x) {
        double v = 0.0;
        for (int w = 0; w < kThreads / 64; ++w)
            v += red[w][e];
        a.partial[(int64_t)e * gridDim.x + blockIdx.x] = v;
    }
}

// One entry of G or c per blockIdx.y (histories longer than the fast path).
template <typename H>
__global__ __launch_bounds__(kThreads) void k_gram_entry(const GramArgs a)
{
    __shared__ double red[kThreads / 64];
    const InstState *s = a.state;
    if (s->status != kRunning)
        return;
    const int64_t k = s->cycle * a.p + a.p - 1;
    if (k >= s->max_iter)
        return;
    const int l = (int)(k < a.m ? k : a.m);
    const int m = a.m;
    const int np = m * (m + 1) / 2;
    const int e = blockIdx.y;
    int ca, cb;   // column pair (cb == -1: c entry against f_k)
    if (e < np) {
        int r = 0, rem = e;
        while (rem >= m - r) {
            rem -= m - r;
            ++r;
        }
        ca = r;
        cb = r + rem;
    } else {
        ca = e - np;
        cb = -1;
    }
    const H *ring = reinterpret_cast<const H *>(a.fring);
    double acc = 0.0;
    if (ca < l && cb < l) {
        const H *fa0 = ring + (int64_t)((k - l + ca) % a.nslots) * a.slot_stride;
        const H *fa1 = ring + (int64_t)((k - l + ca + 1) % a.nslots) * a.slot_stride;
        const H *fb0 = cb >= 0 ? ring + (int64_t)((k - l + cb) % a.nslots) * a.slot_stride : nullptr;
        const H *fb1 = cb >= 0 ? ring + (int64_t)((k - l + cb + 1) % a.nslots) * a.slot_stride
                               : ring + (int64_t)(k % a.nslots) * a.slot_stride;
        const int64_t stride = (int64_t)gridDim.x * blockDim.x;
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.N; i += stride) {
            const double da = (double)Hist<H>::load(fa1, i) - (double)Hist<H>::load(fa0, i);
            const double db = fb0 ? (double)Hist<H>::load(fb1, i) - (double)Hist<H>::load(fb0, i)
                                  : (double)Hist<H>::load(fb1, i);
            acc += da * db;
        }
    }
    acc = wave_sum_a(acc);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = 0.0;
        for (int w = 0; w < kThreads / 64; ++w)
            v += red[w];
        a.partial[(int64_t)e * gridDim.x + blockIdx.x] = v;
    }
}

template <typename H>
static hipError_t launch_gram_h(const GramArgs &a, int blocks, hipStream_t s)
{
    switch (a.m) {
#define AAR_GRAM_CASE(MC)                                                                      \
    case MC:                                                                                   \
        hipLaunchKernelGGL((k_gram<H, MC>), dim3(blocks), dim3(kThreads), 0, s, a);            \
        return hipGetLastError();
        AAR_GRAM_CASE(1)
        AAR_GRAM_CASE(2)
        AAR_GRAM_CASE(3)
        AAR_GRAM_CASE(4)
        AAR_GRAM_CASE(5)
        AAR_GRAM_CASE(6)
        AAR_GRAM_CASE(7)
        AAR_GRAM_CASE(8)
        AAR_GRAM_CASE(9)
        AAR_GRAM_CASE(10)
        AAR_GRAM_CASE(11)
        AAR_GRAM_CASE(12)
#undef AAR_GRAM_CASE
    default:
        hipLaunchKernelGGL((k_gram_entry<H>), dim3(blocks, a.ne), dim3(kThreads), 0, s, a);
        return hipGetLastError();
    }
}

hipError_t launch_gram(Prec prec, const GramArgs &a, int blocks, hipStream_t s)
{
    switch (prec) {
    case Prec::F64:
        return launch_gram_h<double>(a, blocks, s);
    case Prec::F32:
        return launch_gram_h<float>(a, blocks, s);
    case Prec::F32_BF16:
        return launch_gram_h<bf16_t>(a, blocks, s);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Small least-squares solve, convergence test and update plan (one workgroup)
// ---------------------------------------------------------------------------
// Fixed-order sum of one entry's per-workgroup partials (one workgroup per
// entry of G and c): thread-strided sums, then the four wave sums in order.
__global__ __launch_bounds__(kThreads) void k_gram_finish(const double *partial, int blocks, double *out,
                                                          const InstState *state, int p)
{
    __shared__ double red[kThreads / 64];
    if (state->status != kRunning || state->cycle * p + p - 1 >= state->max_iter)
        return;
    const double *col = partial + (int64_t)blockIdx.x * blocks;
    double v = 0.0;
    for (int b = threadIdx.x; b < blocks; b += kThreads)
        v += col[b];
    v = wave_sum_a(v);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0)
        out[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

hipError_t launch_gram_finish(const double *partial, int blocks, double *out, int ne, const InstState *state,
                              int p, hipStream_t s)
{
    hipLaunchKernelGGL(k_gram_finish, dim3(ne), dim3(kThreads), 0, s, partial, blocks, out, state, p);
    return hipGetLastError();
}

__global__ __launch_bounds__(kLsqThreads) void k_lsq(const LsqArgs a)
{
    __shared__ double gsum[kFusedGramNE];
    InstState *st = a.state;
    // residual norm: thread-strided partials, fixed-order wave sum, broadcast
    // (read before the run state is checked, so both loads overlap)
    double r = 0.0;
    for (int i = threadIdx.x; i < a.rho_blocks; i += kLsqThreads)
        r += a.rho_partial[i];
    r = wave_sum_a(r);
    const double *gv = a.gram_final;
    if (a.gram_partial) {
        // Gram entries of the fused pass: lane-strided partial sums in a
        // fixed order, then one transposed wave reduction into LDS.  Two
        // workgroups per lane are loaded at once (70 loads in flight), so
        // the table of a 256-workgroup pass takes two memory round trips;
        // indices past the table are clamped and their values dropped.
        constexpr int kBatch = 2;
        const int nb = a.gram_blocks;
        double acc[kFusedGramNE];
#pragma unroll
        for (int e = 0; e < kFusedGramNE; ++e)
            acc[e] = 0.0;
        for (int b0 = 0; b0 < nb; b0 += kBatch * kLsqThreads) {
            double v[kBatch][kFusedGramNE];
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const int b = b0 + (int)threadIdx.x + u * kLsqThreads;
                const int bc = b < nb ? b : nb - 1;
#pragma unroll
                for (int e = 0; e < kFusedGramNE; ++e)
                    v[u][e] = a.gram_partial[(int64_t)e * nb + bc];
            }
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const bool in = b0 + (int)threadIdx.x + u * kLsqThreads < nb;
#pragma unroll
                for (int e = 0; e < kFusedGramNE; ++e)
                    acc[e] += in ? v[u][e] : 0.0;
            }
        }
        wave_sums_to<kFusedGramNE>(acc, gsum);
        __syncthreads();
        gv = gsum;
    }
    lsq_core(a, st, __shfl(r, 0, 64), gv);
}

hipError_t launch_lsq(const LsqArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_lsq, dim3(1), dim3(kLsqThreads), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Anderson update
// ---------------------------------------------------------------------------
template <typename T, typename H>
__global__ __launch_bounds__(kThreads) void k_update(const UpdateArgs<T> a)
{
    constexpr int V = 16 / (int)sizeof(T);
    using D = typename DxOf<T, H>::type;
    __shared__ const H *fs[kMaxSlots];
    __shared__ T al[kMaxSlots];
    __shared__ const D *ds[kMaxM];
    __shared__ T de[kMaxM];
    __shared__ int nf_s, nd_s, ws_s;
    const InstState *st = a.state;
    const int status = st->status;
    if (a.status_out && blockIdx.x == 0 && threadIdx.x == 0)
        *a.status_out = status;
    if (status != kRunning)
        return;
    const H *ring = reinterpret_cast<const H *>(a.fring);
    if (threadIdx.x == 0) {
        nf_s = st->nf;
        nd_s = st->nd;
        ws_s = st->wslot;
    }
    if (threadIdx.x < kMaxSlots) {
        const int t = threadIdx.x;
        if (t < st->nf) {
            fs[t] = ring + (int64_t)st->fslot[t] * a.slot_stride;
            al[t] = (T)st->alpha[t];
        }
    }
    if (threadIdx.x < kMaxM && (int)threadIdx.x < st->nd) {
        ds[threadIdx.x] = reinterpret_cast<const D *>(a.dxring) + (int64_t)st->dslot[threadIdx.x] * a.dx_stride;
        de[threadIdx.x] = (T)st->delta[threadIdx.x];
    }
    __syncthreads();
    const int nf = nf_s, nd = nd_s;
    // residual recursion: history positions tr0 .. nf - 2 are the cycle's
    // Richardson steps (none when p_rich is 0)
    const int tr0 = a.p_rich > 0 ? nf - a.p_rich : nf;
    D *dxw = ws_s >= 0 ? reinterpret_cast<D *>(a.dxring) + (int64_t)ws_s * a.dx_stride : nullptr;
    const T *fk_ptr = a.fcur;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t nvec = a.N / V;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nvec; v += stride) {
        const int64_t i = v * V;
        T d[V], dr[V];
#pragma unroll
        for (int u = 0; u < V; ++u) {
            d[u] = T(0);
            dr[u] = T(0);
        }
        const int t1 = tr0 < nf - 1 ? tr0 : nf - 1;
        for (int t = 0; t < t1; ++t) {
            const Pack<H, V> h = *reinterpret_cast<const Pack<H, V> *>(fs[t] + i);
#pragma unroll
            for (int u = 0; u < V; ++u)
                d[u] += al[t] * (T)Hist<H>::load(h.v, u);
        }
        for (int t = t1; t < nf - 1; ++t) {   // the cycle's Richardson steps (residual recursion)
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
        const Pack<T, V> xc = *reinterpret_cast<const Pack<T, V> *>(a.xin + i);
        Pack<T, V> xn;
        Pack<D, V> dx;
#pragma unroll
        for (int u = 0; u < V; ++u) {
            const T xk = xc.v[u] + a.omega_rich * dr[u];
            xn.v[u] = xk + d[u];
            dx.v[u] = (D)(xn.v[u] - xk);     // the increment actually taken
        }
        *reinterpret_cast<Pack<T, V> *>(a.xout + i) = xn;
        if (dxw)
            *reinterpret_cast<Pack<D, V> *>(dxw + i) = dx;
    }
    for (int64_t i = nvec * V + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.N; i += stride) {
        T d = 0, dr = 0;
        for (int t = 0; t < nf - 1; ++t) {
            const T fv = (T)Hist<H>::load(fs[t], i);
            d += al[t] * fv;
            dr += t >= tr0 ? fv : T(0);
        }
        const T fk = fk_ptr ? fk_ptr[i] : (T)Hist<H>::load(fs[nf - 1], i);
        d += al[nf - 1] * fk;
        for (int t = 0; t < nd; ++t)
            d += de[t] * (T)ds[t][i];
        const T xk = a.xin[i] + a.omega_rich * dr;
        const T xn = xk + d;
        a.xout[i] = xn;
        if (dxw)
            dxw[i] = (D)(xn - xk);
    }
}

hipError_t launch_update(Prec prec, const UpdateArgs<double> *a64, const UpdateArgs<float> *a32, int blocks,
                         hipStream_t s)
{
    if (a64) {   // FP64 iterate: history in FP64, FP32 or bf16
        switch (prec) {
        case Prec::F64:
            hipLaunchKernelGGL((k_update<double, double>), dim3(blocks), dim3(kThreads), 0, s, *a64);
            break;
        case Prec::F32:
            hipLaunchKernelGGL((k_update<double, float>), dim3(blocks), dim3(kThreads), 0, s, *a64);
            break;
        case Prec::F32_BF16:
            hipLaunchKernelGGL((k_update<double, bf16_t>), dim3(blocks), dim3(kThreads), 0, s, *a64);
            break;
        }
        return hipGetLastError();
    }
    switch (prec) {
    case Prec::F64:
        return hipErrorInvalidValue;
    case Prec::F32:
        hipLaunchKernelGGL((k_update<float, float>), dim3(blocks), dim3(kThreads), 0, s, *a32);
        break;
    case Prec::F32_BF16:
        hipLaunchKernelGGL((k_update<float, bf16_t>), dim3(blocks), dim3(kThreads), 0, s, *a32);
        break;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Norms, state initialisation, casts and the refinement correction
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void k_norm_partial(const T *v, int64_t N, double *partial)
{
    __shared__ double red[kThreads / 64];
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
        const double x = (double)v[i];
        acc += x * x;
    }
    acc = wave_sum_a(acc);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kThreads / 64; ++w)
            s += red[w];
        partial[blockIdx.x] = s;
    }
}

hipError_t launch_norm_partial(bool f64, const void *v, int64_t N, double *partial, int blocks, hipStream_t s)
{
    if (f64)
        hipLaunchKernelGGL((k_norm_partial<double>), dim3(blocks), dim3(kThreads), 0, s,
                           (const double *)v, N, partial);
    else
        hipLaunchKernelGGL((k_norm_partial<float>), dim3(blocks), dim3(kThreads), 0, s,
                           (const float *)v, N, partial);
    return hipGetLastError();
}

__device__ inline double block_fixed_sum(const double *partial, int blocks)
{
    double r = 0.0;
    for (int i = threadIdx.x; i < blocks; i += 64)
        r += partial[i];
    return wave_sum_a(r);
}

__global__ __launch_bounds__(64) void k_init_state(InstState *st, const double *partial, int blocks,
                                                   int64_t max_iter, double tol)
{
    const double s = block_fixed_sum(partial, blocks);
    if (threadIdx.x == 0) {
        st->cycle = 0;
        st->max_iter = max_iter;
        st->tol = tol;
        st->iters = 0;
        st->status = kRunning;
        st->rank = 0;
        st->nb = sqrt(s);
        st->last_r = 0.0;
        st->best_r = INFINITY;
        st->since_best = 0;
        st->log_count = 0;
        st->nf = 0;
        st->nd = 0;
        st->wslot = -1;
        st->restart_pos = 0;
    }
}

__global__ __launch_bounds__(64) void k_init_state_keep(InstState *st, const double *partial, int blocks,
                                                        int64_t budget, double tol, int p)
{
    const double s = block_fixed_sum(partial, blocks);
    if (threadIdx.x == 0) {
        // the previous run stopped at an Anderson step without extrapolating:
        // the next cycle starts the new run
        const int64_t cycle = st->cycle + 1;
        st->cycle = cycle;
        st->restart_pos = cycle * p;
        st->max_iter = cycle * p + budget;
        st->tol = tol;
        st->iters = 0;
        st->status = kRunning;
        st->nb = sqrt(s);
        st->last_r = 0.0;
        st->best_r = INFINITY;
        st->since_best = 0;
        st->log_count = 0;
    }
}

hipError_t launch_init_state_keep(InstState *st, const double *partial, int blocks, int64_t budget, double tol,
                                  int p, hipStream_t s)
{
    hipLaunchKernelGGL(k_init_state_keep, dim3(1), dim3(64), 0, s, st, partial, blocks, budget, tol, p);
    return hipGetLastError();
}

hipError_t launch_init_state(InstState *st, const double *partial, int blocks, int64_t max_iter, double tol,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_init_state, dim3(1), dim3(64), 0, s, st, partial, blocks, max_iter, tol);
    return hipGetLastError();
}

__global__ __launch_bounds__(64) void k_finish_norm(double *out, const double *partial, int blocks)
{
    const double s = block_fixed_sum(partial, blocks);
    if (threadIdx.x == 0)
        *out = sqrt(s);
}

hipError_t launch_finish_norm(double *out, const double *partial, int blocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_finish_norm, dim3(1), dim3(64), 0, s, out, partial, blocks);
    return hipGetLastError();
}

// out = (float)(in / *norm): the scaled FP32 right-hand side of an inner solve
__global__ __launch_bounds__(kThreads) void k_scale_cast(const double *in, float *out, int64_t N,
                                                         const double *norm)
{
    const double inv = 1.0 / *norm;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride)
        out[i] = (float)(in[i] * inv);
}

hipError_t launch_cast_f64_to_f32(const double *in, float *out, int64_t N, const double *norm, hipStream_t s)
{
    hipLaunchKernelGGL(k_scale_cast, dim3(stream_blocks(N)), dim3(kThreads), 0, s, in, out, N, norm);
    return hipGetLastError();
}

template <typename T> __global__ __launch_bounds__(kThreads) void k_zero(T *v, int64_t N)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride)
        v[i] = T(0);
}

hipError_t launch_zero_f32(float *v, int64_t N, hipStream_t s)
{
    hipLaunchKernelGGL((k_zero<float>), dim3(stream_blocks(N)), dim3(kThreads), 0, s, v, N);
    return hipGetLastError();
}

hipError_t launch_zero_f64(double *v, int64_t N, hipStream_t s)
{
    hipLaunchKernelGGL((k_zero<double>), dim3(stream_blocks(N)), dim3(kThreads), 0, s, v, N);
    return hipGetLastError();
}

// Values in [-0.5, 0.5) from a multiplicative hash of the index: timing data
// for the tile autotuner (streaming kernels run measurably faster on zeros).
template <typename T> __global__ __launch_bounds__(kThreads) void k_fill_pattern(T *v, int64_t N)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
        const uint32_t h = (uint32_t)i * 2654435761u;
        v[i] = (T)((double)(h >> 8) * (1.0 / 16777216.0) - 0.5);
    }
}

hipError_t launch_fill_pattern_f64(double *v, int64_t N, hipStream_t s)
{
    hipLaunchKernelGGL((k_fill_pattern<double>), dim3(stream_blocks(N)), dim3(kThreads), 0, s, v, N);
    return hipGetLastError();
}

hipError_t launch_fill_pattern_f32(float *v, int64_t N, hipStream_t s)
{
    hipLaunchKernelGGL((k_fill_pattern<float>), dim3(stream_blocks(N)), dim3(kThreads), 0, s, v, N);
    return hipGetLastError();
}

// x += *scale * d: the correction step of the iterative refinement
__global__ __launch_bounds__(kThreads) void k_correct(double *x, const float *d, const double *scale, int64_t N)
{
    const double sc = *scale;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride)
        x[i] += sc * (double)d[i];
}

hipError_t launch_correct(double *x, const float *d, const double *scale, int64_t N, hipStream_t s)
{
    hipLaunchKernelGGL(k_correct, dim3(stream_blocks(N)), dim3(kThreads), 0, s, x, d, scale, N);
    return hipGetLastError();
}

__global__ __launch_bounds__(kThreads) void k_copy64(const double *in, double *out, int64_t N)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride)
        out[i] = in[i];
}

hipError_t launch_copy_f64(const double *in, double *out, int64_t N, hipStream_t s)
{
    hipLaunchKernelGGL(k_copy64, dim3(stream_blocks(N)), dim3(kThreads), 0, s, in, out, N);
    return hipGetLastError();
}

__global__ __launch_bounds__(kThreads) void k_cast64_32(const double *in, float *out, int64_t N)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride)
        out[i] = (float)in[i];
}

hipError_t launch_cast_f64_f32_plain(const double *in, float *out, int64_t N, hipStream_t s)
{
    hipLaunchKernelGGL(k_cast64_32, dim3(stream_blocks(N)), dim3(kThreads), 0, s, in, out, N);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Constant-mode deflation (periodic systems with A 1 = sigma 1)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_sum_partial(const double *v, int64_t N, double *partial)
{
    __shared__ double red[kThreads / 64];
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride)
        acc += v[i];
    acc = wave_sum_a(acc);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kThreads / 64; ++w)
            s += red[w];
        partial[blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(64) void k_mean_finish(double *out, const double *partial, int blocks, int64_t N)
{
    const double s = block_fixed_sum(partial, blocks);
    if (threadIdx.x == 0)
        *out = s / (double)N;
}

__global__ __launch_bounds__(kThreads) void k_deflate_apply(double *x, double *r, int64_t N, double inv_sigma,
                                                            const double *mean, double *partial)
{
    __shared__ double red[kThreads / 64];
    const double mu = *mean;
    const double dx = mu * inv_sigma;
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
        x[i] += dx;
        const double v = r[i] - mu;
        r[i] = v;
        acc += v * v;
    }
    acc = wave_sum_a(acc);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kThreads / 64; ++w)
            s += red[w];
        partial[blockIdx.x] = s;
    }
}

hipError_t launch_deflate(double *x, double *r, int64_t N, double inv_sigma, double *partial, int blocks,
                          double *scal, hipStream_t s)
{
    hipLaunchKernelGGL(k_sum_partial, dim3(blocks), dim3(kThreads), 0, s, r, N, partial);
    hipLaunchKernelGGL(k_mean_finish, dim3(1), dim3(64), 0, s, scal + 2, partial, blocks, N);
    hipLaunchKernelGGL(k_deflate_apply, dim3(blocks), dim3(kThreads), 0, s, x, r, N, inv_sigma, scal + 2, partial);
    return hipGetLastError();
}


// ---------------------------------------------------------------------------
// Residual recursion: the returned iterate.  The sweeps of a cycle do not
// write x, so when a run stops, x (the cycle's first iterate x_c) receives the
// Richardson steps the unfinished cycle has taken: x_n = x_c + omega sum
// f_j, j = cycle p .. n - 1, with n the iterate being returned (k for a
// decision at Anderson step k, the cap for a capped run).
template <typename T, typename H>
__global__ __launch_bounds__(kThreads) void k_finalize(T *x, const void *fring, const InstState *state, int p,
                                                     int nslots, int64_t slot_stride, T omega, int64_t N)
{
    const int status = state->status;
    if (status == kRunning)
        return;
    const int64_t base = state->cycle * p;
    int64_t n = (status == kMaxIter ? state->iters : state->iters - 1) - base;
    if (n > p - 1)
        n = p - 1;
    if (n <= 0)
        return;
    const H *ring = reinterpret_cast<const H *>(fring);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
        T v = x[i];
        for (int64_t s = 0; s < n; ++s)
            v += omega * (T)Hist<H>::load(ring + (int64_t)((base + s) % nslots) * slot_stride, i);
        x[i] = v;
    }
}

hipError_t launch_finalize_f64(Prec hist, double *x, const void *fring, const InstState *state, int p, int nslots,
                               int64_t slot_stride, double omega, int64_t N, hipStream_t s)
{
    if (hist == Prec::F64)
        hipLaunchKernelGGL((k_finalize<double, double>), dim3(stream_blocks(N)), dim3(kThreads), 0, s, x, fring,
                           state, p, nslots, slot_stride, omega, N);
    else if (hist == Prec::F32)
        hipLaunchKernelGGL((k_finalize<double, float>), dim3(stream_blocks(N)), dim3(kThreads), 0, s, x, fring,
                           state, p, nslots, slot_stride, omega, N);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_finalize_f32(float *x, const void *fring, const InstState *state, int p, int nslots,
                               int64_t slot_stride, float omega, int64_t N, hipStream_t s)
{
    hipLaunchKernelGGL((k_finalize<float, float>), dim3(stream_blocks(N)), dim3(kThreads), 0, s, x, fring, state,
                       p, nslots, slot_stride, omega, N);
    return hipGetLastError();
}

}  // namespace aar
