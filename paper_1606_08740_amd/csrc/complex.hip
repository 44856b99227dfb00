// Complex-valued AAR on gfx950: the method over C (Sec. 2, Eq. 1, with
// complex relaxation parameters and T the conjugate transpose in Eq. 3), for
// the periodic Helmholtz problem of Sec. 3.2 (Eq. 7), whose shift and
// right-hand side are complex.  The operator is A = A_r + i s I: the real
// finite-difference stencil (real weights, the real part of the shift) plus an
// imaginary shift; D = diag(A) is complex.  Values are complex FP64 stored
// interleaved (re, im).
//
// Kernels of one cycle (the iteration without the residual recursion: each
// Richardson sweep reads x and b and writes x and f):
//   stencil passes   the one-point 2.5D tile of the real passes, instantiated
//                    for the complex type (sweep, Anderson-step residual with
//                    the |b - A x|^2 partials, operator apply);
//   k_cgram          G = F^H F (upper triangle) and c = F^H f_k, columns of F
//                    formed as differences of consecutive history slots,
//                    real and imaginary parts accumulated in FP64 in one pass;
//                    per-workgroup partials, summed in a fixed order by
//                    k_gram_finish into [Re G, Re c | Im G, Im c];
//   k_clsq           one wave: convergence test, gamma = G^+ c through the real
//                    form [[Re G, -Im G], [Im G, Re G]] of the Hermitian G (the
//                    one-wave Jacobi pseudoinverse of the real solve, with the
//                    threshold counted on the complex order), update plan with
//                    complex coefficients;
//   k_cupdate        x_{k+1} = x_k + sum alpha_t f_t + sum delta_a dx_a.
#include "stencil_kernels.h"

namespace aar {

// ---------------------------------------------------------------------------
// Stencil passes
// ---------------------------------------------------------------------------
template <int MODE>
static hipError_t launch_cst_mode(int radius, StencilArgs<zd> a, const TileShape &ts, int *blocks_out, hipStream_t s)
{
#define AAR_C_RY(R)                                                                  \
    switch (ts.ry) {                                                                 \
    case 1:                                                                          \
        return launch_one<zd, zd, R, false, MODE, 1>(a, ts, blocks_out, s);          \
    case 2:                                                                          \
        return launch_one<zd, zd, R, false, MODE, 2>(a, ts, blocks_out, s);          \
    default:                                                                         \
        return hipErrorInvalidValue;                                                 \
    }
    switch (radius) {
    case 1:
        AAR_C_RY(1)
    case 2:
        AAR_C_RY(2)
    case 3:
        AAR_C_RY(3)
    case 4:
        AAR_C_RY(4)
    case 5:
        AAR_C_RY(5)
    case 6:
        AAR_C_RY(6)
    default:
        return hipErrorInvalidValue;
    }
#undef AAR_C_RY
}

hipError_t launch_stencil_complex(int mode, int radius, const TileShape &ts, StencilArgs<zd> a, int *blocks_out,
                                  hipStream_t s)
{
    if (ts.pair != 0)
        return hipErrorInvalidValue;
    switch (mode) {
    case kSweep:
        return launch_cst_mode<kSweep>(radius, a, ts, blocks_out, s);
    case kFk:
        return launch_cst_mode<kFk>(radius, a, ts, blocks_out, s);
    case kApply:
        return launch_cst_mode<kApply>(radius, a, ts, blocks_out, s);
    default:
        return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// Hermitian Gram products
// ---------------------------------------------------------------------------
// G = F^H F and c = F^H f_k in one pass over the history, with d_c the
// column differences and (fr, fi) = f_k:
//   Re G_cc2 = sum (dr_c dr_c2 + di_c di_c2)  (c <= c2),
//   Im G_cc2 = sum (dr_c di_c2 - di_c dr_c2)  (c < c2; the diagonal of a
//              Hermitian matrix is real, those entries stay exactly 0),
//   Re c_c = sum (dr_c fr + di_c fi),  Im c_c = sum (dr_c fi - di_c fr),
// entries in the real Gram's order (upper triangle by rows, then c).
// Per-workgroup partials: the real table (NE entries x the grid,
// entry-major), then the imaginary table, each summed by k_gram_finish.
// With a full history the loads of the next point are issued before the
// products of the current one.  Complex values are kept as separate re and
// im doubles, so no run-time selection of a value touches private memory.
// One pass reads the history slots once for both parts.
template <int MC>
__global__ __launch_bounds__(kThreads) void k_cgram(const GramArgs a)
{
    constexpr int NP = MC * (MC + 1) / 2;
    constexpr int NE = NP + MC;
    __shared__ double red_re[kThreads / 64][NE];
    __shared__ double red_im[kThreads / 64][NE];
    const InstState *s = a.state;
    if (s->status != kRunning)
        return;
    const int64_t k = s->cycle * a.p + a.p - 1;
    if (k >= s->max_iter)
        return;
    const int l = (int)(k < a.m ? k : a.m);
    const zd *ring = reinterpret_cast<const zd *>(a.fring);
    const zd *slot[MC + 1];
#pragma unroll
    for (int t = 0; t <= MC; ++t) {
        const int tt = t <= l ? t : l;
        slot[t] = ring + (int64_t)((k - l + tt) % a.nslots) * a.slot_stride;
    }
    double are[NE], aim[NE];
#pragma unroll
    for (int e = 0; e < NE; ++e) {
        are[e] = 0.0;
        aim[e] = 0.0;
    }
    // products of one point: history values (vr, vi)[0..MC], f_k at position
    // lh, differences past the history length are zero
    auto accumulate = [&](const double *vr, const double *vi, int lh) {
        double fr = 0.0, fi = 0.0;
#pragma unroll
        for (int t = 0; t <= MC; ++t) {
            fr = t == lh ? vr[t] : fr;
            fi = t == lh ? vi[t] : fi;
        }
        double dr[MC], di[MC];
#pragma unroll
        for (int c = 0; c < MC; ++c) {
            dr[c] = c < lh ? vr[c + 1] - vr[c] : 0.0;
            di[c] = c < lh ? vi[c + 1] - vi[c] : 0.0;
        }
        int e = 0;
#pragma unroll
        for (int c = 0; c < MC; ++c) {
#pragma unroll
            for (int c2 = c; c2 < MC; ++c2) {
                are[e] += dr[c] * dr[c2] + di[c] * di[c2];
                if (c2 > c)
                    aim[e] += dr[c] * di[c2] - di[c] * dr[c2];
                ++e;
            }
        }
#pragma unroll
        for (int c = 0; c < MC; ++c) {
            are[NP + c] += dr[c] * fr + di[c] * fi;
            aim[NP + c] += dr[c] * fi - di[c] * fr;
        }
    };
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l == MC) {
        double cr[MC + 1], ci[MC + 1], nr[MC + 1], ni[MC + 1];
        if (i < a.N) {
#pragma unroll
            for (int t = 0; t <= MC; ++t) {
                const zd v = slot[t][i];
                cr[t] = v.re;
                ci[t] = v.im;
            }
        }
        for (; i < a.N; i += stride) {
            const int64_t in = i + stride;
            if (in < a.N) {
#pragma unroll
                for (int t = 0; t <= MC; ++t) {
                    const zd v = slot[t][in];
                    nr[t] = v.re;
                    ni[t] = v.im;
                }
            }
            accumulate(cr, ci, MC);
#pragma unroll
            for (int t = 0; t <= MC; ++t) {
                cr[t] = nr[t];
                ci[t] = ni[t];
            }
        }
    } else {
        for (; i < a.N; i += stride) {
            double vr[MC + 1], vi[MC + 1];
#pragma unroll
            for (int t = 0; t <= MC; ++t) {
                const zd v = slot[t][i];
                vr[t] = v.re;
                vi[t] = v.im;
            }
            accumulate(vr, vi, l);
        }
    }
    const int w = threadIdx.x >> 6;
    wave_sums_to<NE>(are, red_re[w]);
    wave_sums_to<NE>(aim, red_im[w]);
    __syncthreads();
    for (int e = threadIdx.x; e < 2 * NE; e += kThreads) {
        double v = 0.0;
        for (int ww = 0; ww < kThreads / 64; ++ww)
            v += e < NE ? red_re[ww][e] : red_im[ww][e - NE];
        a.partial[(int64_t)e * gridDim.x + blockIdx.x] = v;
    }
}

// Complex history lengths whose Gram products run here (the real form of the
// m x m solve has order 2m <= kMaxM)
constexpr int kMaxComplexM = 8;

hipError_t launch_cgram(const GramArgs &a, int blocks, hipStream_t s)
{
    switch (a.m) {
#define AAR_CG(M)                                                                          \
    case M:                                                                                \
        hipLaunchKernelGGL((k_cgram<M>), dim3(blocks), dim3(kThreads), 0, s, a);           \
        return hipGetLastError();
        AAR_CG(1)
        AAR_CG(2)
        AAR_CG(3)
        AAR_CG(4)
        AAR_CG(5)
        AAR_CG(6)
        AAR_CG(7)
        AAR_CG(8)
#undef AAR_CG
    default:
        return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// Convergence test, Hermitian pseudoinverse solve and update plan (one wave)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kLsqThreads) void k_clsq(const LsqArgs a, double omega_im, double beta_im)
{
    __shared__ double S[kMaxM][kMaxM + 1];
    __shared__ double V[kMaxM][kMaxM + 1];
    __shared__ double cvec[kMaxM], wvec[kMaxM], gam[kMaxM];
    __shared__ double rot_c[kMaxM / 2], rot_s[kMaxM / 2];
    __shared__ int pair_p[kMaxM / 2], pair_q[kMaxM / 2];
    __shared__ double Li[kMaxM][kMaxM + 1];
    __shared__ double sh_off;
    __shared__ int sh_stop, sh_fail;
    InstState *st = a.state;
    const int tid = threadIdx.x;
    double r = 0.0;
    for (int i = tid; i < a.rho_blocks; i += kLsqThreads)
        r += a.rho_partial[i];
    r = __shfl(wave_sum_a(r), 0, 64);
    const int status0 = st->status;
    const int64_t cycle0 = st->cycle, max_iter0 = st->max_iter;
    const double nb0 = st->nb, tol0 = st->tol;
    const int log_count0 = st->log_count;
    if (status0 != kRunning)
        return;
    const int64_t k = cycle0 * a.p + a.p - 1;
    if (k >= max_iter0) {
        if (tid == 0) {
            st->iters = max_iter0;
            st->status = kMaxIter;
        }
        return;
    }
    const int l = (int)(k < a.m ? k : a.m);
    const int np = a.m * (a.m + 1) / 2;
    const double rel = sqrt(r) / nb0;
    // the l x l Hermitian G (entries (re, im) of the upper triangle) and c
    bool bad = !isfinite(rel);
    for (int idx = tid; idx < l * l; idx += kLsqThreads) {
        const int i = idx / l, j = idx % l;
        const int e = i <= j ? tri_index(i, j, a.m) : tri_index(j, i, a.m);
        const double gr = a.gram_final[e], gi0 = a.gram_final[a.ne + e];
        const double gi = i <= j ? gi0 : -gi0;       // G_ji = conj(G_ij)
        bad = bad || !isfinite(gr) || !isfinite(gi);
        S[i][j] = gr;
        S[i][j + l] = -gi;
        S[i + l][j] = gi;
        S[i + l][j + l] = gr;
    }
    for (int i = tid; i < l; i += kLsqThreads) {
        cvec[i] = a.gram_final[np + i];
        cvec[i + l] = a.gram_final[a.ne + np + i];
        bad = bad || !isfinite(cvec[i]) || !isfinite(cvec[i + l]);
    }
    bad = __any(bad);
    if (tid == 0) {
        st->last_r = rel;
        if (a.log && log_count0 < a.log_cap)
            a.log[log_count0] = rel;
        if (a.rank_log && log_count0 < a.log_cap)
            a.rank_log[log_count0] = -1;
        st->log_count = log_count0 + 1;
    }
    if (bad || rel < tol0) {
        if (tid == 0) {
            st->iters = k + 1;
            st->status = bad ? kBreakdown : kConverged;
        }
        return;
    }
    __syncthreads();
    // the Cholesky solve of the real form when it provably equals the
    // pseudoinverse (its eigenvalues are those of G, each twice), else the
    // Jacobi eigendecomposition
    bool fast = false;
    if (l > 0 && !a.force_pinv)
        fast = cholesky_proved_solve(2 * l, a.rcond, (double)l, 0.5, S, V, Li, cvec, wvec, gam, sh_fail);
    if (l > 0 && !fast)
        jacobi_pinv(2 * l, a.rcond, (double)l, S, V, cvec, wvec, gam, rot_c, rot_s, pair_p, pair_q, sh_off,
                    sh_stop);
    // gamma_t = gam[t] + i gam[t + l]; lane t writes history position t
    const int t = tid;
    const zd beta(a.beta, beta_im), omega(a.omega, omega_im);
    const zd gcur = t < l ? zd(gam[t], gam[t + l]) : zd();
    const zd gprev = t >= 1 && t <= l ? zd(gam[t - 1], gam[t - 1 + l]) : zd();
    const int pos0 = ((a.p - l) % a.p + a.p) % a.p;
    const int slot0 = (int)((k - l) % a.nslots);
    const int cyc0 = a.q > 0 ? (int)(cycle0 % a.q) : 0;
    const bool anderson = t < l && a.q > 0 && (pos0 + t) % a.p == 0;
    // x_{k+1} = x_k + beta f_k - sum_i gamma_i (dX_i + beta dF_i)
    zd al = (t == l ? beta : zd()) - beta * (gprev - gcur);
    if (t < l && !anderson)
        al = al - omega * gcur;
    const unsigned long long amask = __ballot(anderson);
    if (anderson) {
        const int nd = __popcll(amask & ((1ull << t) - 1ull));
        const int c = cyc0 - 1 + (a.p - l + t) / a.p;
        st->dslot[nd] = ((c % a.q) + a.q) % a.q;
        st->delta[nd] = -gcur.re;
        st->delta_im[nd] = -gcur.im;
    }
    if (t <= l) {
        st->alpha[t] = al.re;
        st->alpha_im[t] = al.im;
        st->fslot[t] = (slot0 + t) % a.nslots;
    }
    if (tid == 0) {
        int kept = 2 * l;
        if (!fast) {
            kept = 0;
            for (int e = 0; e < 2 * l; ++e)
                kept += S[e][e] > sh_off;
        }
        st->rank = kept / 2;
        if (a.rank_log && log_count0 < a.log_cap)
            a.rank_log[log_count0] = kept / 2;
        st->nf = l + 1;
        st->nd = __popcll(amask);
        st->wslot = a.q > 0 ? cyc0 : -1;
        st->cycle = cycle0 + 1;
    }
}

hipError_t launch_clsq(const LsqArgs &a, double omega_im, double beta_im, hipStream_t s)
{
    hipLaunchKernelGGL(k_clsq, dim3(1), dim3(kLsqThreads), 0, s, a, omega_im, beta_im);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Update
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_cupdate(const UpdateArgs<zd> a)
{
    __shared__ const zd *fs[kMaxSlots];
    __shared__ zd al[kMaxSlots];
    __shared__ const zd *ds[kMaxM];
    __shared__ zd de[kMaxM];
    __shared__ int nf_s, nd_s, ws_s;
    const InstState *st = a.state;
    const int status = st->status;
    if (a.status_out && blockIdx.x == 0 && threadIdx.x == 0)
        *a.status_out = status;
    if (status != kRunning)
        return;
    if (threadIdx.x == 0) {
        nf_s = st->nf;
        nd_s = st->nd;
        ws_s = st->wslot;
    }
    const zd *ring = reinterpret_cast<const zd *>(a.fring);
    if (threadIdx.x < kMaxSlots && (int)threadIdx.x < st->nf) {
        fs[threadIdx.x] = ring + (int64_t)st->fslot[threadIdx.x] * a.slot_stride;
        al[threadIdx.x] = zd(st->alpha[threadIdx.x], st->alpha_im[threadIdx.x]);
    }
    if (threadIdx.x < kMaxM && (int)threadIdx.x < st->nd) {
        ds[threadIdx.x] = reinterpret_cast<const zd *>(a.dxring) + (int64_t)st->dslot[threadIdx.x] * a.dx_stride;
        de[threadIdx.x] = zd(st->delta[threadIdx.x], st->delta_im[threadIdx.x]);
    }
    __syncthreads();
    const int nf = nf_s, nd = nd_s;
    zd *dxw = ws_s >= 0 ? reinterpret_cast<zd *>(a.dxring) + (int64_t)ws_s * a.dx_stride : nullptr;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.N; i += stride) {
        zd d = zd();
        for (int t = 0; t < nf; ++t)
            d += al[t] * fs[t][i];
        for (int t = 0; t < nd; ++t)
            d += de[t] * ds[t][i];
        const zd xk = a.xin[i];
        const zd xn = xk + d;
        a.xout[i] = xn;
        if (dxw)
            dxw[i] = xn - xk;
    }
}

hipError_t launch_cupdate(const UpdateArgs<zd> &a, int blocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_cupdate, dim3(blocks), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// ||b|| of a complex vector (per-workgroup partials of |b_i|^2)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_cnorm_partial(const zd *v, int64_t N, double *partial)
{
    __shared__ double red[kThreads / 64];
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride)
        acc += sqnorm(v[i]);
    acc = wave_sum_a(acc);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0)
        partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

hipError_t launch_cnorm_partial(const zd *v, int64_t N, double *partial, int blocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_cnorm_partial, dim3(blocks), dim3(kThreads), 0, s, v, N, partial);
    return hipGetLastError();
}

}  // namespace aar
