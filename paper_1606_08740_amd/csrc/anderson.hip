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
//   k_lsq     one wave: finishes the residual norm, tests convergence on
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

namespace aar {

template <typename T> __device__ inline T wave_sum_a(T v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v += __shfl_down(v, off, 64);
    return v;
}

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
int gram_blocks(int64_t N)
{
    int64_t b = (N + kThreads * 8 - 1) / (kThreads * 8);
    if (b < 1)
        b = 1;
    if (b > 1024)
        b = 1024;
    return (int)b;
}

// ---------------------------------------------------------------------------
// Gram products
// ---------------------------------------------------------------------------
// V consecutive elements moved by one 16-byte (8-byte for bf16) access.
template <typename E, int V> struct alignas(sizeof(E) * V) Pack {
    E v[V];
};

template <typename H> struct VecWidth {
    static constexpr int value = 16 / (int)sizeof(H) > 8 ? 8 : 16 / (int)sizeof(H);
};
template <> struct VecWidth<bf16_t> {
    static constexpr int value = 4;
};

template <typename H, int V>
__device__ inline void load_vec(const H *p, int64_t i, double *out)
{
    const Pack<H, V> pk = *reinterpret_cast<const Pack<H, V> *>(p + i);
#pragma unroll
    for (int u = 0; u < V; ++u)
        out[u] = (double)Hist<H>::load(pk.v, u);
}

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
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nvec; v += stride) {
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
#pragma unroll
    for (int e = 0; e < NE; ++e) {
        const double v = wave_sum_a(acc[e]);
        if (lane == 0)
            red[wave][e] = v;
    }
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

constexpr int kLsqThreads = 64;   // one wave: barriers are cheap

__global__ __launch_bounds__(kLsqThreads) void k_lsq(const LsqArgs a)
{
    __shared__ double S[kMaxM][kMaxM + 1];
    __shared__ double V[kMaxM][kMaxM + 1];
    __shared__ double cvec[kMaxM];
    __shared__ double wvec[kMaxM];
    __shared__ double gam[kMaxM];
    __shared__ double rot_c[kMaxM / 2], rot_s[kMaxM / 2];
    __shared__ int pair_p[kMaxM / 2], pair_q[kMaxM / 2];
    __shared__ double Li[kMaxM][kMaxM + 1];
    __shared__ double sh_off;
    __shared__ int sh_stop;
    __shared__ int sh_fail;

    InstState *st = a.state;
    if (st->status != kRunning)
        return;
    const int tid = threadIdx.x;
    const int64_t k = st->cycle * a.p + a.p - 1;
    if (k >= st->max_iter) {
        if (tid == 0) {
            st->iters = st->max_iter;
            st->status = kMaxIter;
        }
        return;
    }
    const int l = (int)(k < a.m ? k : a.m);
    const int np = a.m * (a.m + 1) / 2;

    // residual norm: thread-strided partials, fixed-order wave sum, broadcast
    double r = 0.0;
    for (int i = tid; i < a.rho_blocks; i += kLsqThreads)
        r += a.rho_partial[i];
    r = wave_sum_a(r);
    const double rho2 = __shfl(r, 0, 64);
    // G (upper triangle, row-major over the m x m layout) and c
    for (int e = tid; e < a.ne; e += kLsqThreads) {
        const double v = a.gram_final[e];
        if (e < np) {
            int row = 0, rem = e;
            while (rem >= a.m - row) {
                rem -= a.m - row;
                ++row;
            }
            const int col = row + rem;
            if (row < l && col < l) {
                S[row][col] = v;
                S[col][row] = v;
            }
        } else if (e - np < l) {
            cvec[e - np] = v;
        }
    }
    __syncthreads();

    const double rel = sqrt(rho2) / st->nb;
    if (tid == 0) {
        st->last_r = rel;
        if (a.log && st->log_count < a.log_cap)
            a.log[st->log_count] = rel;
        st->log_count += 1;
    }
    bool bad = !isfinite(rel);
    for (int i = 0; i < l && !bad; ++i) {
        bad = !isfinite(cvec[i]);
        for (int j = 0; j < l && !bad; ++j)
            bad = !isfinite(S[i][j]);
    }
    if (bad || rel < st->tol) {
        if (tid == 0) {
            st->iters = k + 1;
            st->status = bad ? kBreakdown : kConverged;
        }
        return;
    }
    if (a.stagnation_window > 0) {
        // inner solves of the refinement stop when the best residual has not
        // fallen by the given factor over the last `window` Anderson steps
        if (tid == 0) {
            if (rel < a.stagnation_factor * st->best_r) {
                st->best_r = rel;
                st->since_best = 0;
            } else {
                st->since_best += 1;
            }
            sh_stop = st->since_best >= a.stagnation_window;
        }
        __syncthreads();
        if (sh_stop) {
            if (tid == 0) {
                st->iters = k + 1;
                st->status = kStagnated;
            }
            return;
        }
    }

    // ---- fast path: Cholesky S = L L^T ----
    // When every eigenvalue of S provably exceeds the pseudoinverse threshold
    // rcond * l * lambda_max, the pseudoinverse is the inverse and
    // gamma = L^-T L^-1 c.  The proof: lambda_min >= 1 / ||L^-1||_F^2 and
    // lambda_max <= trace(S).  Otherwise the eigendecomposition below runs.
    int fast = 0;
    if (l > 0) {
        for (int i = tid; i < l * l; i += kLsqThreads)
            V[i / l][i % l] = S[i / l][i % l];
        if (tid == 0)
            sh_fail = 0;
        __syncthreads();
        for (int j = 0; j < l; ++j) {
            if (tid == 0) {
                const double piv = V[j][j];
                if (!(piv > 0.0))
                    sh_fail = 1;
                else
                    V[j][j] = sqrt(piv);
            }
            __syncthreads();
            if (sh_fail)
                break;
            for (int i = j + 1 + tid; i < l; i += kLsqThreads)
                V[i][j] /= V[j][j];
            __syncthreads();
            const int w = l - j - 1;   // trailing block (j+1 .. l-1)^2, lower part
            for (int idx = tid; idx < w * w; idx += kLsqThreads) {
                const int i = j + 1 + idx / w, kk = j + 1 + idx % w;
                if (kk <= i)
                    V[i][kk] -= V[i][j] * V[kk][j];
            }
            __syncthreads();
        }
        if (!sh_fail) {
            // columns of L^-1, one lane per column
            for (int c = tid; c < l; c += kLsqThreads) {
                for (int i = 0; i < c; ++i)
                    Li[i][c] = 0.0;
                for (int i = c; i < l; ++i) {
                    double acc = i == c ? 1.0 : 0.0;
                    for (int kk = c; kk < i; ++kk)
                        acc -= V[i][kk] * Li[kk][c];
                    Li[i][c] = acc / V[i][i];
                }
            }
            __syncthreads();
            double fro = 0.0, tr = 0.0;
            for (int i = tid; i < l * l; i += kLsqThreads)
                fro += Li[i / l][i % l] * Li[i / l][i % l];
            for (int i = tid; i < l; i += kLsqThreads)
                tr += S[i][i];
            fro = __shfl(wave_sum_a(fro), 0, 64);
            tr = __shfl(wave_sum_a(tr), 0, 64);
            fast = (1.0 / fro > a.rcond * (double)l * tr) && fro == fro;
            if (fast) {
                for (int i = tid; i < l; i += kLsqThreads) {   // y = L^-1 c
                    double y = 0.0;
                    for (int kk = 0; kk <= i; ++kk)
                        y += Li[i][kk] * cvec[kk];
                    wvec[i] = y;
                }
                __syncthreads();
                for (int i = tid; i < l; i += kLsqThreads) {   // gamma = L^-T y
                    double g = 0.0;
                    for (int kk = i; kk < l; ++kk)
                        g += Li[kk][i] * wvec[kk];
                    gam[i] = g;
                }
                __syncthreads();
            }
        }
    }

    if (!fast) {
    // ---- gamma = pinv(S) c by parallel cyclic Jacobi (round-robin pairs) ----
    const int L = l + (l & 1);   // even order; index l is a dummy when l is odd
    for (int i = tid; i < kMaxM * kMaxM; i += kLsqThreads) {
        const int row = i / kMaxM, col = i % kMaxM;
        if (row < L && col < L) {
            V[row][col] = row == col ? 1.0 : 0.0;
            if (row >= l || col >= l)
                S[row][col] = 0.0;
        }
    }
    __syncthreads();
    const int half = L / 2;
    const int M1 = L - 1;
    // Sweeps stop when one applies no rotation: a pair is rotated only while
    // |s_pq| > 1e-15 sqrt(|s_pp s_qq|) (negligible against both diagonals).
    for (int sweep = 0; sweep < 40 && L >= 2; ++sweep) {
        if (tid == 0)
            sh_stop = 1;
        __syncthreads();
        for (int round = 0; round < M1; ++round) {
            if (tid < half) {
                // circle method: index L-1 meets `round`; the others pair
                // (round + i) mod (L-1) with (round - i) mod (L-1)
                int p, qq;
                if (tid == 0) {
                    p = round;
                    qq = L - 1;
                } else {
                    p = (round + tid) % M1;
                    qq = (round - tid + M1) % M1;
                }
                if (p > qq) {
                    const int t = p;
                    p = qq;
                    qq = t;
                }
                double c = 1.0, sn = 0.0;
                if (qq < l) {
                    const double apq = S[p][qq];
                    const double app = S[p][p], aqq = S[qq][qq];
                    if (fabs(apq) > 1e-15 * sqrt(fabs(app * aqq)) && fabs(apq) > 1e-300) {
                        const double theta = (aqq - app) / (2.0 * apq);
                        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                        c = 1.0 / sqrt(t * t + 1.0);
                        sn = t * c;
                        sh_stop = 0;
                    }
                }
                pair_p[tid] = p;
                pair_q[tid] = qq;
                rot_c[tid] = c;
                rot_s[tid] = sn;
            }
            __syncthreads();
            // rows: S <- J^T S
            for (int it = tid; it < half * L; it += kLsqThreads) {
                const int pi = it / L, col = it % L;
                const int p = pair_p[pi], qq = pair_q[pi];
                const double c = rot_c[pi], sn = rot_s[pi];
                const double sp = S[p][col], sq = S[qq][col];
                S[p][col] = c * sp - sn * sq;
                S[qq][col] = sn * sp + c * sq;
            }
            __syncthreads();
            // columns: S <- S J, V <- V J
            for (int it = tid; it < half * L; it += kLsqThreads) {
                const int pi = it / L, row = it % L;
                const int p = pair_p[pi], qq = pair_q[pi];
                const double c = rot_c[pi], sn = rot_s[pi];
                const double sp = S[row][p], sq = S[row][qq];
                S[row][p] = c * sp - sn * sq;
                S[row][qq] = sn * sp + c * sq;
                const double vp = V[row][p], vq = V[row][qq];
                V[row][p] = c * vp - sn * vq;
                V[row][qq] = sn * vp + c * vq;
            }
            __syncthreads();
            // the annihilated pairs are zero in exact arithmetic
            if (tid < half) {
                const int p = pair_p[tid], qq = pair_q[tid];
                if (qq < l && rot_s[tid] != 0.0) {
                    S[p][qq] = 0.0;
                    S[qq][p] = 0.0;
                }
            }
            __syncthreads();
        }
        if (sh_stop)
            break;
    }
    // eigenvalues on the diagonal; drop those <= rcond * l * lambda_max
    if (tid == 0) {
        double lmax = 0.0;
        for (int i = 0; i < l; ++i)
            lmax = fmax(lmax, S[i][i]);
        sh_off = a.rcond * (double)l * lmax;
    }
    __syncthreads();
    const double thresh = sh_off;
    for (int e = tid; e < l; e += kLsqThreads) {
        const double lam = S[e][e];
        double proj = 0.0;
        for (int i = 0; i < l; ++i)
            proj += V[i][e] * cvec[i];
        wvec[e] = lam > thresh ? proj / lam : 0.0;
    }
    __syncthreads();
    for (int i = tid; i < l; i += kLsqThreads) {
        double g = 0.0;
        for (int e = 0; e < l; ++e)
            g += V[i][e] * wvec[e];
        gam[i] = g;
    }
    __syncthreads();
    }   // !fast

    // ---- update plan ----
    // x_{k+1} = x_k + beta f_k - sum_i gamma_i (dX_i + beta dF_i), column i
    // covering iteration j_i = k - l + i:  dF_i = f_{j_i+1} - f_{j_i},
    // dX_i = omega f_{j_i} (Richardson j_i) or the stored increment (Anderson j_i).
    if (tid == 0) {
        int rank = l;
        if (!fast) {
            rank = 0;
            for (int e = 0; e < l; ++e)
                rank += S[e][e] > sh_off;
        }
        st->rank = rank;
        int nd = 0;
        for (int t = 0; t <= l; ++t) {
            const double gprev = t >= 1 ? gam[t - 1] : 0.0;
            const double gcur = t < l ? gam[t] : 0.0;
            double al = (t == l ? a.beta : 0.0) - a.beta * (gprev - gcur);
            if (t < l) {
                const int64_t j = k - l + t;
                const bool anderson = ((j + 1) % a.p) == 0;
                if (anderson && a.q > 0) {
                    const int64_t cyc = (j + 1) / a.p - 1;
                    st->dslot[nd] = (int)(cyc % a.q);
                    st->delta[nd] = -gcur;
                    ++nd;
                } else {
                    al -= a.omega * gcur;
                }
            }
            st->alpha[t] = al;
            st->fslot[t] = (int)((k - l + t) % a.nslots);
        }
        st->nf = l + 1;
        st->nd = nd;
        st->wslot = a.q > 0 ? (int)(st->cycle % a.q) : -1;
        st->cycle = st->cycle + 1;
    }
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
    __shared__ const H *fs[kMaxSlots];
    __shared__ T al[kMaxSlots];
    __shared__ const T *ds[kMaxM];
    __shared__ T de[kMaxM];
    __shared__ int nf_s, nd_s, ws_s;
    const InstState *st = a.state;
    if (st->status != kRunning)
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
        ds[threadIdx.x] = a.dxring + (int64_t)st->dslot[threadIdx.x] * a.dx_stride;
        de[threadIdx.x] = (T)st->delta[threadIdx.x];
    }
    __syncthreads();
    const int nf = nf_s, nd = nd_s;
    T *dxw = ws_s >= 0 ? a.dxring + (int64_t)ws_s * a.dx_stride : nullptr;
    const T *fk_ptr = a.fcur;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t nvec = a.N / V;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nvec; v += stride) {
        const int64_t i = v * V;
        T d[V];
#pragma unroll
        for (int u = 0; u < V; ++u)
            d[u] = T(0);
        for (int t = 0; t < nf - 1; ++t) {
            const Pack<H, V> h = *reinterpret_cast<const Pack<H, V> *>(fs[t] + i);
#pragma unroll
            for (int u = 0; u < V; ++u)
                d[u] += al[t] * (T)Hist<H>::load(h.v, u);
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
            const Pack<T, V> h = *reinterpret_cast<const Pack<T, V> *>(ds[t] + i);
#pragma unroll
            for (int u = 0; u < V; ++u)
                d[u] += de[t] * h.v[u];
        }
        const Pack<T, V> xk = *reinterpret_cast<const Pack<T, V> *>(a.xin + i);
        Pack<T, V> xn, dx;
#pragma unroll
        for (int u = 0; u < V; ++u) {
            xn.v[u] = xk.v[u] + d[u];
            dx.v[u] = xn.v[u] - xk.v[u];     // the increment actually taken
        }
        *reinterpret_cast<Pack<T, V> *>(a.xout + i) = xn;
        if (dxw)
            *reinterpret_cast<Pack<T, V> *>(dxw + i) = dx;
    }
    for (int64_t i = nvec * V + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.N; i += stride) {
        T d = 0;
        for (int t = 0; t < nf - 1; ++t)
            d += al[t] * (T)Hist<H>::load(fs[t], i);
        const T fk = fk_ptr ? fk_ptr[i] : (T)Hist<H>::load(fs[nf - 1], i);
        d += al[nf - 1] * fk;
        for (int t = 0; t < nd; ++t)
            d += de[t] * ds[t][i];
        const T xk = a.xin[i];
        const T xn = xk + d;
        a.xout[i] = xn;
        if (dxw)
            dxw[i] = xn - xk;
    }
}

hipError_t launch_update(Prec prec, const UpdateArgs<double> *a64, const UpdateArgs<float> *a32, int blocks,
                         hipStream_t s)
{
    switch (prec) {
    case Prec::F64:
        hipLaunchKernelGGL((k_update<double, double>), dim3(blocks), dim3(kThreads), 0, s, *a64);
        break;
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
    }
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

}  // namespace aar
